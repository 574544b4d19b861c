// list.hip -- k-clique listing (filled in below).
#include "internal.h"

int search_list(const dist_graph* g, int k, const dist_config& cfg, dist_sink sink, void* user, hipStream_t s,
                dist_result* out) {
  (void)g; (void)k; (void)cfg; (void)sink; (void)user; (void)s; (void)out;
  return DIST_E_UNSUPPORTED;
}
