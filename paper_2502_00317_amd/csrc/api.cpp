// api.cpp -- the C ABI declared in include/dist.h.
#include <string.h>

#include <new>

#include "internal.h"

namespace {

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void free_graph_arrays(dist_graph* g) {
  dev_free(g->rank);
  dev_free(g->orig);
  dev_free(g->dptr);
  dev_free(g->dcol);
  dev_free(g->gw);
  dev_free(g->roots);
  dev_free(g->d_root_deg);
  g->rank = g->orig = g->dptr = g->dcol = g->roots = g->d_root_deg = nullptr;
  g->gw = nullptr;
}

int valid_k(int k) { return k >= 1 && k <= DIST_K_MAX; }

uint64_t g_graph_serial = 0;

}  // namespace

extern "C" {

void dist_config_init(dist_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->memo = 1;
  cfg->prune = 1;
  cfg->fingerprint = 1;
  cfg->memo_entries = 0;
  cfg->memo_bytes = 0;
  cfg->deadline_ms = 0;
}

const char* dist_strerror(int status) {
  switch (status) {
    case DIST_OK: return "ok";
    case DIST_E_INVALID: return "invalid input graph";
    case DIST_E_K: return "k out of range";
    case DIST_E_NOMEM: return "out of memory";
    case DIST_E_DEVICE: return "HIP runtime error";
    case DIST_E_OVERFLOW: return "count exceeds 64 bits (128-bit result is exact)";
    case DIST_E_CANCELLED: return "cancelled (sink stop or deadline)";
    case DIST_E_UNSUPPORTED: return "root out-degree or k beyond the supported range";
    case DIST_E_SCRATCH: return "the call needs more than the fixed scratch of dist_count_noalloc holds";
    default: return "unknown status";
  }
}

int dist_orient(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz, int order_mode,
                const dist_config* cfg, void* hip_stream, dist_graph** out) {
  if (!out) return DIST_E_INVALID;
  *out = nullptr;
  if (n < 0 || nnz < 0 || nnz >= ((int64_t)1 << 31) || !row_ptr || (nnz > 0 && !col))
    return DIST_E_INVALID;
  if (order_mode != DIST_ORDER_DEGREE && order_mode != DIST_ORDER_DEGENERACY && order_mode != DIST_ORDER_INPUT)
    return DIST_E_INVALID;
  hipStream_t s = (hipStream_t)hip_stream;
  dist_graph* g = new (std::nothrow) dist_graph();
  if (!g) return DIST_E_NOMEM;
  if (cfg) g->cfg = *cfg;
  else dist_config_init(&g->cfg);
  (void)hipGetDevice(&g->device);
  g->serial = ++g_graph_serial;

  const int32_t* d_rp = row_ptr;
  const int32_t* d_col = col;
  int32_t* own_rp = nullptr;
  int32_t* own_col = nullptr;
  int rc = DIST_OK;
  if (!is_device_ptr(row_ptr)) {
    rc = dev_alloc((void**)&own_rp, sizeof(int32_t) * ((size_t)n + 1));
    if (!rc && hipMemcpyAsync(own_rp, row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s) !=
                   hipSuccess)
      rc = DIST_E_DEVICE;
    d_rp = own_rp;
  }
  if (!rc && nnz > 0 && !is_device_ptr(col)) {
    rc = dev_alloc((void**)&own_col, sizeof(int32_t) * (size_t)nnz);
    if (!rc && hipMemcpyAsync(own_col, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s) != hipSuccess)
      rc = DIST_E_DEVICE;
    d_col = own_col;
  }
  if (!rc) rc = orient_build(d_rp, d_col, n, nnz, order_mode, s, g);
  if (own_rp || own_col) (void)hipStreamSynchronize(s);
  dev_free(own_rp);
  dev_free(own_col);
  if (rc) {
    free_graph_arrays(g);
    delete g;
    return rc;
  }
  *out = g;
  return DIST_OK;
}

int dist_count_ex(const dist_graph* g, int k, const dist_config* cfg, uint64_t* per_root, void* hip_stream,
                  dist_result* out) {
  if (!g || !out) return DIST_E_INVALID;
  if (!valid_k(k)) return DIST_E_K;
  SearchLaunch L;
  L.g = g;
  L.k = k;
  L.cfg = cfg ? *cfg : g->cfg;
  L.stream = (hipStream_t)hip_stream;
  L.per_root = nullptr;
  u64* own = nullptr;
  bool host_pr = per_root && !is_device_ptr(per_root);
  if (per_root) {
    if (host_pr) {
      int rc = dev_alloc((void**)&own, sizeof(u64) * 3 * ((size_t)g->n + 1));
      if (rc) return rc;
      L.per_root = own;
    } else {
      L.per_root = (u64*)per_root;
    }
  }
  dist_stats st{};
  int rc = search_count(L, out, &st);
  g->stats = st;
  if (host_pr) {
    if (hipMemcpyAsync(per_root, own, sizeof(u64) * 3 * (size_t)g->n, hipMemcpyDeviceToHost, L.stream) != hipSuccess)
      rc = rc ? rc : DIST_E_DEVICE;
    if (hipStreamSynchronize(L.stream) != hipSuccess) rc = rc ? rc : DIST_E_DEVICE;
    dev_free(own);  // reused at once: only after the stream has finished
  }
  return rc;
}

int dist_count(const dist_graph* g, int k, void* hip_stream, dist_result* out) {
  return dist_count_ex(g, k, nullptr, nullptr, hip_stream, out);
}

int dist_count_noalloc(const dist_graph* g, int k, const dist_config* cfg, void* hip_stream, dist_result* out) {
  if (!g || !out) return DIST_E_INVALID;
  if (!valid_k(k)) return DIST_E_K;
  SearchLaunch L;
  L.g = g;
  L.k = k;
  L.cfg = cfg ? *cfg : g->cfg;
  L.cfg.memo = 0;
  L.stream = (hipStream_t)hip_stream;
  L.per_root = nullptr;
  dist_stats st{};
  int rc = search_count(L, out, &st, true);
  g->stats = st;
  return rc;
}

int dist_count_all(const dist_graph* g, int kmax, const dist_config* cfg, uint64_t* per_root, int per_root_k,
                   void* hip_stream, dist_result* out) {
  if (!g || !out) return DIST_E_INVALID;
  if (kmax < 1 || kmax > DIST_ALL_K_MAX) return DIST_E_K;
  if (per_root && (per_root_k < 2 || per_root_k > kmax)) return DIST_E_K;
  hipStream_t s = (hipStream_t)hip_stream;
  u64* own = nullptr;
  u64* pr = nullptr;
  const bool host_pr = per_root && !is_device_ptr(per_root);
  if (per_root) {
    if (host_pr) {
      if (dev_alloc((void**)&own, sizeof(u64) * 3 * ((size_t)g->n + 1))) return DIST_E_NOMEM;
      pr = own;
    } else {
      pr = (u64*)per_root;
    }
  }
  dist_stats st{};
  int rc = search_count_all(g, kmax, cfg ? *cfg : g->cfg, pr, per_root_k, s, out, &st);
  g->stats = st;
  if (host_pr) {
    if (hipMemcpyAsync(per_root, own, sizeof(u64) * 3 * (size_t)g->n, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = rc ? rc : DIST_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) rc = rc ? rc : DIST_E_DEVICE;
    dev_free(own);
  }
  return rc;
}

int dist_list(const dist_graph* g, int k, dist_sink sink, void* user, void* hip_stream, dist_result* out) {
  if (!g || !out || !sink) return DIST_E_INVALID;
  if (!valid_k(k)) return DIST_E_K;
  dist_stats st{};
  int rc = search_list(g, k, g->cfg, sink, user, 0, (hipStream_t)hip_stream, out, &st);
  g->stats = st;
  return rc;
}

int dist_list_ex(const dist_graph* g, int k, const dist_config* cfg, int flags, dist_sink sink, void* user,
                 void* hip_stream, dist_result* out) {
  if (!g || !out || !sink) return DIST_E_INVALID;
  if (!valid_k(k)) return DIST_E_K;
  dist_stats st{};
  int rc = search_list(g, k, cfg ? *cfg : g->cfg, sink, user, flags, (hipStream_t)hip_stream, out, &st);
  g->stats = st;
  return rc;
}

int dist_ist_inspect(const dist_graph* g, int k, int32_t root, const dist_config* cfg, const uint64_t* ret_set,
                     int ret_l, int32_t cap, int32_t* local_ids, int32_t* d, uint64_t* sets, uint64_t* marked,
                     uint32_t* lc, uint32_t* ls, int32_t* n_nodes, int32_t* rows, int64_t rows_cap,
                     int64_t* n_rows, int64_t* n_ret, void* hip_stream) {
  if (!g || !local_ids || !d || !sets || !marked || !lc || !ls || !n_nodes || !n_rows || !n_ret)
    return DIST_E_INVALID;
  if (!valid_k(k)) return DIST_E_K;
  return search_ist_inspect(g, k, root, cfg ? *cfg : g->cfg, ret_set, ret_l, cap, local_ids, d, sets, marked, lc, ls,
                            n_nodes, rows, rows_cap, n_rows, n_ret, (hipStream_t)hip_stream);
}

int dist_count_batch_ex(const dist_graph* const* gs, const int* ks, int n, const dist_config* cfg, int use_graph,
                        const int64_t* pair_deadline_ms, void* hip_stream, dist_result* out, int* pair_status,
                        double* ms) {
  if (n < 0 || (n > 0 && (!gs || !ks || !out))) return DIST_E_INVALID;
  if (n == 0) return DIST_OK;
  dist_config c;
  if (cfg) c = *cfg;
  else dist_config_init(&c);
  return search_count_batch(gs, ks, n, c, use_graph, pair_deadline_ms, (hipStream_t)hip_stream, out, pair_status,
                            ms);
}

int dist_count_batch_tuned(const dist_graph* const* gs, const int* ks, int n, const dist_config* cfg,
                           const dist_pair_switches* sw, int use_graph, const int64_t* pair_deadline_ms,
                           void* hip_stream, dist_result* out, int* pair_status, double* ms) {
  if (n < 0 || (n > 0 && (!gs || !ks || !out))) return DIST_E_INVALID;
  if (n == 0) return DIST_OK;
  for (int i = 0; sw && i < n; ++i) {
    const dist_pair_switches& w = sw[i];
    if (w.min_width > 16 || w.memo > 2 || w.reserved != 0) return DIST_E_INVALID;
  }
  dist_config c;
  if (cfg) c = *cfg;
  else dist_config_init(&c);
  return search_count_batch(gs, ks, n, c, use_graph, pair_deadline_ms, (hipStream_t)hip_stream, out, pair_status,
                            ms, nullptr, nullptr, nullptr, sw);
}

int dist_count_batch_stream(const dist_graph* const* gs, const int* ks, int n, const dist_config* cfg,
                            const int64_t* pair_deadline_ms, const double* pair_cost, void* hip_stream,
                            dist_result* out, int* pair_status, dist_pair_done on_done, void* user) {
  if (n < 0 || (n > 0 && (!gs || !ks || !out || !on_done))) return DIST_E_INVALID;
  if (n == 0) return DIST_OK;
  dist_config c;
  if (cfg) c = *cfg;
  else dist_config_init(&c);
  return search_count_batch(gs, ks, n, c, 0, pair_deadline_ms, (hipStream_t)hip_stream, out, pair_status, nullptr,
                            on_done, user, pair_cost);
}

int dist_estimate_cost(const dist_graph* g, int k, double* out) {
  if (!g || !out) return DIST_E_INVALID;
  if (k < 1 || k > DIST_K_MAX) return DIST_E_K;
  *out = estimate_cost(g, k);
  return DIST_OK;
}

int dist_count_batch(const dist_graph* const* gs, const int* ks, int n, void* hip_stream, dist_result* out) {
  return dist_count_batch_ex(gs, ks, n, nullptr, 1, nullptr, hip_stream, out, nullptr, nullptr);
}

int dist_root_soft_embed(const dist_graph* g, int cap, int32_t* r_out, void* hip_stream) {
  if (!g || !r_out || cap < 1 || cap > 255) return DIST_E_INVALID;
  hipStream_t s = (hipStream_t)hip_stream;
  int32_t* d = r_out;
  int32_t* own = nullptr;
  bool host = !is_device_ptr(r_out);
  if (host) {
    int rc = dev_alloc((void**)&own, sizeof(int32_t) * ((size_t)g->n + 1));
    if (rc) return rc;
    d = own;
  }
  int rc = search_root_soft_embed(g, cap, d, s);
  if (host) {
    if (!rc && hipMemcpyAsync(r_out, own, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = DIST_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = DIST_E_DEVICE;
    dev_free(own);  // reused at once: only after the stream has finished
  }
  return rc;
}

int dist_graph_ranks(const dist_graph* g, int32_t* r_out, void* hip_stream) {
  if (!g || !r_out) return DIST_E_INVALID;
  hipStream_t s = (hipStream_t)hip_stream;
  if (g->n == 0) return DIST_OK;
  hipMemcpyKind kind = is_device_ptr(r_out) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  DIST_CHECK(hipMemcpyAsync(r_out, g->rank, sizeof(int32_t) * (size_t)g->n, kind, s));
  DIST_CHECK(hipStreamSynchronize(s));
  return DIST_OK;
}

int dist_graph_info_get(const dist_graph* g, dist_graph_info* out) {
  if (!g || !out) return DIST_E_INVALID;
  out->n = g->n;
  out->m = g->m;
  out->order_mode = g->order_mode;
  out->max_outdeg = g->max_outdeg;
  out->order_bound = g->order_bound;
  out->orient_ms = g->orient_ms;
  return DIST_OK;
}

int dist_stats_get(const dist_graph* g, dist_stats* out) {
  if (!g || !out) return DIST_E_INVALID;
  *out = g->stats;
  return DIST_OK;
}

void dist_graph_free(dist_graph* g) {
  if (!g) return;
  batch_forget(g);
  free_graph_arrays(g);
  delete g;
}

}  // extern "C"
