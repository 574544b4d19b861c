// internal.h -- types shared by the host API and the HIP kernels of libdist.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/dist.h"

typedef unsigned long long u64;

// Mersenne prime 2^61 - 1: modulus of the clique fingerprint.
#define DIST_P61 0x1FFFFFFFFFFFFFFFull

// Device-resident oriented graph.
struct dist_graph {
  int32_t n = 0;
  int64_t m = 0;          // undirected edges = DAG arcs
  int order_mode = 0;
  int device = 0;
  dist_config cfg{};
  int32_t* rank = nullptr;   // rank[v]  (input id -> position in the order)
  int32_t* orig = nullptr;   // orig[r]  (position -> input id)
  int32_t* dptr = nullptr;   // DAG out-lists in rank space, n+1
  int32_t* dcol = nullptr;   // m ranks, ascending within a row
  u64* gw = nullptr;         // gw[r] = g(orig[r])
  int32_t* roots = nullptr;  // all ranks sorted by out-degree descending (ties: rank)
  std::vector<int32_t> root_deg;  // host: out-degree of roots[i], non-increasing
  int32_t* d_root_deg = nullptr;  // the same on the device
  std::vector<std::pair<int32_t, int64_t>> deg_hist;  // (out-degree, roots) runs of root_deg
  int32_t max_outdeg = 0;
  int32_t order_bound = 0;
  double orient_ms = 0;
  uint64_t serial = 0;       // unique per oriented graph in this process
  mutable dist_stats stats{};
};

// ---- orientation (orient.hip) ------------------------------------------
int orient_build(const int32_t* d_row_ptr, const int32_t* d_col, int32_t n,
                 int64_t nnz, int order_mode, hipStream_t s, dist_graph* g);

// ---- search (search.hip) -----------------------------------------------
struct SearchLaunch {
  const dist_graph* g;
  int k;
  dist_config cfg;
  u64* per_root;       // device, 3 per input id, or null
  hipStream_t stream;
};
// no_alloc: the form behind dist_count_noalloc (no per-root output, no memo,
// every buffer in the library's static scratch block).
int search_count(const SearchLaunch& L, dist_result* out, dist_stats* st, bool no_alloc = false);
int search_root_soft_embed(const dist_graph* g, int cap, int32_t* d_out,
                           hipStream_t s);

int search_count_batch(const dist_graph* const* gs, const int* ks, int n, const dist_config& cfg, int use_graph,
                       const int64_t* pair_deadline_ms, hipStream_t s, dist_result* out, int* pair_status,
                       double* ms, dist_pair_done on_done = nullptr, void* user = nullptr,
                       const double* pair_cost = nullptr, const dist_pair_switches* sw = nullptr);

// Upper bound on the search size of (g, k): sum over roots of C(d+, k - 1).
double estimate_cost(const dist_graph* g, int k);

void batch_forget(const dist_graph* g);  // drop a cached batch plan that uses g

// ---- every k at once, by pivoting (pivot.hip) ------------------------------
int search_count_all(const dist_graph* g, int kmax, const dist_config& cfg, u64* per_root, int per_root_k,
                     hipStream_t s, dist_result* out, dist_stats* st);

// ---- listing (the Induced Subgraph Trie: ist.hip) -------------------------
int search_list(const dist_graph* g, int k, const dist_config& cfg, dist_sink sink, void* user, int flags,
                hipStream_t s, dist_result* out, dist_stats* st = nullptr);
int search_ist_inspect(const dist_graph* g, int k, int32_t root_id, const dist_config& cfg, const uint64_t* ret_set,
                       int ret_l, int32_t cap, int32_t* local_ids, int32_t* d_out, uint64_t* sets, uint64_t* marked,
                       uint32_t* lc, uint32_t* ls, int32_t* n_nodes, int32_t* rows, int64_t rows_cap,
                       int64_t* n_rows, int64_t* n_ret, hipStream_t s);

// ---- memory: block cache (frees never wait for the device) ---------------
int dev_alloc(void** p, size_t bytes);   // device memory of the current device
void dev_free(void* p);                  // any block from dev_alloc or pinned_alloc
int pinned_alloc(void** p, size_t bytes, unsigned flags = hipHostMallocDefault);
void pinned_free(void* p);
#define DIST_CHECK(call)                         \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return DIST_E_DEVICE;  \
  } while (0)
