// orient.hip -- input validation and orientation of the graph into a DAG
// (Section II-A: the DAG of G under a total order keeps arc (u, v) iff
// {u, v} is an edge and u precedes v; Algorithm 2 starts by computing it).
//
// Two total orders:
//   degree      -- (degree, id) ascending;
//   degeneracy  -- bulk minimum-degree peeling (Section II-A defines the
//                  degeneracy order by removing a minimum-degree vertex
//                  repeatedly; removing every vertex whose current degree is
//                  at most the current level in one round keeps the property
//                  that matters here: each vertex has at most delta(G)
//                  out-neighbours).  Order = (round, id) ascending.
//
// Output (all in rank space, int32): orig[r], rank[v], DAG out-lists
// dptr/dcol sorted ascending, fingerprint weights gw[r] = g(orig[r]), and the
// roots sorted by out-degree descending for the search.
#include "internal.h"

#include <algorithm>
#include <chrono>

namespace {

constexpr int kWave = 64;

// ---- fingerprint weight g(v) -------------------------------------------
// One SplitMix64 step (Steele, Lea, Flood 2014) from state 0x44495354 ^ v,
// reduced to [1, 2^61 - 2].
__device__ __forceinline__ u64 fp_weight(u64 v) {
  u64 z = (0x44495354ull ^ v) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 1 + z % (DIST_P61 - 1);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ u64 lanemask_lt() {
  int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// ---- validation -------------------------------------------------------------

// row_ptr must start at 0, end at nnz and never decrease.
__global__ void k_validate_ptr(const int32_t* rp, int32_t n, int64_t nnz, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i <= n; i += stride) {
    int32_t a = rp[i];
    if (a < 0 || (int64_t)a > nnz) atomicOr(bad, 1);
    if (i == 0 && a != 0) atomicOr(bad, 1);
    if (i == n && (int64_t)a != nnz) atomicOr(bad, 1);
    if (i < n && rp[i + 1] < a) atomicOr(bad, 1);
  }
}

// Rows strictly increasing, ids in range, no self-loops, symmetric.  Runs
// only after k_validate_ptr found row_ptr well formed.
__global__ void k_validate_col(const int32_t* rp, const int32_t* col, int32_t n, int* bad) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int lane = lane_id();
  for (int64_t v = wave; v < n; v += nw) {
    int32_t b = rp[v], e = rp[v + 1];
    for (int32_t i = b + lane; i < e; i += kWave) {
      int32_t x = col[i];
      if (x < 0 || x >= n || x == (int32_t)v) { atomicOr(bad, 1); continue; }
      if (i > b && col[i - 1] >= x) atomicOr(bad, 1);
      int32_t lo = rp[x], hi = rp[x + 1];
      while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < (int32_t)v) lo = mid + 1; else hi = mid;
      }
      if (lo >= rp[x + 1] || col[lo] != (int32_t)v) atomicOr(bad, 1);
    }
  }
}

// ---- stable LSD radix sort of (u32 key, i32 value) pairs ------------------

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* keys, int32_t n, int shift,
                                                        uint32_t* counts, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) {
    int64_t idx = base + i;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `total` counters in place (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_scan_small_u32(uint32_t* c, int64_t total) {
  __shared__ uint32_t part[1024];
  int64_t per = (total + 1023) / 1024;
  int64_t beg = threadIdx.x * per;
  int64_t end = beg + per < total ? beg + per : total;
  uint32_t s = 0;
  for (int64_t i = beg; i < end; ++i) s += c[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int64_t i = beg; i < end; ++i) {
    uint32_t x = c[i];
    c[i] = run;
    run += x;
  }
}

// Stable scatter: within a tile items keep their input order; a digit's
// slot is (global offset of digit in this tile) + (earlier items of the
// same digit in this tile).  Lanes with equal digits are matched with one
// ballot per digit bit.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* kin, const int32_t* vin,
                                                           uint32_t* kout, int32_t* vout, int32_t n,
                                                           int shift, const uint32_t* offs,
                                                           int nblocks) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[4][256];
  int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wc[w][tid] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int s = 0; s < kRsItems; ++s) {
    int64_t idx = base + (int64_t)s * kRsThreads + tid;
    bool valid = idx < n;
    uint32_t key = valid ? kin[idx] : 0u;
    uint32_t dig = (key >> shift) & 255u;
    u64 match = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      u64 bb = __ballot(valid && ((dig >> b) & 1u));
      match &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    u64 lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int rw = __popcll(match & lt);
    if (valid && rw == 0) wc[wid][dig] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rw;
      for (int w = 0; w < wid; ++w) pos += wc[w][dig];
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
    for (int w = 0; w < 4; ++w) wc[w][tid] = 0;
    __syncthreads();
  }
}

__global__ void k_iota(int32_t* v, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) v[i] = (int32_t)i;
}

__global__ void k_max_u32(const uint32_t* a, int32_t n, uint32_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t m = 0;
  for (; i < n; i += stride) m = a[i] > m ? a[i] : m;
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(m, off);
    m = o > m ? o : m;
  }
  if (lane_id() == 0) atomicMax(out, m);
}

int grid_for(int64_t items, int threads, int cap = 65536) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Sorts (keys, vals) by key, stably, using `bits` low key bits.  tmp
// buffers must hold n items; counts must hold 256 * ceil(n / tile).
int radix_sort(uint32_t* keys, int32_t* vals, uint32_t* ktmp, int32_t* vtmp,
               uint32_t* counts, int32_t n, int bits, hipStream_t s) {
  if (n <= 1) return DIST_OK;
  int nblocks = (int)((n + kRsTile - 1) / kRsTile);
  uint32_t* ki = keys; int32_t* vi = vals;
  uint32_t* ko = ktmp; int32_t* vo = vtmp;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kRsThreads), 0, s, ki, n, shift, counts, nblocks);
    hipLaunchKernelGGL(k_scan_small_u32, dim3(1), dim3(1024), 0, s, counts, (int64_t)256 * nblocks);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, s, ki, vi, ko, vo, n, shift,
                       counts, nblocks);
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (passes & 1) {
    DIST_CHECK(hipMemcpyAsync(keys, ki, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    DIST_CHECK(hipMemcpyAsync(vals, vi, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  DIST_CHECK(hipGetLastError());
  return DIST_OK;
}

// ---- exclusive scan of int32 (n items -> n + 1 offsets) -------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* in, int32_t n, uint32_t* sums) {
  __shared__ uint32_t red[kScanThreads / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    int64_t idx = base + i;
    if (idx < n) s += (uint32_t)in[idx];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* in, int32_t n, const uint32_t* offs,
                                                             int32_t* out) {
  __shared__ uint32_t part[kScanThreads];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t loc[kScanItems];
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    int64_t idx = base + j;
    loc[j] = idx < n ? (uint32_t)in[idx] : 0u;
    s += loc[j];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = offs[blockIdx.x] + (threadIdx.x ? part[threadIdx.x - 1] : 0u);
  for (int j = 0; j < kScanItems; ++j) {
    int64_t idx = base + j;
    if (idx < n) out[idx] = (int32_t)run;
    if (idx == n - 1) out[n] = (int32_t)(run + loc[j]);
    run += loc[j];
  }
}

int scan_exclusive(const int32_t* in, int32_t* out, int32_t n, uint32_t* sums, hipStream_t s) {
  if (n == 0) return hipMemsetAsync(out, 0, sizeof(int32_t), s) == hipSuccess ? DIST_OK : DIST_E_DEVICE;
  int nb = (int)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_small_u32, dim3(1), dim3(1024), 0, s, sums, (int64_t)nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, in, n, sums, out);
  DIST_CHECK(hipGetLastError());
  return DIST_OK;
}

// ---- order keys -------------------------------------------------------------

__global__ void k_degree_keys(const int32_t* rp, int32_t n, uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) key[i] = (uint32_t)(rp[i + 1] - rp[i]);
}

// Bulk peeling.  round_of[v] < 0 while v is alive.
__global__ void k_peel_init(const int32_t* rp, int32_t n, int32_t* degc, int32_t* round_of) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    degc[i] = rp[i + 1] - rp[i];
    round_of[i] = -1;
  }
}

// Append every alive vertex of current degree <= level to the frontier
// (one atomic per wave).
__global__ void k_peel_seed(const int32_t* degc, const int32_t* round_of, int32_t n, int32_t level,
                            int32_t* frontier, int32_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t end = ((int64_t)n + kWave - 1) / kWave * kWave;
  for (; i < end; i += stride) {
    bool take = i < n && round_of[i] < 0 && degc[i] <= level;
    u64 b = __ballot(take);
    int base = 0;
    if (lane_id() == 0 && b) base = atomicAdd(cnt, __popcll(b));
    base = __shfl(base, 0);
    if (take) frontier[base + __popcll(b & lanemask_lt())] = (int32_t)i;
  }
}

__global__ void k_peel_min(const int32_t* degc, const int32_t* round_of, int32_t n, int32_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t m = 0x7fffffff;
  for (; i < n; i += stride)
    if (round_of[i] < 0 && degc[i] < m) m = degc[i];
  for (int off = 32; off > 0; off >>= 1) {
    int32_t o = __shfl_xor(m, off);
    m = o < m ? o : m;
  }
  if (lane_id() == 0) atomicMin(out, m);
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

__global__ void k_peel_mark(const int32_t* frontier, const int32_t* cnt, int32_t* round_of, int32_t round) {
  int32_t c = *cnt;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < c; i += stride) round_of[frontier[i]] = round;
}

// Remove the frontier: decrement every alive neighbour; a neighbour whose
// degree falls from level + 1 to level joins the next frontier.
__global__ void k_peel_step(const int32_t* rp, const int32_t* col, const int32_t* frontier,
                            const int32_t* cnt, int32_t* degc, const int32_t* round_of, int32_t level,
                            int32_t* next, int32_t* ncnt) {
  int32_t c = *cnt;
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int lane = lane_id();
  for (int64_t f = wave; f < c; f += nw) {
    int32_t v = frontier[f];
    int32_t b = rp[v], e = rp[v + 1];
    for (int32_t i0 = b; i0 < e; i0 += kWave) {
      int32_t i = i0 + lane;
      bool join = false;
      int32_t x = -1;
      if (i < e) {
        x = col[i];
        if (round_of[x] < 0) {
          int32_t old = atomicSub(&degc[x], 1);
          join = (old == level + 1);
        }
      }
      u64 bj = __ballot(join);
      int base = 0;
      if (lane == 0 && bj) base = atomicAdd(ncnt, __popcll(bj));
      base = __shfl(base, 0);
      if (join) next[base + __popcll(bj & lanemask_lt())] = x;
    }
  }
}

__global__ void k_round_keys(const int32_t* round_of, int32_t n, uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) key[i] = (uint32_t)round_of[i];
}

// ---- DAG build --------------------------------------------------------------

__global__ void k_rank_of(const int32_t* orig, int32_t n, int32_t* rank) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) rank[orig[i]] = (int32_t)i;
}

// outdeg[rank[v]] = number of neighbours of higher rank.
__global__ void k_outdeg(const int32_t* rp, const int32_t* col, const int32_t* rank, int32_t n,
                         int32_t* outdeg) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int lane = lane_id();
  for (int64_t v = wave; v < n; v += nw) {
    int32_t r = rank[v];
    int32_t b = rp[v], e = rp[v + 1];
    int32_t c = 0;
    for (int32_t i0 = b; i0 < e; i0 += kWave) {
      int32_t i = i0 + lane;
      bool up = i < e && rank[col[i]] > r;
      c += __popcll(__ballot(up));
    }
    if (lane == 0) outdeg[r] = c;
  }
}

// Unsorted out-lists (ranks) into tmp at the final row offsets.
__global__ void k_fill_unsorted(const int32_t* rp, const int32_t* col, const int32_t* rank, int32_t n,
                                const int32_t* dptr, int32_t* tmp) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int lane = lane_id();
  for (int64_t v = wave; v < n; v += nw) {
    int32_t r = rank[v];
    int32_t b = rp[v], e = rp[v + 1];
    int32_t out = dptr[r];
    for (int32_t i0 = b; i0 < e; i0 += kWave) {
      int32_t i = i0 + lane;
      int32_t x = i < e ? rank[col[i]] : -1;
      bool up = i < e && x > r;
      u64 bu = __ballot(up);
      if (up) tmp[out + __popcll(bu & lanemask_lt())] = x;
      out += __popcll(bu);
    }
  }
}

// Sort each row: the slot of an element is the number of smaller elements
// in its row (elements of a row are distinct).  Rows up to kSortLds items
// are staged in LDS.
constexpr int kSortLds = 4096;
__global__ __launch_bounds__(64) void k_sort_rows(const int32_t* dptr, const int32_t* tmp, int32_t n,
                                                  int32_t* dcol) {
  __shared__ int32_t row[kSortLds];
  int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    int32_t b = dptr[r], e = dptr[r + 1], d = e - b;
    if (d == 0) continue;
    const int32_t* src = tmp + b;
    if (d <= kSortLds) {
      for (int32_t i = lane; i < d; i += kWave) row[i] = tmp[b + i];
      __syncthreads();
      src = row;
    }
    for (int32_t i = lane; i < d; i += kWave) {
      int32_t x = src[i];
      int32_t pos = 0;
      for (int32_t j = 0; j < d; ++j) pos += src[j] < x;
      dcol[b + pos] = x;
    }
    __syncthreads();
  }
}

__global__ void k_weights(const int32_t* orig, int32_t n, u64* gw) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) gw[i] = fp_weight((u64)(uint32_t)orig[i]);
}

__global__ void k_root_keys(const int32_t* outdeg, int32_t n, int32_t maxd, uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) key[i] = (uint32_t)(maxd - outdeg[i]);
}

int bits_for(uint32_t maxkey) {
  int b = 0;
  while (b < 32 && (maxkey >> b)) ++b;
  return b;
}

// Freed blocks are reused at once, so scratch is released only after the
// stream's work (also on an error path) has finished.
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  ~Scratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
    for (void* p : ptrs) dev_free(p);
  }
  template <class T>
  int get(T** p, size_t count) {
    void* q = nullptr;
    if (dev_alloc(&q, count * sizeof(T) + 16) != DIST_OK) return DIST_E_NOMEM;
    ptrs.push_back(q);
    *p = (T*)q;
    return DIST_OK;
  }
};

#define TRY(x)                 \
  do {                         \
    int rc_ = (x);             \
    if (rc_ != DIST_OK) return rc_; \
  } while (0)

}  // namespace

int orient_build(const int32_t* rp, const int32_t* col, int32_t n, int64_t nnz, int order_mode,
                 hipStream_t s, dist_graph* g) {
  Scratch sc(s);
  const int T = 256;
  int32_t* hflags = nullptr;  // pinned host words for small readbacks
  if (pinned_alloc((void**)&hflags, 4 * sizeof(int32_t)) != DIST_OK) return DIST_E_NOMEM;
  struct HostFree {
    int32_t* p;
    hipStream_t s;
    ~HostFree() {
      (void)hipStreamSynchronize(s);
      pinned_free(p);
    }
  } hf{hflags, s};
  int32_t* dflag;
  TRY(sc.get(&dflag, 4));

  hipEvent_t e0, e1;
  DIST_CHECK(hipEventCreate(&e0));
  DIST_CHECK(hipEventCreate(&e1));
  struct EvFree {
    hipEvent_t a, b;
    ~EvFree() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ef{e0, e1};
  DIST_CHECK(hipEventRecord(e0, s));

  // 1. validate
  DIST_CHECK(hipMemsetAsync(dflag, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(k_validate_ptr, dim3(grid_for((int64_t)n + 1, T)), dim3(T), 0, s, rp, n, nnz, dflag);
  DIST_CHECK(hipMemcpyAsync(hflags, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  if (hflags[0]) return DIST_E_INVALID;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_validate_col, dim3(grid_for((int64_t)n * kWave, T)), dim3(T), 0, s, rp, col, n, dflag);
    DIST_CHECK(hipMemcpyAsync(hflags, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DIST_CHECK(hipStreamSynchronize(s));
    if (hflags[0]) return DIST_E_INVALID;
  }
  g->n = n;
  g->m = nnz / 2;
  g->order_mode = order_mode;

  int nn = n > 0 ? n : 1;
  uint32_t *key, *ktmp, *counts;
  int32_t *vals, *vtmp;
  uint32_t* dmax;
  TRY(sc.get(&key, nn));
  TRY(sc.get(&ktmp, nn));
  TRY(sc.get(&vals, nn));
  TRY(sc.get(&vtmp, nn));
  TRY(sc.get(&counts, 256 * ((size_t)nn / kRsTile + 2)));
  TRY(sc.get(&dmax, 4));

  TRY(dev_alloc((void**)&g->rank, sizeof(int32_t) * nn));
  TRY(dev_alloc((void**)&g->orig, sizeof(int32_t) * nn));
  TRY(dev_alloc((void**)&g->dptr, sizeof(int32_t) * (nn + 1)));
  TRY(dev_alloc((void**)&g->dcol, sizeof(int32_t) * (g->m > 0 ? g->m : 1)));
  TRY(dev_alloc((void**)&g->gw, sizeof(u64) * nn));
  TRY(dev_alloc((void**)&g->roots, sizeof(int32_t) * nn));

  // 2. order keys
  int gridn = grid_for(n, T);
  if (order_mode == DIST_ORDER_DEGREE) {
    hipLaunchKernelGGL(k_degree_keys, dim3(gridn), dim3(T), 0, s, rp, n, key);
    g->order_bound = 0;
  } else if (order_mode == DIST_ORDER_INPUT) {
    hipLaunchKernelGGL(k_iota, dim3(gridn), dim3(T), 0, s, (int32_t*)key, n);  // key = id
    g->order_bound = 0;
  } else {
    int32_t *degc, *round_of, *fa, *fb, *cnts;
    TRY(sc.get(&degc, nn));
    TRY(sc.get(&round_of, nn));
    TRY(sc.get(&fa, nn));
    TRY(sc.get(&fb, nn));
    TRY(sc.get(&cnts, 4));
    hipLaunchKernelGGL(k_peel_init, dim3(gridn), dim3(T), 0, s, rp, n, degc, round_of);
    int32_t level = 0, round = 0;
    int64_t removed = 0;
    int32_t* cur = fa;
    int32_t* nxt = fb;
    int64_t guard = 2 * (int64_t)n + 16;  // each step removes a vertex or raises the level
    while (removed < n) {
      if (--guard < 0) return DIST_E_DEVICE;
      DIST_CHECK(hipMemsetAsync(cnts, 0, 2 * sizeof(int32_t), s));
      hipLaunchKernelGGL(k_peel_seed, dim3(gridn), dim3(T), 0, s, degc, round_of, n, level, cur, cnts);
      DIST_CHECK(hipMemcpyAsync(hflags, cnts, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      DIST_CHECK(hipStreamSynchronize(s));
      int32_t c = hflags[0];
      if (c == 0) {
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, cnts + 2, (int32_t)0x7fffffff);
        hipLaunchKernelGGL(k_peel_min, dim3(gridn), dim3(T), 0, s, degc, round_of, n, cnts + 2);
        DIST_CHECK(hipMemcpyAsync(hflags + 2, cnts + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DIST_CHECK(hipStreamSynchronize(s));
        if (hflags[2] == 0x7fffffff) break;  // nothing alive
        level = hflags[2];
        continue;
      }
      int32_t* cnt_cur = cnts;      // size of cur
      int32_t* cnt_nxt = cnts + 1;  // size of nxt
      while (c > 0) {
        hipLaunchKernelGGL(k_peel_mark, dim3(grid_for(c, T)), dim3(T), 0, s, cur, cnt_cur, round_of, round);
        DIST_CHECK(hipMemsetAsync(cnt_nxt, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_peel_step, dim3(grid_for((int64_t)c * kWave, T)), dim3(T), 0, s, rp, col, cur,
                           cnt_cur, degc, round_of, level, nxt, cnt_nxt);
        DIST_CHECK(hipMemcpyAsync(hflags, cnt_nxt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DIST_CHECK(hipStreamSynchronize(s));
        removed += c;
        ++round;
        c = hflags[0];
        std::swap(cur, nxt);
        std::swap(cnt_cur, cnt_nxt);
      }
      if (level > g->order_bound) g->order_bound = level;
    }
    hipLaunchKernelGGL(k_round_keys, dim3(gridn), dim3(T), 0, s, round_of, n, key);
  }
  DIST_CHECK(hipGetLastError());

  // 3. stable sort of ids by key -> orig
  DIST_CHECK(hipMemsetAsync(dmax, 0, sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_max_u32, dim3(gridn), dim3(T), 0, s, key, n, dmax);
  DIST_CHECK(hipMemcpyAsync(hflags, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  int bits = bits_for((uint32_t)hflags[0]);
  hipLaunchKernelGGL(k_iota, dim3(gridn), dim3(T), 0, s, g->orig, n);
  TRY(radix_sort(key, g->orig, ktmp, vtmp, counts, n, bits, s));
  hipLaunchKernelGGL(k_rank_of, dim3(gridn), dim3(T), 0, s, g->orig, n, g->rank);

  // 4. DAG in rank space
  int32_t* outdeg;
  uint32_t* sums;
  TRY(sc.get(&outdeg, nn));
  TRY(sc.get(&sums, (size_t)nn / 2048 + 2));
  int gridw = grid_for((int64_t)n * kWave, T);
  hipLaunchKernelGGL(k_outdeg, dim3(gridw), dim3(T), 0, s, rp, col, g->rank, n, outdeg);
  TRY(scan_exclusive(outdeg, g->dptr, n, sums, s));
  if (g->m > 0) {
    int32_t* tmp;
    TRY(sc.get(&tmp, (size_t)g->m));
    hipLaunchKernelGGL(k_fill_unsorted, dim3(gridw), dim3(T), 0, s, rp, col, g->rank, n, g->dptr, tmp);
    hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(n, 1, 65536)), dim3(kWave), 0, s, g->dptr, tmp, n, g->dcol);
  }
  hipLaunchKernelGGL(k_weights, dim3(gridn), dim3(T), 0, s, g->orig, n, g->gw);

  // 5. roots by out-degree descending (ties: rank ascending)
  DIST_CHECK(hipMemsetAsync(dmax, 0, sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_max_u32, dim3(gridn), dim3(T), 0, s, (const uint32_t*)outdeg, n, dmax);
  DIST_CHECK(hipMemcpyAsync(hflags, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  g->max_outdeg = hflags[0];
  if (order_mode != DIST_ORDER_DEGENERACY) g->order_bound = g->max_outdeg;
  hipLaunchKernelGGL(k_root_keys, dim3(gridn), dim3(T), 0, s, outdeg, n, g->max_outdeg, key);
  hipLaunchKernelGGL(k_iota, dim3(gridn), dim3(T), 0, s, g->roots, n);
  TRY(radix_sort(key, g->roots, ktmp, vtmp, counts, n, bits_for((uint32_t)g->max_outdeg), s));
  std::vector<uint32_t> hk(n);
  if (n) DIST_CHECK(hipMemcpyAsync(hk.data(), key, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipEventRecord(e1, s));
  DIST_CHECK(hipStreamSynchronize(s));
  DIST_CHECK(hipGetLastError());
  g->root_deg.resize(n);
  for (int32_t i = 0; i < n; ++i) g->root_deg[i] = g->max_outdeg - (int32_t)hk[i];
  g->deg_hist.clear();
  for (int32_t i = 0; i < n; ++i) {
    if (g->deg_hist.empty() || g->deg_hist.back().first != g->root_deg[i])
      g->deg_hist.push_back({g->root_deg[i], 0});
    g->deg_hist.back().second += 1;
  }
  TRY(dev_alloc((void**)&g->d_root_deg, sizeof(int32_t) * nn));
  if (n) {
    DIST_CHECK(hipMemcpyAsync(g->d_root_deg, g->root_deg.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    DIST_CHECK(hipStreamSynchronize(s));
  }
  float ms = 0;
  DIST_CHECK(hipEventElapsedTime(&ms, e0, e1));
  g->orient_ms = ms;
  return DIST_OK;
}
