// device_common.h -- device code shared by the count and list kernels:
// lane helpers, arithmetic mod 2^61 - 1, the per-wave LDS layout, the
// construction of a root's 1-induced subgraph G_u as bitmap rows, the
// fingerprint weight sums and Algorithm 5 evaluated level by level.
#pragma once

#include "internal.h"

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ u64 lanemask_lt() {
  int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// ---- arithmetic mod p = 2^61 - 1 ------------------------------------------
__device__ __forceinline__ u64 addp(u64 a, u64 b) {
  u64 s = a + b;
  return s >= DIST_P61 ? s - DIST_P61 : s;
}

__device__ __forceinline__ u64 subp(u64 a, u64 b) {
  return a >= b ? a - b : a + (DIST_P61 - b);
}

// a, b < p.  With a = a1 2^32 + a0 and b = b1 2^32 + b0 (a1, b1 < 2^29),
// a b = a1 b1 2^64 + (a0 b1 + a1 b0) 2^32 + a0 b0, and since 2^61 = 1 mod p:
// 2^64 = 8, a middle term m = mh 2^29 + ml gives m 2^32 = mh + ml 2^32, and
// a0 b0 = (its bits from 61 up) + (its low 61 bits).  Four 32 x 32 -> 64
// multiply-adds in place of the six multiplies of a full 64 x 64 -> 128
// product; the sum of the five terms stays below 2^63.
__device__ __forceinline__ u64 mulp(u64 a, u64 b) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const u64 p00 = (u64)a0 * b0;
  const u64 mid = (u64)a0 * b1 + (u64)a1 * b0;
  const u64 p11 = (u64)a1 * b1;
  u64 r = (p11 << 3) + (mid >> 29) + ((mid & ((1ull << 29) - 1)) << 32) + (p00 >> 61) + (p00 & DIST_P61);
  r = (r & DIST_P61) + (r >> 61);
  return r >= DIST_P61 ? r - DIST_P61 : r;
}

// The LDS address space of a pointer into the workgroup's LDS: a function
// that is not inlined sees its array arguments as generic pointers and would
// otherwise read them with flat loads.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(3))) T* as_lds(const T* p) {
  return (const __attribute__((address_space(3))) T*)p;
}

// Lane l's value of v (l uniform); valid in divergent code, since it reads
// the register directly.
__device__ __forceinline__ u64 readlane64(u64 v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((u64)hi << 32) | lo;
}

// A 64-bit value moved across lanes by a DPP pattern (lanes the pattern or
// the row mask leaves out receive 0).  Patterns: quad_perm [1,0,3,2] (0xB1)
// and [2,3,0,1] (0x4E), row_half_mirror (0x141), row_mirror (0x140),
// row_bcast:15 (0x142) and row_bcast:31 (0x143).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ u64 dpp64(u64 v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
  return ((u64)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Wave sums (every lane active): pairs, quads, half-rows and rows by DPP
// within each row of 16 lanes, then rows 0+1 and 2+3 by broadcasting lane 15
// of a row into the next, and the two halves by broadcasting lane 31; lane 63
// ends with the total, read back for every lane.  Each step is a VALU move
// rather than a round trip through the LDS crossbar.
__device__ __forceinline__ u64 wave_sum(u64 x) {
  x += dpp64<0xB1>(x);
  x += dpp64<0x4E>(x);
  x += dpp64<0x141>(x);
  x += dpp64<0x140>(x);
  x += dpp64<0x142, 0xA>(x);
  x += dpp64<0x143, 0xC>(x);
  return readlane64(x, 63);
}

__device__ __forceinline__ u64 wave_sum_p(u64 x) {
  x = addp(x, dpp64<0xB1>(x));
  x = addp(x, dpp64<0x4E>(x));
  x = addp(x, dpp64<0x141>(x));
  x = addp(x, dpp64<0x140>(x));
  x = addp(x, dpp64<0x142, 0xA>(x));
  x = addp(x, dpp64<0x143, 0xC>(x));
  return readlane64(x, 63);
}

__device__ __forceinline__ u64 ld_coherent(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device memory private to one wave (a per-wave stack, trie or memo table),
// written by some of its lanes and read back by others.  The wave's lanes run
// on one CU, whose vector L1 is write-through and shared by the CU's waves,
// so workgroup scope is enough: the fence waits for the wave's stores, and the
// loads may hit L1 and L2.  (Agent scope would write back and bypass the
// XCD's own L2 on every use.)
__device__ __forceinline__ u64 ld_wave(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// ---- LDS layout -------------------------------------------------------------
// u64 part: A (D*W), gl (D, only with fingerprints), per-level stacks, R (W).  Then a union of the
// arrays used only while G_u is built (nb, rowbeg, rowptr) with the arrays
// used only afterwards (mem, pos, rcap).  Then the small per-level arrays.
struct Lds {
  u64* A;        // D * W
  u64* gl;       // D (null without fingerprints)
  u64* wtab;     // W * 256 nibble table of weight sums (fingerprints, W <= kTabMaxW; else null)
  u64* stP;      // (k-1) * W
  u64* stQ;      // (k-1) * W
  u64* stCnt;    // (k-1) * 2
  u64* stFp;     // (k-1)
  u64* R;        // W   (soft-embedding level bitmap)
  u64* ctl;      // 4   (per-wave state used once per work unit or memo call)
  int32_t* nb;      // D       (build)
  int32_t* rowbeg;  // D + 1   (build)
  int32_t* rowptr;  // D       (build)
  uint16_t* mem;    // D       (search)
  uint16_t* pos;    // D       (search)
  uint8_t* rcap;    // D       (search)
  uint16_t* stX;    // k - 1
  uint8_t* stMemo;  // k - 1
};

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// Fingerprint weight sums over bitmaps use a table of 16 entries per nibble
// (2 KB per bitmap word) for widths up to this; wider launches, whose rows
// already take most of the LDS, sum bit by bit.
constexpr int kTabMaxW = 6;

__host__ __device__ inline size_t wtab_words(int W, int fp) { return (fp && W <= kTabMaxW) ? (size_t)W * 256 : 0; }

// Rows of a launch: its largest root out-degree rounded up to 16, within
// the width class.
__host__ __device__ inline int lds_rows(int W, int dmax) {
  int D = (dmax + 15) & ~15;
  if (D < 16) D = 16;
  return D < 64 * W ? D : 64 * W;
}

// D = rows: the largest out-degree among the launch's roots (at most 64 W),
// so that a launch whose roots are narrower than its class uses less LDS.
// fp = 0 leaves out the fingerprint weights (8 D bytes).
__host__ __device__ inline size_t lds_bytes(int W, int k, int fp, int Drows) {
  size_t D = (size_t)Drows, L = (size_t)(k > 1 ? k - 1 : 1);
  size_t b = 8 * (D * W + (fp ? D : 0) + wtab_words(W, fp) + 2 * L * W + 3 * L + W + 4);
  size_t build = 4 * (3 * D + 1), post = 5 * D;
  b += align8(build > post ? build : post);
  b += align8(3 * L);
  return b;
}

template <int W>
__device__ inline Lds carve(char* base, int k, int fp, int Drows) {
  const size_t D = (size_t)Drows, L = (size_t)(k > 1 ? k - 1 : 1);
  Lds s;
  u64* p = (u64*)base;
  s.A = p; p += D * W;
  s.gl = nullptr;
  if (fp) {
    s.gl = p;
    p += D;
  }
  s.wtab = nullptr;
  if (wtab_words(W, fp)) {
    s.wtab = p;
    p += wtab_words(W, fp);
  }
  s.stP = p; p += L * W;
  s.stQ = p; p += L * W;
  s.stCnt = p; p += 2 * L;
  s.stFp = p; p += L;
  s.R = p; p += W;
  s.ctl = p; p += 4;
  char* u = (char*)p;
  s.nb = (int32_t*)u;
  s.rowbeg = s.nb + D;
  s.rowptr = s.rowbeg + D + 1;
  s.mem = (uint16_t*)u;
  s.pos = s.mem + D;
  s.rcap = (uint8_t*)(s.pos + D);
  size_t build = 4 * (3 * D + 1), post = 5 * D;
  char* t = u + align8(build > post ? build : post);
  s.stX = (uint16_t*)t;
  s.stMemo = (uint8_t*)(s.stX + L);
  return s;
}

// ---- bitmap helpers (W words) -------------------------------------------------

// Σ_{z in q} g(z) mod p over a W-word bitmap held in registers.
template <int W>
__device__ __forceinline__ u64 weight_sum(const u64 (&q)[W], const u64* gl, u64& bits_visited) {
  u64 s = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    u64 b = q[w];
    while (b) {
      int t = __ffsll((unsigned long long)b) - 1;
      b &= b - 1;
      s += gl[w * 64 + t];
      s = (s & DIST_P61) + (s >> 61);
      ++bits_visited;
    }
  }
  return s >= DIST_P61 ? s - DIST_P61 : s;
}

// The nibble table of a root's weights: tab[16 (16 w + n) + v] = sum of
// g(64 w + 4 n + b) over the set bits b of v (mod p), for vertices below d.
template <int W>
__device__ void build_weight_table(const Lds& s, int d) {
  for (int e = lane_id(); e < W * 256; e += kWave) {
    const int base = (e >> 4) * 4, v = e & 15;
    u64 a = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (((v >> b) & 1) && base + b < d) a += s.gl[base + b];
    a = (a & DIST_P61) + (a >> 61);
    s.wtab[e] = a >= DIST_P61 ? a - DIST_P61 : a;
  }
  __syncthreads();
}

// The same sum as weight_sum, sixteen table loads per nonzero word.  Each
// entry is below p < 2^61 and a folded sum below p + 16, so folding after six,
// six and four entries keeps every partial sum below 2^64.
template <int W>
__device__ __forceinline__ u64 weight_sum_tab(const u64 (&q)[W], const u64* tab, u64& bits_visited) {
  u64 s = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 x = q[w];
    if (x) {
      bits_visited += (u64)__popcll(x);
      const u64* t = tab + w * 256;
      u64 a = 0;
#pragma unroll
      for (int n = 0; n < 16; ++n) {
        a += t[n * 16 + (int)((x >> (4 * n)) & 15ull)];
        if (n == 5 || n == 11) a = (a & DIST_P61) + (a >> 61);
      }
      s += (a & DIST_P61) + (a >> 61);
      s = (s & DIST_P61) + (s >> 61);
    }
  }
  return s >= DIST_P61 ? s - DIST_P61 : s;
}

// Σ_{z in q} g(z) mod p: by table where the launch has one.
template <int W>
__device__ __forceinline__ u64 weight_sum_any(const u64 (&q)[W], const u64* gl, const u64* tab, u64& bits) {
  if constexpr (W <= kTabMaxW) {
    if (tab) return weight_sum_tab<W>(q, tab, bits);
  }
  return weight_sum<W>(q, gl, bits);
}

// Word w of the bitmap of local ids >= x.
__device__ __forceinline__ u64 cut_mask(int x, int w) {
  const int lo_b = w * 64;
  return (x <= lo_b) ? ~0ull : (x >= lo_b + 64 ? 0ull : (~0ull << (x - lo_b)));
}

// Edges of G[Y] and their fingerprint sum Σ g(y) g(z) over edges y<z (rows
// hold forward neighbours only).  For each y the sum over its neighbours z
// above it is taken directly, or, where they are the majority of the members
// above y, as the weight of all members above y (kept as a running
// remainder) minus that of the non-neighbours among them: in a dense G[Y] the
// second set is mostly empty words, which the table sum skips.
template <int W>
__device__ __forceinline__ void edges_in(const u64 (&Y)[W], const u64* A, const u64* gl, const u64* tab, int fpon,
                                         u64& cnt, u64& fp, u64& wops, u64& bits) {
  int rest = 0;   // members of Y above the current y
  u64 wrest = 0;  // and their weight sum
  if (fpon) {
#pragma unroll
    for (int w = 0; w < W; ++w) rest += __popcll(Y[w]);
    wrest = weight_sum_any<W>(Y, gl, tab, bits);
  }
#pragma unroll
  for (int w = 0; w < W; ++w) {
    u64 b = Y[w];
    while (b) {
      int t = __ffsll((unsigned long long)b) - 1;
      b &= b - 1;
      int y = w * 64 + t;
      u64 q[W];
      int c = 0;
#pragma unroll
      for (int v = 0; v < W; ++v) {
        q[v] = Y[v] & A[y * W + v];
        c += __popcll(q[v]);
      }
      wops += W;
      cnt += (u64)c;
      if (fpon) {
        const u64 gy = gl[y];
        wrest = subp(wrest, gy);
        --rest;
        if (c) {
          const bool comp = 2 * c > rest;
          u64 z[W];
#pragma unroll
          for (int v = 0; v < W; ++v) z[v] = comp ? (Y[v] & cut_mask(y + 1, v) & ~A[y * W + v]) : q[v];
          const u64 ws = weight_sum_any<W>(z, gl, tab, bits);
          fp = addp(fp, mulp(gy, comp ? subp(wrest, ws) : ws));
        }
      }
    }
  }
}

// ---- Algorithm 5, level by level -------------------------------------------
// Algorithm 5 scans the out-neighbours of x from the highest down and raises
// r(x) from c to c + 1 at the first neighbour y (below the previous one)
// with r(y) >= c.  Pass c therefore needs only R_c = {y : r(y) >= c} and the
// position reached at pass c - 1, and all x can take pass c in parallel.
// rcap[x] = min(r_{G_u}(x), K - 1).  Returns min(r_{G'}(u), K) for the root.
template <int W>
__device__ int soft_embed_levels(const Lds& s, int d, int K) {
  const int lane = lane_id();
  for (int i = lane; i < d; i += kWave) {
    s.rcap[i] = 1;
    s.pos[i] = (uint16_t)d;
  }
  __syncthreads();
  for (int c = 1; c <= K - 2; ++c) {
    for (int w = 0; w < W; ++w) {
      int idx = w * 64 + lane;
      u64 b = __ballot(idx < d && s.rcap[idx] >= c);
      if (lane == 0) s.R[w] = b;
    }
    __syncthreads();
    int raised = 0;
    for (int i = lane; i < d; i += kWave) {
      if (s.rcap[i] != c) continue;
      int ps = s.pos[i];  // search strictly below ps
      int found = -1;
      for (int w = (ps - 1) >> 6; w >= 0 && found < 0; --w) {
        u64 m = s.A[i * W + w] & s.R[w];
        int top = ps - w * 64;  // bits >= top are excluded
        if (top < 64) m &= (top <= 0) ? 0ull : ((1ull << top) - 1);
        if (m) found = w * 64 + 63 - __clzll((long long)m);
      }
      if (found >= 0) {
        s.rcap[i] = (uint8_t)(c + 1);
        s.pos[i] = (uint16_t)found;
        raised = 1;
      }
    }
    __syncthreads();
    if (!__any(raised)) break;
  }
  // root: its out-neighbours are all local vertices
  int r = 1, ps = d;
  for (int c = 1; c <= K - 1; ++c) {
    int found = -1;
    for (int base = ((ps - 1) >> 6) << 6; base >= 0 && ps > 0; base -= 64) {
      int idx = base + lane;
      u64 b = __ballot(idx < ps && s.rcap[idx] >= c);
      if (b) {
        found = base + 63 - __clzll((long long)b);
        break;
      }
    }
    if (found < 0) break;
    r = c + 1;
    ps = found;
  }
  return r;
}

// ---- G_u = G[N+(u)] as bitmap rows in LDS -----------------------------------
// Local id i is the i-th out-neighbour of root r in rank order; row i holds
// the local ids j > i with v_j in N+(v_i).  Each out-list N+(v_i) is read
// from HBM (flattened over the wave so that reads are coalesced) and every
// entry is located in N+(r) by binary search in LDS.  If oid is set, oid[i]
// receives the input id of local vertex i.  Returns the arcs read (per lane).
//
// build_rows takes the vertex list from s.nb[0, d) (ascending rank, written
// before a wave barrier); build_subgraph fills it with N+(r) first.
template <int W>
__device__ u64 build_rows(const Lds& s, const int32_t* dptr, const int32_t* dcol, const u64* gw,
                          const int32_t* orig, int32_t* oid, int d) {
  const int lane = lane_id();
  u64 arcs = 0;
  for (int i = lane; i < d; i += kWave) {
    const int32_t v = s.nb[i];
    if (s.gl) s.gl[i] = gw[v];
    if (oid) oid[i] = orig[v];
    int32_t b = dptr[v];
    s.rowptr[i] = b;
    s.rowbeg[i] = dptr[v + 1] - b;  // length, scanned below
  }
  for (int i = lane; i < d * W; i += kWave) s.A[i] = 0;
  __syncthreads();
  // exclusive scan of row lengths (in chunks of 64)
  int carry = 0;
  for (int base = 0; base < d; base += kWave) {
    int i = base + lane;
    int len = i < d ? s.rowbeg[i] : 0;
    int incl = len;
    for (int off = 1; off < kWave; off <<= 1) {
      int o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (i < d) s.rowbeg[i] = carry + incl - len;
    carry += __shfl(incl, kWave - 1);
  }
  if (lane == 0) s.rowbeg[d] = carry;
  __syncthreads();
  const int total = carry;
  const int32_t top_rank = d ? s.nb[d - 1] : 0;
  for (int t = lane; t < total; t += kWave) {
    // row i: largest i with rowbeg[i] <= t
    int lo = 0, hi = d - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (s.rowbeg[mid] <= t) lo = mid; else hi = mid - 1;
    }
    int i = lo;
    int32_t x = dcol[s.rowptr[i] + (t - s.rowbeg[i])];
    ++arcs;
    if (x > top_rank) continue;
    // locate x among nb[i+1 .. d-1]
    int a = i + 1, b = d;
    while (a < b) {
      int mid = (a + b) >> 1;
      if (s.nb[mid] < x) a = mid + 1; else b = mid;
    }
    if (a < d && s.nb[a] == x) atomicOr(&s.A[i * W + (a >> 6)], 1ull << (a & 63));
  }
  __syncthreads();
  return arcs;
}

template <int W>
__device__ u64 build_subgraph(const Lds& s, const int32_t* dptr, const int32_t* dcol, const u64* gw,
                              const int32_t* orig, int32_t* oid, int32_t beg, int d) {
  // each lane reads back only the entries it wrote
  for (int i = lane_id(); i < d; i += kWave) s.nb[i] = dcol[beg + i];
  return build_rows<W>(s, dptr, dcol, gw, orig, oid, d);
}

}  // namespace
