// pivot.hip -- pivot-based exact clique counting for every k at once.
//
// The paper cites pivot-based counting (Jain and Seshadhri, "The Power of
// Pivoting for Exact Clique Counting") among exact methods that count
// without listing.  This kernel implements it per root, one wavefront per
// root, on the same oriented graph and the same per-root subgraph G_u as the
// search, here with symmetric adjacency rows (both directions) in LDS:
//
//   every clique C of G_u is found exactly once as a root-to-leaf path of a
//   tree of (held, pivot) sets: at a node with candidate set P, choose a
//   pivot p in P with the most neighbours in P; the cliques within P either
//   avoid every non-neighbour of p -- then p is optional: child
//   (P & N(p), p added to the pivots) -- or contain a first non-neighbour v
//   of p in a fixed order: child ((P & N(v)) minus the non-neighbours taken
//   before v, v added to the held set).  A leaf (P empty) with held set H
//   (including the root u) and pivot set Q stands for the cliques H + S,
//   S any subset of Q: for every k, C(|Q|, k - |H|) k-cliques whose
//   fingerprint sum is prod_{v in H} g(v) * e_{k-|H|}(g(Q)).
//
// The elementary symmetric sums of the pivot weights are kept as a
// polynomial, one coefficient per lane (lane j: e_j), multiplied by
// (1 + g(p) t) on entering a pivot child.  Counts and fingerprints for
// k = 1..K accumulate per lane (lane k).  Exact 128-bit counts, fingerprints
// mod 2^61 - 1.
#include "device_common.h"
#include "pivot.h"

namespace {

constexpr int kPivOut = 4 * 64;  // per wave: count lo, hi, fp for k = 0..63, then counters

// Symmetric G_u: row i holds every local j adjacent to i (j < i and j > i).
template <int W>
__device__ u64 build_sym(const Lds& s, const int32_t* dptr, const int32_t* dcol, const u64* gw, int32_t beg, int d) {
  const int lane = lane_id();
  u64 arcs = 0;
  for (int i = lane; i < d; i += kWave) {
    const int32_t v = dcol[beg + i];
    s.nb[i] = v;
    if (s.gl) s.gl[i] = gw[v];
    const int32_t b = dptr[v];
    s.rowptr[i] = b;
    s.rowbeg[i] = dptr[v + 1] - b;
  }
  for (int i = lane; i < d * W; i += kWave) s.A[i] = 0;
  __syncthreads();
  int carry = 0;
  for (int base = 0; base < d; base += kWave) {
    const int i = base + lane;
    const int len = i < d ? s.rowbeg[i] : 0;
    int incl = len;
    for (int off = 1; off < kWave; off <<= 1) {
      const int o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (i < d) s.rowbeg[i] = carry + incl - len;
    carry += __shfl(incl, kWave - 1);
  }
  if (lane == 0) s.rowbeg[d] = carry;
  __syncthreads();
  const int total = carry;
  const int32_t top = d ? s.nb[d - 1] : 0;
  for (int t = lane; t < total; t += kWave) {
    int lo = 0, hi = d - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s.rowbeg[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int i = lo;
    const int32_t x = dcol[s.rowptr[i] + (t - s.rowbeg[i])];
    ++arcs;
    if (x > top) continue;
    int a = i + 1, b = d;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (s.nb[mid] < x) a = mid + 1; else b = mid;
    }
    if (a < d && s.nb[a] == x) {
      atomicOr(&s.A[i * W + (a >> 6)], 1ull << (a & 63));
      atomicOr(&s.A[a * W + (i >> 6)], 1ull << (i & 63));
    }
  }
  __syncthreads();
  return arcs;
}

// Per-wave stack in device memory, one frame per tree depth: the candidate
// set P, the non-neighbours R of the pivot still to branch on, those already
// taken (D), and the polynomial of the pivot weights (K + 1 words).
struct PivFrame {
  u64* P;
  u64* R;
  u64* Dn;
  u64* E;
};

// 128-bit C(n, r) from the binomial table (n <= 1024, r <= 16), else by the
// multiplicative formula (exact while it fits).
__device__ __forceinline__ void binom_at(const u64* tab, int n, int r, u64& lo, u64& hi) {
  if (r < 0 || r > n) {
    lo = hi = 0;
    return;
  }
  if (tab && n <= 1024 && r <= 16) {
    const u64* e = tab + ((size_t)n * 17 + (size_t)r) * 2;
    lo = e[0];
    hi = e[1];
    return;
  }
  lo = 1;
  hi = 0;
  for (int i = 0; i < r; ++i) {
    const u64 m = (u64)(n - i);
    const u64 plo = lo * m;
    hi = hi * m + __umul64hi(lo, m);
    lo = plo;
    // divide (hi:lo) by i + 1 in 32-bit limbs
    const u64 dv = (u64)(i + 1);
    u64 rem = 0;
    uint32_t limb[4] = {(uint32_t)(hi >> 32), (uint32_t)hi, (uint32_t)(lo >> 32), (uint32_t)lo};
    for (int q = 0; q < 4; ++q) {
      const u64 cur = (rem << 32) | limb[q];
      limb[q] = (uint32_t)(cur / dv);
      rem = cur % dv;
    }
    hi = ((u64)limb[0] << 32) | limb[1];
    lo = ((u64)limb[2] << 32) | limb[3];
  }
}

// Stack words are written by some lanes and read back by all (wave-private).
__device__ __forceinline__ u64 sld(const u64* a) { return ld_wave(a); }

template <int W>
__global__ __launch_bounds__(64, 1) void k_pivot(PivParams p) {
  extern __shared__ __align__(16) char smem[];
  const int lane = lane_id();
  const int K = p.kmax;
  const bool fp = p.fingerprint != 0;
  const Lds s = carve<W>(smem, 2, p.fingerprint, p.drows);
  const int D = p.drows;
  // this wave's stack: frames of fw words for depths 0 .. D + 1, then four
  // scalar words per depth (h, q, prod, pivot)
  const size_t fw = (size_t)3 * W + (size_t)(K + 1);
  u64* stack = p.stack + (size_t)blockIdx.x * pivot_stack_words(W, K, D);
  u64* scal = stack + (size_t)(D + 2) * fw;
  auto F = [&](int depth) {
    PivFrame f;
    u64* b = stack + (size_t)depth * fw;
    f.P = b;
    f.R = b + W;
    f.Dn = b + 2 * W;
    f.E = b + 3 * W;
    return f;
  };
  // accumulators: lane j holds the j-cliques (count, fp) found so far
  u64 acc_lo = 0, acc_hi = 0, acc_fp = 0;
  u64 n_nodes = 0, n_leaves = 0, n_roots = 0, arcs = 0;
  bool aborted = false;
  const u64 t_start = wall_clock64();
  const u64 deadline = p.deadline ? t_start + p.deadline : 0;
  // A heavy root is shared by nsub units.  Every unit builds G_u and walks
  // the tree down to depth split_depth (the pivot choice is
  // deterministic, so all of them see the same nodes in the same order); the
  // nodes at that depth are dealt out round-robin, and the leaves above it
  // count in unit 0 only.
  const uint32_t nsub = p.nsub > 1 ? (uint32_t)p.nsub : 1u;
  const int split_depth = p.split_depth > 0 ? p.split_depth : 1;
  const uint32_t nunits = (uint32_t)p.nroots * nsub;
  for (;;) {
    uint32_t ui = 0;
    if (lane == 0) ui = atomicAdd(p.cursor, 1u);
    ui = (uint32_t)__shfl((int)ui, 0);
    if (ui >= nunits) break;
    const uint32_t ri = ui / nsub, sub = ui % nsub;
    if (__hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      aborted = true;
      break;
    }
    const int32_t r = p.roots[ri];
    const int32_t beg = p.dptr[r];
    const int d = p.dptr[r + 1] - beg;
    if (sub == 0) ++n_roots;
    arcs += build_sym<W>(s, p.dptr, p.dcol, p.gw, beg, d);
    u64 r_lo = 0, r_hi = 0, r_fp = 0;  // this root's cliques of size per_root_k
    {
      PivFrame f0 = F(0);
      if (lane < W) {
        const int lo_b = lane * 64;
        f0.P[lane] = d >= lo_b + 64 ? ~0ull : (d <= lo_b ? 0ull : ((1ull << (d - lo_b)) - 1));
      }
      if (lane <= K) f0.E[lane] = lane == 0 ? 1ull : 0ull;
    }
    wave_fence();
    int depth = 0;
    int h = 1, q = 0;  // held (the root first) and pivot counts
    u64 prod = fp ? p.gw[r] : 0ull;
    enum { ENTER, NEXT, FINISH } mode = ENTER;
    uint32_t n_split = 0;  // nodes entered so far at depth split_depth
    while (true) {
      const PivFrame f = F(depth);
      if (mode == ENTER) {
        const bool shared = nsub > 1 && depth < split_depth;  // walked by every unit of the root
        if (nsub > 1 && depth == split_depth && (n_split++ % nsub) != sub) {
          mode = FINISH;
          continue;
        }
        if (!shared || sub == 0) ++n_nodes;
        if (deadline && (n_nodes & 63) == 0 && wall_clock64() > deadline) {
          if (lane == 0) atomicOr(p.abort_flag, 1);
          aborted = true;
          break;
        }
        u64 P[W];
        int np = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          P[w] = sld(f.P + w);
          np += __popcll(P[w]);
        }
        if (np == 0 || h >= K) {
          // a leaf: the cliques H + S, S any subset of the pivots Q.  With
          // h = K only S = {} still has size <= K: the held set alone.
          if (shared && sub != 0) {
            mode = FINISH;
            continue;
          }
          ++n_leaves;
          const int qq = np == 0 ? q : 0;
          const u64 e_here = (lane <= K) ? sld(f.E + lane) : 0ull;
          const int need = lane - h;  // lane j: j-cliques take j - h pivots
          const u64 e_need = __shfl(e_here, (need >= 0 && need <= K) ? need : 0);
          if (lane >= h && lane <= K && need <= qq) {
            u64 clo, chi;
            binom_at(p.binom, qq, need, clo, chi);
            const u64 nlo = acc_lo + clo;
            acc_hi += chi + (nlo < acc_lo ? 1ull : 0ull);
            acc_lo = nlo;
            u64 f2 = 0;
            if (fp) {
              f2 = mulp(prod, np == 0 ? e_need : (need == 0 ? 1ull : 0ull));
              acc_fp = addp(acc_fp, f2);
            }
            if (lane == p.per_root_k) {
              const u64 t = r_lo + clo;
              r_hi += chi + (t < r_lo ? 1ull : 0ull);
              r_lo = t;
              r_fp = addp(r_fp, f2);
            }
          }
          mode = FINISH;
          continue;
        }
        // members of P, then the pivot: the member with the most neighbours
        // in P (ties: the lowest local id)
#pragma unroll
        for (int w = 0, nb = 0; w < W; ++w) {
          const u64 bw = P[w];
          if ((bw >> lane) & 1ull) s.mem[nb + __popcll(bw & lanemask_lt())] = (uint16_t)(w * 64 + lane);
          nb += __popcll(bw);
        }
        __syncthreads();
        int best = -1, bestc = -1;
        u64 csum = 0;  // neighbours in P, summed over the members
        for (int base = 0; base < np; base += kWave) {
          const int i = base + lane;
          int c = -1, idx = -1;
          if (i < np) {
            idx = s.mem[i];
            c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += __popcll(P[w] & s.A[idx * W + w]);
            csum += (u64)c;
          }
          for (int off = 32; off > 0; off >>= 1) {
            const int oc = __shfl_xor(c, off), oi = __shfl_xor(idx, off);
            if (oc > c || (oc == c && oi >= 0 && (idx < 0 || oi < idx))) {
              c = oc;
              idx = oi;
            }
          }
          if (c > bestc) {
            bestc = c;
            best = idx;
          }
        }
        __syncthreads();
        if (wave_sum(csum) == (u64)np * (u64)(np - 1)) {
          // a complete P: its tree is the chain of pivot children down to an
          // empty set, i.e. one leaf whose pivots gain every member of P
          // (the polynomial times (1 + g(v) t) for each)
          if (shared && sub != 0) {
            mode = FINISH;
            continue;
          }
          ++n_leaves;
          u64 e = (lane <= K) ? sld(f.E + lane) : 0ull;
          if (fp) {
            for (int i = 0; i < np; ++i) {
              const u64 g = s.gl[s.mem[i]];
              const u64 prev = __shfl_up(e, 1);
              if (lane >= 1 && lane <= K) e = addp(e, mulp(prev, g));
            }
          }
          const int qq = q + np;
          const int need = lane - h;
          const u64 e_need = __shfl(e, (need >= 0 && need <= K) ? need : 0);
          if (lane >= h && lane <= K && need <= qq) {
            u64 clo, chi;
            binom_at(p.binom, qq, need, clo, chi);
            const u64 nlo = acc_lo + clo;
            acc_hi += chi + (nlo < acc_lo ? 1ull : 0ull);
            acc_lo = nlo;
            u64 f2 = 0;
            if (fp) {
              f2 = mulp(prod, e_need);
              acc_fp = addp(acc_fp, f2);
            }
            if (lane == p.per_root_k) {
              const u64 t = r_lo + clo;
              r_hi += chi + (t < r_lo ? 1ull : 0ull);
              r_lo = t;
              r_fp = addp(r_fp, f2);
            }
          }
          __syncthreads();
          mode = FINISH;
          continue;
        }
        // R: members of P that are neither the pivot nor its neighbours
        if (lane < W) {
          u64 rw = P[lane] & ~s.A[best * W + lane];
          if ((best >> 6) == lane) rw &= ~(1ull << (best & 63));
          f.R[lane] = rw;
          f.Dn[lane] = 0;
        }
        if (lane == 0) {
          scal[4 * depth + 0] = (u64)h;
          scal[4 * depth + 1] = (u64)q;
          scal[4 * depth + 2] = prod;
          scal[4 * depth + 3] = (u64)best;
        }
        // pivot child: P & N(p), p joins the pivots (polynomial times (1 + g(p) t))
        const PivFrame c = F(depth + 1);
        if (lane < W) c.P[lane] = P[lane] & s.A[best * W + lane];
        {
          const u64 e = (lane <= K) ? sld(f.E + lane) : 0ull;
          const u64 prev = __shfl_up(e, 1);
          u64 ne = e;
          if (fp && lane >= 1 && lane <= K) ne = addp(e, mulp(prev, s.gl[best]));
          if (lane <= K) c.E[lane] = ne;
        }
        wave_fence();
        ++depth;
        ++q;
        continue;
      }
      if (mode == NEXT) {
        // the next non-neighbour v of this depth's pivot: child
        // (P & N(v)) minus the non-neighbours taken before v, v held
        int v = -1;
#pragma unroll
        for (int w = W - 1; w >= 0; --w) {
          const u64 rw = sld(f.R + w);
          if (rw) v = w * 64 + __ffsll((unsigned long long)rw) - 1;
        }
        if (v < 0) {
          mode = FINISH;
          continue;
        }
        h = (int)sld(scal + 4 * depth + 0);
        q = (int)sld(scal + 4 * depth + 1);
        prod = sld(scal + 4 * depth + 2);
        const PivFrame c = F(depth + 1);
        if (lane < W) {
          const u64 dn = sld(f.Dn + lane);
          c.P[lane] = sld(f.P + lane) & s.A[v * W + lane] & ~dn;
          const u64 rw = sld(f.R + lane);
          const u64 bit = (v >> 6) == lane ? (1ull << (v & 63)) : 0ull;
          f.R[lane] = rw & ~bit;
          f.Dn[lane] = dn | bit;
        }
        if (lane <= K) c.E[lane] = sld(f.E + lane);
        wave_fence();
        if (fp) prod = mulp(prod, s.gl[v]);
        ++h;
        ++depth;
        mode = ENTER;
        continue;
      }
      // FINISH: back to the parent, which continues with its non-neighbours
      if (depth == 0) break;
      --depth;
      mode = NEXT;
    }
    if (aborted) break;
    if (p.per_root) {
      const int src = (p.per_root_k >= 0 && p.per_root_k < kWave) ? p.per_root_k : 0;
      const u64 rl = __shfl(r_lo, src), rh = __shfl(r_hi, src), rf = __shfl(r_fp, src);
      if (lane == 0) {
        u64* o = p.per_root + 3 * (u64)p.orig[r];
        if (nsub == 1) {
          o[0] = rl;
          o[1] = rh;
          o[2] = rf;
        } else {
          // the root's units add up (the output starts at zero)
          const u64 old = atomicAdd((unsigned long long*)&o[0], (unsigned long long)rl);
          atomicAdd((unsigned long long*)&o[1], (unsigned long long)(rh + (old + rl < old ? 1ull : 0ull)));
          u64 cur = o[2], seen;
          do {
            seen = cur;
            cur = atomicCAS((unsigned long long*)&o[2], seen, addp(seen, rf));
          } while (cur != seen);
        }
      }
    }
  }
  u64* o = p.wave_out + (u64)blockIdx.x * kPivOut;
  if (lane <= K) {
    o[3 * lane + 0] = acc_lo;
    o[3 * lane + 1] = acc_hi;
    o[3 * lane + 2] = acc_fp;
  }
  const u64 na = wave_sum(arcs);
  if (lane == 0) {
    o[192] = n_nodes;
    o[193] = n_leaves;
    o[194] = n_roots;
    o[195] = na;
    o[196] = aborted ? 1 : 0;
  }
}

}  // namespace

int pivot_launch(int W, const PivParams& prm, int grid, size_t lds, hipStream_t s) {
  const void* fn = nullptr;
  switch (W) {
    case 1: fn = (const void*)k_pivot<1>; break;
    case 2: fn = (const void*)k_pivot<2>; break;
    case 3: fn = (const void*)k_pivot<3>; break;
    case 4: fn = (const void*)k_pivot<4>; break;
    case 5: fn = (const void*)k_pivot<5>; break;
    case 6: fn = (const void*)k_pivot<6>; break;
    case 8: fn = (const void*)k_pivot<8>; break;
    default: fn = (const void*)k_pivot<16>; break;
  }
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return DIST_E_DEVICE;
  PivParams p = prm;
  void* args[] = {&p};
  if (hipLaunchKernel(fn, dim3(grid), dim3(64), args, lds, s) != hipSuccess) return DIST_E_DEVICE;
  return hipGetLastError() == hipSuccess ? DIST_OK : DIST_E_DEVICE;
}

int pivot_occupancy(int W, size_t lds) {
  const void* fn = nullptr;
  switch (W) {
    case 1: fn = (const void*)k_pivot<1>; break;
    case 2: fn = (const void*)k_pivot<2>; break;
    case 3: fn = (const void*)k_pivot<3>; break;
    case 4: fn = (const void*)k_pivot<4>; break;
    case 5: fn = (const void*)k_pivot<5>; break;
    case 6: fn = (const void*)k_pivot<6>; break;
    case 8: fn = (const void*)k_pivot<8>; break;
    default: fn = (const void*)k_pivot<16>; break;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, lds) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

size_t pivot_lds_bytes(int W, int fp, int drows) { return lds_bytes(W, 2, fp, drows); }
