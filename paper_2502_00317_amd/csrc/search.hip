// search.hip -- per-root k-clique search on the oriented graph.
//
// NodeParallel over roots (Section VII-D): one wavefront owns one root at a
// time and takes the next root from a global counter (roots sorted by
// out-degree descending, widest first).  For root u with d = |N+(u)|:
//
//  * the 1-induced subgraph G_u = G[N+(u)] (Section II-A, Table 1) is built
//    in LDS as d bitmap rows of W = ceil(d/64) words: row i holds the local
//    ids j > i with v_j in N+(v_i).  Out-lists are read from HBM coalesced
//    and located in N+(u) by binary search in LDS;
//  * Algorithm 5 is evaluated on G_u level by level (bit-parallel form of
//    the same greedy scan, see soft_embed_levels) giving r_{G_u}(x) capped at
//    k-1 for every local x, and r_{G'}(u) for G' = G[N(u) u {u}]; the root is
//    dropped if r_{G'}(u) < k (Section V: applied at Algorithm 2 line 10);
//  * the (k-1)-cliques of G_u are counted by depth-first search over
//    candidate bitmaps (Algorithm 1's Listing): a search node holds the set
//    P of candidates and the number l of vertices still needed; the child
//    for candidate x is P & A[x].  Children of one node are evaluated one
//    per lane (AND + popcount over W words), survivors are kept in a bitmap
//    and expanded highest vertex first.  A child x survives only if
//    |P & A[x]| >= l - 1 and r_{G_u}(x) >= l (Lemma 1: a vertex whose
//    soft-embedding bound is below l is the minimum of no l-clique);
//  * nodes with l = 2 count the edges of G[P]; nodes with l = 3 let every
//    lane count the edges of its own child, so the last two levels run
//    lane-parallel;
//  * dense nodes (criterion (1): 2 m l > (l - 1) n^2 for n = |P|, m = edges
//    of G[P], l >= 4) switch to the memoised search of Algorithm 3 in
//    counting form: every node below keeps, per wave, a hash table keyed by
//    (root, l, P) holding the number of l-cliques of G[P] and their
//    fingerprint sum.  Keys are vertex sets, i.e. Induced Subgraph Trie
//    nodes (a trie node is identified by its identifying string, which is
//    its vertex set).  After the child of x completes, the node inserts the
//    prefix P & [x, inf) -- the trie node t_i of Algorithm 3's path, marked
//    for l -- and on entry a node resumes from its longest memoised prefix,
//    the retrieval of Algorithm 4 summed instead of enumerated:
//      cnt(t, l) = cnt(L^C_t(l), l - 1) + cnt(L^S_t(l), l).
//
// Every quantity is an integer; the result is exact (u128 count, fp mod
// 2^61 - 1) and independent of scheduling.  Listing (records of cliques)
// runs in ist.hip on the linked trie of Algorithms 3 and 4.
#include "device_common.h"
#include "ist.h"
#include "pivot.h"

#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <thread>
#include <type_traits>

namespace {

constexpr int kOutWords = 16;
// The memo table is direct-mapped: a key lives in its home slot only, so an
// insert is a plain store (no read first) and a lookup reads one entry.
constexpr int kMemoProbe = 1;
// A root stops using its memo table once at least kMemoMinLook lookups
// found fewer than one hit in kMemoMinRatio, or at least kMemoMinLook
// inserts were answered by fewer than one hit in kMemoMinInsRatio (the table
// is a cache: using it or not never changes a result).  Where the closed
// forms already cover the dense branches, hits mostly save single leaf
// frames and do not repay the lookups and inserts; one hit in four lookups
// is about where they break even, and inserts (a trie node after each child)
// outnumber lookups, so they are bounded on their own.  A wave stops for
// all its later units once kMemoWaveIns inserts drew fewer than one hit in
// kMemoWaveRatio.  The samples are short: a launch holds thousands of waves,
// and since complete child sets are counted without frames, a hit saves
// little, so an unproductive table costs more than a late decision gains.
constexpr int kMemoMinLook = 256;
constexpr int kMemoMinRatio = 4;
constexpr int kMemoMinInsRatio = 8;
constexpr u64 kMemoWaveIns = 256;
constexpr u64 kMemoWaveRatio = 16;

// Batched counting: one entry per (graph, k) pair, and the units of a
// launch as segments [unit_begin, next unit_begin) of consecutive roots of
// one pair (one unit per root).
// An EdgeParallel work unit (Section VII-D): the arc (u, v) of a heavy root
// u, searched for (k-2)-cliques in G[N+(u) & N+(v)].  That vertex set is
// row v of G_u, stored as a bitmap over N+(u) (wu words from word `row` of
// the edge row store).
struct EdgeRec {
  int32_t u, v;  // ranks
  int32_t d;     // |N+(u) & N+(v)|; 0: the arc cannot start a k-clique's second vertex
  int32_t wu;    // words of the row
  u64 row;
};

struct BatchGraph {
  const int32_t* dptr;
  const int32_t* dcol;
  const int32_t* orig;
  const int32_t* roots;
  const u64* gw;
  int32_t k;
  int32_t own_clock;  // 1: the budget runs from the pair's first unit; 0: from the batch's
  u64 budget;         // wall-clock ticks this pair may use; 0 = no limit
  int32_t memo = -1;  // this pair's memo switch; < 0: the launch's
  int32_t pad_ = 0;
  // EdgeParallel units: roots[i] indexes edges, and k is the clique size
  // minus one (the units start one level down)
  const EdgeRec* edges = nullptr;
  const u64* erows = nullptr;
};

struct BatchSeg {
  uint32_t unit_begin;
  int32_t pair;
  int32_t a;          // first root (index into the pair's roots array)
  int32_t upr;        // work units per root in this segment (>= 1)
  uint32_t pair_end;  // end of the pair's units in this launch (they are contiguous)
  int32_t sub;        // units per range of depth-1 children (>= 1; upr is a multiple)
};

struct Params {
  const int32_t* dptr;
  const int32_t* dcol;
  const u64* gw;
  const int32_t* orig;
  const int32_t* roots;
  int32_t root_begin, root_end;
  int k;            // clique size (search) or cap (soft-embedding mode)
  int prune;
  int memo;
  int fingerprint;
  int soft_only;    // 1: only compute r_{G'}(u) (capped at k) into soft_out
  int32_t* soft_out;
  unsigned* cursor;
  const int32_t* root_deg;   // out-degree of roots[i]
  const BatchGraph* bg;      // batch mode (null: one graph, the fields above)
  const BatchSeg* segs;
  int32_t nsegs;
  u64* pair_out;             // batch: 4 words per pair, accumulated: count lo, hi; fingerprint
                             // residues summed exactly as 128 bits (lo, hi), reduced mod p at the end
  int* pair_abort;           // batch: set for a pair that ran out of its budget
  unsigned* pair_rem;        // batch: units of each pair not finished yet
  unsigned long long* pair_t0;  // batch: [0] first unit of the batch, [1 + i] first unit of pair i
  u64* pair_host;            // batch: host-mapped {flag, lo, hi, fp, t_first, t_last} per pair
  uint32_t units;            // work units in this bucket
  int chunk_work;            // the unit-size switch the host planned with (0 = automatic)
  int32_t drows;             // LDS rows of G_u for this launch (>= every root's out-degree)
  u64* wave_out;
  u64* per_root;
  u64* memo_base;
  u64 memo_mask;
  u64 tag_base;
  const u64* epoch;          // if set, root tags start at *epoch + tag_base
  u64 deadline;     // wall_clock64() limit; 0 = none
  int* abort_flag;
  u64 tau;          // > 0: memo shared by the consecutive roots of a wave (see below)
  uint32_t chunk;   // units a wave takes from the cursor at a time (>= 1)
};


// ---- per-wave memo table (Induced Subgraph Trie nodes, counting form) --------
// Entry: [tag][key W words][cnt_lo][cnt_hi][fp]; tag = (root tag << 8) | l.

// Keys are candidate sets read from LDS: P (W words), optionally cut to its
// members >= x (x < 0: no cut), i.e. the trie node P & [x, inf).
template <int W>
__device__ __forceinline__ u64 memo_hash(u64 tag, const u64* P, int x) {
  u64 h = tag * 0x9E3779B97F4A7C15ull;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    h ^= P[w] & cut_mask(x, w);
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
  }
  h ^= h >> 32;
  return h;
}

// A lookup's lanes cover (key, entry word) pairs: every word of every probed
// entry is loaded by its own lane in one round, so a lookup of one key, or of
// a node's prefixes together, costs one memory latency and each lane holds a
// single word.

// ---- the shared form (p.tau > 0) ---------------------------------------------
// Section VI keeps one Induced Subgraph Trie for the consecutive depth-1
// subtasks a thread takes, bounded by tau nodes: past tau it is cleared
// before the next subtask, and it never grows past 2 tau.  Here a wave's table
// lives on across the roots it takes (units come in runs of consecutive
// roots), so a node must be named by something every root agrees on: its
// vertex set as global ranks, not as a root's local ids.  An entry holds the
// tag (the wave's clear tag << 8 | l), a hash of the ranks, their number and
// the ranks themselves (two per word), so a hit is an exact match of the set.
// Sets of more than kShMax members are not memoised in this form.  The count
// (and fingerprint) of the l-cliques of G[S] depends on S alone -- pruning and
// closed forms never change it -- so an entry made under one root is valid
// under every other root of the same graph.
constexpr int kShMax = 60;
constexpr uint32_t kShChunk = 8;  // units a wave takes at a time in the shared form
constexpr int kShES = 6 + kShMax / 2;  // entry words

// Position of the t-th set bit of v (t < popcount(v)).
__device__ __forceinline__ int select_bit(u64 v, int t) {
  int pos = 0;
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) {
    const u64 low = (1ull << sh) - 1;
    const int c = __popcll(v & low);
    if (t >= c) {
      t -= c;
      v >>= sh;
      pos += sh;
    } else {
      v &= low;
    }
  }
  return pos;
}

// The members of P & [x, inf) as global ranks (nbr: the root's out-neighbour
// list, local id i = nbr[i]); lane t holds the t-th (ranks ascend with local
// ids), h their hash.  Returns their number, or -1 past kShMax.
template <int W>
__device__ __forceinline__ int shared_key(const u64 (&P)[W], int x, const int32_t* nbr, uint32_t& rank, u64& h) {
  const int lane = lane_id();
  int base = 0, mine = -1;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 bits = P[w] & cut_mask(x, w);
    const int c = __popcll(bits);
    if (lane >= base && lane < base + c) mine = w * 64 + select_bit(bits, lane - base);
    base += c;
  }
  if (base > kShMax) return -1;
  rank = mine >= 0 ? (uint32_t)nbr[mine] : 0xffffffffu;
  u64 z = mine >= 0 ? ((u64)rank + 1) * 0x9E3779B97F4A7C15ull : 0ull;
  z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
  h = wave_sum(mine >= 0 ? (z ^ (z >> 29)) : 0ull) + (u64)base;
  h ^= h >> 32;
  return base;
}

// Entry word w of the shared form for the key (tag, ranks in lanes, n).
// Wave-collective (lane shuffles): call it on every lane.
__device__ __forceinline__ u64 shared_word(int w, u64 tag, u64 h, int n, uint32_t rank) {
  const int i = w >= 6 ? w - 6 : 0;
  const uint32_t r0 = (uint32_t)__shfl((int)rank, 2 * i);
  const uint32_t r1 = (2 * i + 1 < n) ? (uint32_t)__shfl((int)rank, 2 * i + 1) : 0xffffffffu;
  if (w == 0) return tag;
  if (w == 1) return h;
  if (w == 2) return (u64)n;
  return ((u64)r1 << 32) | r0;
}

// Not inlined (the shared form is a mode of its own; inline, its key code
// would add registers to every memo call of the search).  P is in LDS.
struct ShHit {
  u64 lo, hi, fp;
  bool hit;
};

template <int W>
__device__ __noinline__ ShHit shared_find(u64* table, u64 mask, u64 tag, const u64* P_, int x, const int32_t* nbr) {
  const auto* P = as_lds(P_);
  const int lane = lane_id();
  ShHit r{0, 0, 0, false};
  uint32_t rank = 0;
  u64 h = 0;
  u64 Pw[W];
#pragma unroll
  for (int w = 0; w < W; ++w) Pw[w] = P[w];
  const int n = shared_key<W>(Pw, x, nbr, rank, h);
  if (n < 0) return r;
  const int w = lane;
  u64 v = 0;
  if (w < kShES) v = ld_wave(table + (h & mask) * kShES + w);
  const u64 want = shared_word(w, tag, h, n, rank);
  const bool ok = w >= kShES || (w >= 3 && w < 6) || (w >= 6 && 2 * (w - 6) >= n) || v == want;
  if (__ballot(!ok)) return r;
  r.lo = __shfl(v, 3);
  r.hi = __shfl(v, 4);
  r.fp = __shfl(v, 5);
  r.hit = true;
  return r;
}

template <int W>
__device__ __noinline__ void shared_put(u64* table, u64 mask, u64 tag, const u64* P_, int x, const int32_t* nbr,
                                        u64 lo, u64 hi, u64 fp) {
  const auto* P = as_lds(P_);
  const int lane = lane_id();
  uint32_t rank = 0;
  u64 h = 0;
  u64 Pw[W];
#pragma unroll
  for (int w = 0; w < W; ++w) Pw[w] = P[w];
  const int n = shared_key<W>(Pw, x, nbr, rank, h);
  if (n < 0) return;
  const u64 kw = shared_word(lane, tag, h, n, rank);  // every lane: it reads ranks across lanes
  const u64 v = lane == 3 ? lo : (lane == 4 ? hi : (lane == 5 ? fp : kw));
  if (lane < kShES) table[(h & mask) * kShES + lane] = v;
}

// Wave-collective lookup of the keys P & [cut_i, inf), i = 0..ncut-1, where
// cut_i = cuts[i] (cuts == nullptr: one key, no cut).  Returns the smallest i
// whose key is in the table (its count and fingerprint in lo, hi, fp), or -1.
// nbr (shared form only): the root's out-neighbour list; the shared form
// takes one key per lookup.
template <int W>
__device__ __forceinline__ int memo_find(const Params& p, const u64* table, u64 tag, const u64* P,
                                         const uint16_t* cuts, int ncut, u64& lo, u64& hi, u64& fp,
                                         const int32_t* nbr = nullptr) {
  if (p.tau) {
    if (ncut != 1) return -1;
    const ShHit r = shared_find<W>(const_cast<u64*>(table), p.memo_mask, tag, P, cuts ? (int)cuts[0] : -1, nbr);
    if (!r.hit) return -1;
    lo = r.lo;
    hi = r.hi;
    fp = r.fp;
    return 0;
  }
  constexpr int ES = W + 4;
  constexpr int GPR = kWave / ES;  // (key, slot) groups per round
  const int lane = lane_id();
  const int groups = ncut * kMemoProbe;
  for (int g0 = 0; g0 < groups; g0 += GPR) {
    const int gi = lane / ES, w = lane % ES, g = g0 + gi;
    bool ok = false;
    u64 v = 0;
    if (gi < GPR && g < groups) {
      const int i = g / kMemoProbe, t = g % kMemoProbe;
      const int x = cuts ? (int)cuts[i] : -1;
      const u64 h = memo_hash<W>(tag, P, x);
      v = ld_wave(table + ((h + (u64)t) & p.memo_mask) * ES + w);
      ok = w > W || v == (w == 0 ? tag : (P[w - 1] & cut_mask(x, w - 1)));
    }
    const u64 b = __ballot(ok);
    constexpr u64 kFull = (ES >= 64) ? ~0ull : ((1ull << ES) - 1);
    for (int q = 0; q < GPR && g0 + q < groups; ++q) {
      if (((b >> (q * ES)) & kFull) == kFull) {
        lo = __shfl(v, q * ES + W + 1);
        hi = __shfl(v, q * ES + W + 2);
        fp = __shfl(v, q * ES + W + 3);
        return (g0 + q) / kMemoProbe;
      }
    }
  }
  return -1;
}

// Wave-collective insert of (tag, P & [x, inf)) -> (lo, hi, fp) into the
// key's home slot, one entry word per lane (a coalesced store; an older entry
// there is evicted).
template <int W>
__device__ __forceinline__ void memo_put(const Params& p, u64* table, u64 tag, const u64* P, int x, u64 lo, u64 hi,
                                         u64 fp, const int32_t* nbr = nullptr, bool room = true) {
  if (p.tau) {
    if (room) shared_put<W>(table, p.memo_mask, tag, P, x, nbr, lo, hi, fp);
    return;
  }
  constexpr int ES = W + 4;
  const int lane = lane_id();
  if (lane < ES) {
    const u64 h = memo_hash<W>(tag, P, x);
    const u64 v = lane == 0 ? tag
                            : (lane <= W ? (P[lane - 1] & cut_mask(x, lane - 1))
                                         : (lane == W + 1 ? lo : (lane == W + 2 ? hi : fp)));
    table[(h & p.memo_mask) * ES + lane] = v;
  }
}

// Work units per root.  A root with more than 64 out-neighbours is cut into
// ranges of depth-1 children so that many waves share it; every unit
// rebuilds G_u in its wave's LDS, so a unit should hold enough search to
// repay that build.  With chunk_work > 0 a range holds max(1, chunk_work / d)
// children.  Automatic (chunk_work 0): for k <= 6 the same with 1024; for
// deeper searches a depth-1 subtree costs roughly (d/64)^(k-3), and a range
// holds children worth about kUnitCost of that, so light roots stay whole
// (one build) while the children of heavy roots become units of their own.
// (For shallow searches the ranges this gives are too coarse: the few heavy
// ones then hold the launch.)  Roots of up to 64 stay one unit.
constexpr double kUnitCost = 512.0;

inline int children_per_unit(int d, int k, int chunk_work) {
  if (k <= 3 || d <= 64) return d;
  const double c = chunk_work > 0 ? (double)(chunk_work / d)
                   : k <= 6       ? (double)(1024 / d)
                                  : kUnitCost / std::pow((double)d / 64.0, (double)(k - 3));
  if (c < 1.0) return 1;
  if (c >= (double)d) return d;
  return (int)c;
}

inline int units_per_root(int d, int k, int chunk_work) {
  const int c = children_per_unit(d, k, chunk_work);
  return (d + c - 1) / c;
}

// At most this many units share one range of depth-1 children (k >= 6).
constexpr int kMaxSub = 32;

// (hi * 2^64 + lo) mod p, p = 2^61 - 1 (2^64 = 8 mod p).
__device__ __forceinline__ u64 fold_p(u64 hi, u64 lo) {
  const u64 l = (lo & DIST_P61) + (lo >> 61);
  const u64 h = (hi & DIST_P61) + (hi >> 61);
  return addp(mulp(h % DIST_P61, 8ull), l % DIST_P61);
}

// 128-bit atomic accumulation (lo word, then the carry into the hi word).
__device__ __forceinline__ void atomic_add128(u64* o, u64 lo, u64 hi) {
  const u64 old = atomicAdd((unsigned long long*)o, (unsigned long long)lo);
  const u64 carry = (old + lo < old) ? 1ull : 0ull;
  if (hi + carry) atomicAdd((unsigned long long*)(o + 1), (unsigned long long)(hi + carry));
}

// Every unit of a batch ends here (searched, skipped or cut off); n units
// at once when a wave skips the rest of a cut-off pair.  The last unit of a
// pair publishes the pair's result to host-mapped memory, so the host can
// complete that query while the rest of the batch still runs.
__device__ void finish_units(const Params& p, int pair, uint32_t n) {
  if (!p.pair_rem || pair < 0) return;
  if (lane_id() == 0) {
    __threadfence();  // this unit's additions to pair_out come first
    unsigned left = atomicSub(p.pair_rem + pair, n);
    if (left == n) {
      __threadfence();
      const u64* o = p.pair_out + 4 * (u64)pair;
      u64 lo = __hip_atomic_load(o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      u64 hi = __hip_atomic_load(o + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      u64 fp = fold_p(__hip_atomic_load(o + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(o + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      int ab = __hip_atomic_load(p.pair_abort + pair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      u64 t1 = __hip_atomic_load(p.pair_t0 + 1 + pair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      u64* h = p.pair_host + 6 * (u64)pair;
      __hip_atomic_store(h + 1, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(h + 2, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(h + 3, fp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(h + 4, t1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(h + 5, (u64)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __threadfence_system();
      __hip_atomic_store(h, ab ? 2ull : 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// A cut-off pair: hand out none of its remaining units in this launch (its
// units are contiguous up to pair_end) and count them as finished.
__device__ uint32_t skip_rest(const Params& p, uint32_t pair_end) {
  uint32_t skipped = 0;
  if (lane_id() == 0) {
    uint32_t old = atomicMax(p.cursor, pair_end);
    skipped = old < pair_end ? pair_end - old : 0u;
  }
  return __shfl(skipped, 0);
}

// The first wall-clock time stored in *slot (set by whichever wave gets
// there first).
__device__ u64 first_time(unsigned long long* slot, u64 now) {
  u64 t = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (t) return t;
  u64 old = atomicCAS(slot, 0ull, (unsigned long long)now);
  return old ? old : now;
}

// ---- complete candidate sets ------------------------------------------------
// If G[P] is complete every l-subset of P is an l-clique: the node holds
// C(|P|, l) cliques whose fingerprint sum is the elementary symmetric sum
// e_l of the weights of P.  Exact; it replaces the search below the node.

// 128-bit value divided by a small d (< 2^31), in 32-bit limbs.
__device__ __forceinline__ void div_small(u64& hi, u64& lo, u64 d) {
  u64 r = 0;
  uint32_t limb[4] = {(uint32_t)(hi >> 32), (uint32_t)hi, (uint32_t)(lo >> 32), (uint32_t)lo};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    u64 cur = (r << 32) | limb[i];
    limb[i] = (uint32_t)(cur / d);
    r = cur % d;
  }
  hi = ((u64)limb[0] << 32) | limb[1];
  lo = ((u64)limb[2] << 32) | limb[3];
}

// C(n, r) for n <= 1024 and r <= 16, filled once per device by
// k_fill_binom (entry (0, 0) = 1 marks it filled): a closed form then costs a
// load instead of r 128-bit multiply-divides.
constexpr int kBinomN = 1024;
constexpr int kBinomR = 16;
__device__ u64 g_binom[(kBinomN + 1) * (kBinomR + 1) * 2];

// C(n, r) as 128 bits; false if it may not fit (then nothing is claimed).
__device__ __forceinline__ bool binom128(int n, int r, u64& lo, u64& hi) {
  if (r >= 0 && r <= kBinomR && n >= 0 && n <= kBinomN && g_binom[0] == 1ull) {
    const u64* e = g_binom + ((size_t)n * (kBinomR + 1) + (size_t)r) * 2;
    lo = e[0];
    hi = e[1];
    return true;
  }
  lo = 1;
  hi = 0;
  for (int i = 0; i < r; ++i) {
    const u64 m = (u64)(n - i);  // < 2^11
    if (hi >> 52) return false;
    // (hi:lo) * m
    const u64 plo = lo * m;
    const u64 carry = __umul64hi(lo, m);
    hi = hi * m + carry;
    lo = plo;
    div_small(hi, lo, (u64)(i + 1));
  }
  return true;
}

// Row n of the table: C(n, r) for r = 0..kBinomR by C(n, r) = C(n, r-1) (n-r+1) / r
// (exact; C(1024, 16) < 2^117).
__global__ void k_fill_binom() {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n > kBinomN) return;
  u64 lo = 1, hi = 0;
  for (int r = 0; r <= kBinomR; ++r) {
    if (r > n) {
      lo = 0;
      hi = 0;
    } else if (r > 0) {
      const u64 m = (u64)(n - r + 1);
      const u64 plo = lo * m;
      hi = hi * m + __umul64hi(lo, m);
      lo = plo;
      div_small(hi, lo, (u64)r);
    }
    g_binom[((size_t)n * (kBinomR + 1) + (size_t)r) * 2] = lo;
    g_binom[((size_t)n * (kBinomR + 1) + (size_t)r) * 2 + 1] = hi;
  }
}

// e_j of the weights of the np members of P for j = 0..l (wave-collective):
// lane j holds e_j while the members are added one at a time.  Used where l
// exceeds kEsymMaxL.
__device__ __forceinline__ u64 esym_serial(const uint16_t* mem_, int np, const u64* gl_, int l) {
  const auto* mem = as_lds(mem_);
  const auto* gl = as_lds(gl_);
  const int lane = lane_id();
  u64 e = lane == 0 ? 1ull : 0ull;
  for (int i = 0; i < np; ++i) {
    const u64 g = gl[mem[i]];
    const u64 prev = __shfl_up(e, 1);
    if (lane >= 1 && lane <= l) e = addp(e, mulp(prev, g));
  }
  return e;
}

// The same by Newton's identities: with the power sums p_m = sum_x g(x)^m,
//   j e_j = sum_{i=1..j} (-1)^(i-1) e_{j-i} p_i,
// and j is invertible mod the prime p.  Every lane adds the powers of its own
// members, the wave sums each p_m, and the e_j follow in l^2 / 2 products, so
// no step waits on the previous member.
constexpr int kEsymMaxL = 16;

constexpr u64 mulp_host(u64 a, u64 b) { return (u64)((unsigned __int128)a * b % DIST_P61); }
constexpr u64 powp_host(u64 b, u64 e) {
  u64 r = 1;
  while (e) {
    if (e & 1) r = mulp_host(r, b);
    b = mulp_host(b, b);
    e >>= 1;
  }
  return r;
}
// inverses of 1..kEsymMaxL mod p (Fermat: j^(p-2)), evaluated by the compiler
struct InvSmall {
  u64 v[kEsymMaxL + 1];
};
constexpr InvSmall make_inv_small() {
  InvSmall t{};
  for (int j = 1; j <= kEsymMaxL; ++j) t.v[j] = powp_host((u64)j, DIST_P61 - 2);
  return t;
}
constexpr InvSmall kInvSmall = make_inv_small();
// the same, in constant memory for a loop index
__constant__ u64 c_inv_small[kEsymMaxL + 1] = {
    kInvSmall.v[0],  kInvSmall.v[1],  kInvSmall.v[2],  kInvSmall.v[3],  kInvSmall.v[4],  kInvSmall.v[5],
    kInvSmall.v[6],  kInvSmall.v[7],  kInvSmall.v[8],  kInvSmall.v[9],  kInvSmall.v[10], kInvSmall.v[11],
    kInvSmall.v[12], kInvSmall.v[13], kInvSmall.v[14], kInvSmall.v[15], kInvSmall.v[16]};

// Not inlined, and its loops are not unrolled: it is called at most search
// frames, so it has to stay small in the instruction cache.  Lane j returns
// e_j (j <= l), the rest 0.  A lane holds at most W members (np <= 64 W);
// lane m keeps p_m, lane j keeps e_j, and the products of the identities take
// their factors from other lanes by readlane (uniform loop indices).
template <int W>
__device__ __noinline__ u64 esym_lanes(const uint16_t* mem_, int np, const u64* gl_, int l) {
  if (l > kEsymMaxL) return esym_serial(mem_, np, gl_, l);
  const auto* mem = as_lds(mem_);
  const auto* gl = as_lds(gl_);
  const int lane = lane_id();
  u64 g[W], pw[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int i = lane + t * kWave;
    g[t] = i < np ? gl[mem[i]] : 0ull;
    pw[t] = g[t];
  }
  const int nt = (np + kWave - 1) / kWave;  // slots in use (uniform)
  u64 pl = 0;                               // lane m: p_m
#pragma unroll 1
  for (int m = 1; m <= l; ++m) {
    u64 acc = pw[0];
    pw[0] = mulp(pw[0], g[0]);
#pragma unroll
    for (int t = 1; t < W; ++t) {
      if (t < nt) {
        acc = addp(acc, pw[t]);
        pw[t] = mulp(pw[t], g[t]);
      }
    }
    acc = wave_sum_p(acc);
    if (lane == m) pl = acc;
  }
  u64 el = lane == 0 ? 1ull : 0ull;  // lane j: e_j
#pragma unroll 1
  for (int j = 1; j <= l; ++j) {
    u64 pos = 0, neg = 0;
#pragma unroll 1
    for (int i = 1; i <= j; ++i) {
      const u64 t = mulp(readlane64(el, j - i), readlane64(pl, i));
      if (i & 1) pos = addp(pos, t);
      else neg = addp(neg, t);
    }
    const u64 ej = mulp(subp(pos, neg), c_inv_small[j]);
    if (lane == j) el = ej;
  }
  return el;
}

// e_l of the weights of the np members of P (wave-collective).
template <int W>
__device__ __forceinline__ u64 esym_members(const uint16_t* mem, int np, const u64* gl, int l) {
  return __shfl(esym_lanes<W>(mem, np, gl, l), l);
}

// Nearly complete candidate sets: if G[P] misses e <= 8 edges, its l-cliques
// are the l-subsets of P containing none of them; by inclusion-exclusion over
// the subsets S of the missing edges, with V(S) the endpoints of S,
//   count = sum_S (-1)^|S| C(|P| - |V(S)|, l - |V(S)|),
//   fp    = sum_S (-1)^|S| prod_{v in V(S)} g(v) e_{l-|V(S)|}(g(P \ V(S))),
// since the l-subsets containing V(S) are V(S) plus an (l - |V(S)|)-subset of
// the rest.  Lanes take the 2^e subsets in turn.  Exact.
constexpr int kNearMissing = 8;
// The fingerprint form keeps l + 1 coefficients per lane: l <= kNearFpL.
constexpr int kNearFpL = 15;

__device__ __forceinline__ void wave_sum128(u64& lo, u64& hi) {
  for (int off = 32; off > 0; off >>= 1) {
    const u64 lo2 = __shfl_xor(lo, off), hi2 = __shfl_xor(hi, off);
    const u64 nlo = lo + lo2;
    hi = hi + hi2 + (nlo < lo ? 1ull : 0ull);
    lo = nlo;
  }
}

// Not inlined: its three callers (the leaf counter, leaf frames, and frames
// with l >= 4) would otherwise push the search kernel past 256 VGPRs.
// pairs: the e missing edges as local-id pairs (2e entries) in LDS.  Only
// |V(S)| varies between count terms, so lanes 0..16 first compute the
// binomials C(|P| - v, l - v) for every possible v; a term is then a lookup.
// With FP, e_{l - v}(P \ V(S)) comes from the coefficients of
// prod_{x in P} (1 + g(x) t) (mem, gl: the members and their weights) divided
// by (1 + g(v) t) for each v in V(S): q_0 = 1, q_j = f_j - g(v) q_{j-1}.
// The result comes back by value (in registers, not through the stack).
struct Closed {
  u64 lo, hi, fp;
  bool ok;
};

template <int W, bool FP>
__device__ __noinline__ Closed near_complete_impl(const uint16_t* pairs_, int e, int np, int l, const uint16_t* mem,
                                                  const u64* gl_) {
  const auto* pairs = as_lds(pairs_);
  const auto* gl = as_lds(gl_);
  const int lane = lane_id();
  Closed r{0, 0, 0, false};
  if (FP && l > kNearFpL) return r;
  // distinct endpoints: lane t < 2e holds the t-th endpoint; idx numbers the
  // distinct ones in order of first appearance
  const int a = lane < 2 * e ? (int)pairs[lane] : -1;
  int first = lane;
  for (int t = 2 * e - 1; t >= 0; --t) {
    const int b = __shfl(a, t);
    if (t < lane && b == a) first = t;
  }
  const u64 firsts = __ballot(lane < 2 * e && first == lane);
  const int nv = __popcll(firsts);
  const int idx = __shfl(__popcll(firsts & lanemask_lt()), first);
  // endpoint masks of the missing edges, 16 bits each, four per word
  u64 em0 = 0, em1 = 0;
#pragma unroll
  for (int i = 0; i < kNearMissing; ++i) {
    const int i0 = __shfl(idx, 2 * i), i1 = __shfl(idx, 2 * i + 1);
    const u64 m = i < e ? (u64)((1u << i0) | (1u << i1)) : 0ull;
    if (i < 4) em0 |= m << (16 * i);
    else em1 |= m << (16 * (i - 4));
  }
  // lane v <= nv: C(np - v, l - v)
  u64 cvlo = 0, cvhi = 0;
  bool ok = true;
  if (lane <= nv && lane <= l) ok = binom128(np - lane, l - lane, cvlo, cvhi);
  if (__ballot(!ok)) return r;
  // fingerprint: lane j holds the coefficient f_j = e_j(g(P)) and lane i the
  // weight of the i-th distinct endpoint; read back with readlane (uniform
  // lane numbers), so only the quotient stays in registers per lane
  u64 ep = 0, gyl = 0;
  if constexpr (FP) {
    ep = esym_lanes<W>(mem, np, gl_, l);
    const u64 wt = lane < 2 * e ? gl[a] : 0ull;
    u64 fb = firsts;
    for (int i = 0; i < nv; ++i) {
      const int t = __ffsll((unsigned long long)fb) - 1;
      fb &= fb - 1;
      const u64 gi = __shfl(wt, t);
      if (lane == i) gyl = gi;
    }
  }
  u64 plo = 0, phi = 0, nlo = 0, nhi = 0;  // positive and negative count terms
  u64 fpos = 0, fneg = 0;                  // and fingerprint terms
  const int ns = 1 << e;
  for (int base = 0; base < ns; base += kWave) {
    const int S = base + lane;
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kNearMissing; ++i)
      if ((S >> i) & 1) m |= (uint32_t)(((i < 4 ? em0 : em1) >> (16 * (i & 3))) & 0xffffull);
    const int v = __popc(m);
    const u64 clo = __shfl(cvlo, v), chi = __shfl(cvhi, v);
    if (S < ns) {
      const bool neg = __popc((unsigned)S) & 1;
      if (neg) {
        const u64 t = nlo + clo;
        nhi += chi + (t < nlo ? 1ull : 0ull);
        nlo = t;
      } else {
        const u64 t = plo + clo;
        phi += chi + (t < plo ? 1ull : 0ull);
        plo = t;
      }
      if constexpr (FP) {
        if (v <= l) {
          u64 q[kNearFpL + 1];
#pragma unroll
          for (int j = 0; j <= kNearFpL; ++j) q[j] = j <= l ? readlane64(ep, j) : 0ull;
          u64 gprod = 1;
#pragma unroll 1
          for (int i = 0; i < nv; ++i) {
            const u64 gi = readlane64(gyl, i);  // uniform i: read even where lanes diverge
            if ((m >> i) & 1u) {
              gprod = mulp(gprod, gi);
#pragma unroll
              for (int j = 1; j <= kNearFpL; ++j)
                if (j <= l) q[j] = subp(q[j], mulp(gi, q[j - 1]));
            }
          }
          u64 c = 0;
#pragma unroll
          for (int j = 0; j <= kNearFpL; ++j)
            if (j == l - v) c = q[j];
          const u64 term = mulp(gprod, c);
          if (neg) fneg = addp(fneg, term);
          else fpos = addp(fpos, term);
        }
      }
    }
  }
  wave_sum128(plo, phi);
  wave_sum128(nlo, nhi);
  r.lo = plo - nlo;
  r.hi = phi - nhi - (plo < nlo ? 1ull : 0ull);
  r.fp = FP ? subp(wave_sum_p(fpos), wave_sum_p(fneg)) : 0ull;
  r.ok = true;
  return r;
}

template <int W, bool FP>
__device__ __forceinline__ bool near_complete(const uint16_t* pairs, int e, int np, int l, const uint16_t* mem,
                                              const u64* gl, u64& lo, u64& hi, u64& fp) {
  const Closed r = near_complete_impl<W, FP>(pairs, e, np, l, mem, gl);
  lo = r.lo;
  hi = r.hi;
  fp = r.fp;
  return r.ok;
}

// Collects the missing edges of G[P] (members mem[0..np), candidate words Pr)
// into pairs (at most kNearMissing are stored); returns how many there are.
template <int W>
__device__ __forceinline__ int missing_edges(const Lds& s, const u64 (&Pr)[W], int np, uint16_t* pairs) {
  const int lane = lane_id();
  int base = 0;
  for (int b0 = 0; b0 < np; b0 += kWave) {
    const int i = b0 + lane;
    int c = 0;
    int x = 0;
    if (i < np) {
      x = s.mem[i];
#pragma unroll
      for (int w = 0; w < W; ++w) c += __popcll(Pr[w] & cut_mask(x + 1, w) & ~s.A[x * W + w]);
    }
    int incl = c;
    for (int off = 1; off < kWave; off <<= 1) {
      const int t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    int o = base + incl - c;
    if (c) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 b = Pr[w] & cut_mask(x + 1, w) & ~s.A[x * W + w];
        while (b) {
          const int t = __ffsll((unsigned long long)b) - 1;
          b &= b - 1;
          if (o < kNearMissing) {
            pairs[2 * o] = (uint16_t)x;
            pairs[2 * o + 1] = (uint16_t)(w * 64 + t);
          }
          ++o;
        }
      }
    }
    base += __shfl(incl, kWave - 1);
  }
  __syncthreads();
  return base;
}

// The 3-cliques of G[P] (a leaf frame, l = 3) and their fingerprint sum, with
// the members of P in s.mem: the edges of G[P] are counted first, so that a
// complete or nearly complete P takes its closed form; otherwise each member x
// counts the edges among its forward neighbours P & A[x].  Wave-collective.
template <int W, bool FP>
__device__ __forceinline__ void leaf3_count(const Lds& s, const u64 (&Pr)[W], int np, u64& lo, u64& hi, u64& fp,
                                            u64& wops, u64& bits) {
  const int lane = lane_id();
  u64 m = 0;
  for (int i = lane; i < np; i += kWave) {
    const int x = s.mem[i];
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += __popcll(Pr[w] & s.A[x * W + w]);
    m += (u64)c;
  }
  wops += (u64)((np + kWave - 1 - lane) / kWave) * W;
  m = wave_sum(m);
  const u64 full = (u64)np * (u64)(np - 1) / 2;
  u64 clo, chi, cfp;
  if (m < full && full - m <= (u64)kNearMissing) {
    const int e = missing_edges<W>(s, Pr, np, s.pos);
    if (e == (int)(full - m) && near_complete<W, FP>(s.pos, e, np, 3, s.mem, s.gl, clo, chi, cfp)) {
      lo = clo;
      hi = chi;
      fp = cfp;
      return;
    }
  }
  if (m == full && binom128(np, 3, clo, chi)) {
    lo = clo;
    hi = chi;
    fp = FP ? esym_members<W>(s.mem, np, s.gl, 3) : 0;
    return;
  }
  u64 c_acc = 0, f_acc = 0;
  for (int i = lane; i < np; i += kWave) {
    const int x = s.mem[i];
    u64 q[W];
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      q[w] = Pr[w] & s.A[x * W + w];
      c += __popcll(q[w]);
    }
    wops += W;
    if (c >= 2 && s.rcap[x] >= 3) {
      u64 ec = 0, ef = 0;
      edges_in<W>(q, s.A, s.gl, s.wtab, FP, ec, ef, wops, bits);
      c_acc += ec;
      if (FP && ec) f_acc = addp(f_acc, mulp(s.gl[x], ef));
    }
  }
  lo = wave_sum(c_acc);
  hi = 0;
  fp = FP ? wave_sum_p(f_acc) : 0;
}

// Children x of a frame (the bits of Q) whose child frames need L vertices
// (3 <= L <= kLaneEsymMaxL) and whose sets c = P & A[x] are complete or miss
// at most two edges, one child per lane instead of a frame each.  A lane
// lists the missing edges of G[c] (its test stops at a third).  By
// inclusion-exclusion over the subsets S of the missing edges, with V(S)
// their endpoints, c holds
//   sum_S (-1)^|S| C(n - |V(S)|, L - |V(S)|)
// L-cliques, with fingerprint sum
//   sum_S (-1)^|S| prod_{v in V(S)} g(v) e_{L-|V(S)|}(c \ V(S)),
// where the polynomial prod_{v in c} (1 + g(v) t) is built member by member
// (e_t += e_{t-1} g) and divided by (1 + g(v) t) for each v in V(S).  Such
// children leave Q; with count = false (the children of a unit's root frame
// that are shared split frames, outside sub-unit 0) they add nothing, as
// their own frames would.  A set whose binomials do not fit 128 bits stays
// in Q.  s.pos is scratch.
constexpr int kLaneEsymMaxL = 8;

struct ChildSum {
  u64 lo, hi, fp, wops;
};

// C(n, r) as 128 bits (0 outside 0 <= r <= n); false if it does not fit.
__device__ __forceinline__ bool binom_or_zero(int n, int r, u64& lo, u64& hi) {
  if (r < 0 || r > n) {
    lo = hi = 0;
    return true;
  }
  return binom128(n, r, lo, hi);
}

// e_r of (prod over c of (1 + g t)) / prod over the nv removed vertices
// (weights v0..v3) of (1 + g(v) t), the quotient taken on a copy of the
// coefficients.  Values, not arrays, so that everything stays in registers.
__device__ __forceinline__ u64 quotient_coef(const u64 (&e)[kLaneEsymMaxL + 1], u64 v0, u64 v1, u64 v2, u64 v3,
                                             int nv, int L, int r) {
  u64 q[kLaneEsymMaxL + 1];
#pragma unroll
  for (int t = 0; t <= kLaneEsymMaxL; ++t) q[t] = e[t];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < nv) {
      const u64 g = i == 0 ? v0 : i == 1 ? v1 : i == 2 ? v2 : v3;
#pragma unroll
      for (int t = 1; t <= kLaneEsymMaxL; ++t)
        if (t <= L) q[t] = subp(q[t], mulp(g, q[t - 1]));
    }
  }
  u64 out = 0;
#pragma unroll
  for (int t = 0; t <= kLaneEsymMaxL; ++t)
    if (t == r) out = q[t];
  return out;
}

template <int W, bool FP>
__device__ __noinline__ ChildSum complete_children(const Lds& s, u64* Q, const u64* P_, int L, bool count) {
  const auto* A = as_lds(s.A);
  const auto* gl = as_lds(s.gl);
  const auto* P = as_lds(P_);
  const auto* Qr = as_lds(Q);
  const int lane = lane_id();
  u64 Pr[W];
#pragma unroll
  for (int w = 0; w < W; ++w) Pr[w] = P[w];
  int nq = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 bw = Qr[w];
    if ((bw >> lane) & 1ull) s.pos[nq + __popcll(bw & lanemask_lt())] = (uint16_t)(w * 64 + lane);
    nq += __popcll(bw);
  }
  __syncthreads();
  u64 lo = 0, hi = 0, fp = 0, wops = 0;
  for (int i0 = 0; i0 < nq; i0 += kWave) {
    const int i = i0 + lane;
    if (i >= nq) continue;
    const int x = s.pos[i];
    u64 c[W];
    int n = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      c[w] = Pr[w] & A[x * W + w];
      n += __popcll(c[w]);
    }
    wops += W;
    // the missing edges (y, z), y < z, of G[c]: at most two are kept
    int miss = 0, a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    int above = n;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      u64 b = c[w];
      while (b && miss <= 2) {
        const int y = w * 64 + __ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        --above;
        int cy = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) cy += __popcll(c[v] & A[y * W + v]);
        wops += W;
        if (cy == above) continue;
#pragma unroll
        for (int v = 0; v < W; ++v) {
          u64 mz = c[v] & cut_mask(y + 1, v) & ~A[y * W + v];
          while (mz && miss <= 2) {
            const int z = v * 64 + __ffsll((unsigned long long)mz) - 1;
            mz &= mz - 1;
            if (miss == 0) {
              a0 = y;
              b0 = z;
            } else if (miss == 1) {
              a1 = y;
              b1 = z;
            }
            ++miss;
          }
        }
      }
    }
    if (miss > 2) continue;
    // endpoints of both edges (3 if they share one, else 4)
    const int nv2 = 4 - (a1 == a0 || a1 == b0) - (b1 == a0 || b1 == b0);
    u64 c0l, c0h, c1l = 0, c1h = 0, c2l = 0, c2h = 0;
    // the same test in every unit that shares the frame
    if (!binom_or_zero(n, L, c0l, c0h)) continue;
    if (miss >= 1 && !binom_or_zero(n - 2, L - 2, c1l, c1h)) continue;
    if (miss == 2 && !binom_or_zero(n - nv2, L - nv2, c2l, c2h)) continue;
    if (count) {
      // c0 - miss * c1 + [miss == 2] c2 (never negative)
      u64 tl = c0l, th = c0h;
      for (int m = 0; m < miss; ++m) {
        th -= c1h + (tl < c1l ? 1ull : 0ull);
        tl -= c1l;
      }
      if (miss == 2) {
        const u64 nl = tl + c2l;
        th += c2h + (nl < tl ? 1ull : 0ull);
        tl = nl;
      }
      const u64 nlo = lo + tl;
      hi += th + (nlo < lo ? 1ull : 0ull);
      lo = nlo;
      if (FP) {
        u64 e[kLaneEsymMaxL + 1];
        e[0] = 1;
#pragma unroll
        for (int t = 1; t <= kLaneEsymMaxL; ++t) e[t] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          u64 b = c[w];
          while (b) {
            const int y = w * 64 + __ffsll((unsigned long long)b) - 1;
            b &= b - 1;
            const u64 g = gl[y];
#pragma unroll
            for (int t = kLaneEsymMaxL; t >= 2; --t)
              if (t <= L) e[t] = addp(e[t], mulp(e[t - 1], g));
            e[1] = addp(e[1], g);
          }
        }
        u64 f = 0;
#pragma unroll
        for (int t = 1; t <= kLaneEsymMaxL; ++t)
          if (t == L) f = e[t];
        const u64 ga0 = gl[a0], gb0 = gl[b0];
        if (miss >= 1) f = subp(f, mulp(mulp(ga0, gb0), quotient_coef(e, ga0, gb0, 0, 0, 2, L, L - 2)));
        if (miss == 2) {
          const u64 ga1 = gl[a1], gb1 = gl[b1];
          f = subp(f, mulp(mulp(ga1, gb1), quotient_coef(e, ga1, gb1, 0, 0, 2, L, L - 2)));
          // both edges: their distinct endpoints (a shared one once)
          const bool na = a1 != a0 && a1 != b0, nb = b1 != a0 && b1 != b0;
          const u64 w2 = na ? ga1 : gb1, w3 = gb1;  // the new endpoints, in order
          const u64 pv = mulp(mulp(ga0, gb0), mulp(na ? ga1 : 1ull, nb ? gb1 : 1ull));
          f = addp(f, mulp(pv, L - nv2 >= 0 ? quotient_coef(e, ga0, gb0, w2, w3, nv2, L, L - nv2) : 0ull));
        }
        fp = addp(fp, mulp(gl[x], f));
      }
    }
    atomicAnd((unsigned long long*)&Q[x >> 6], ~(1ull << (x & 63)));
  }
  __syncthreads();
  wave_sum128(lo, hi);
  return ChildSum{lo, hi, FP ? wave_sum_p(fp) : 0ull, wops};
}

// ---- the kernel ----------------------------------------------------------------

// Counting kernels of up to 6 words are held to 256 VGPRs, i.e. two waves per
// SIMD (the register file holds 512 per lane): crossing it halves occupancy.
template <int W, bool FP>
__global__ __launch_bounds__(64, (W <= 6 ? 2 : 1)) void k_search(Params p) {
  extern __shared__ __align__(16) char smem[];
  const int lane = lane_id();
  int k = p.k;  // batch mode: the largest k of the launch (sizes the stacks)
  int memo_mode = p.memo;  // batch mode: the unit's pair's
  const Lds s = carve<W>(smem, p.k, FP, p.drows);
  const u64 ES = p.tau ? (u64)kShES : (u64)(W + 4);  // entry words
  u64* table = p.memo_base ? p.memo_base + (u64)blockIdx.x * (p.memo_mask + 1) * ES : nullptr;

  // per-wave totals (uniform) and per-lane counters
  u64 tot_lo = 0, tot_hi = 0, tot_fp = 0;
  u64 n_units = 0, n_builds = 0, n_pruned = 0, n_frames = 0, n_look = 0, n_hit = 0, n_ins = 0;
  u64 wops = 0, bits = 0, arcs = 0;
  bool aborted = false;
  const u64 t_start = wall_clock64();
  const u64 deadline = p.deadline ? t_start + p.deadline : 0;
  u64 pair_budget = 0;
  u64 pair_deadline = 0;
  int own_clock = 0;
  const u64 tag0 = p.tag_base + (p.epoch ? __hip_atomic_load(p.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull);

  int cur_rel = -1;       // root whose G_u is in LDS
  int cur_pair = -1;
  // shared memo state, in LDS (it is used once per unit or memo call):
  // ctl[0] the wave's clear tag (~0: none yet), ctl[1] the inserts counted at
  // its last clear, ctl[2] the wave's run of units (next | end << 32),
  // ctl[3] the root's first arc (its out-neighbour list maps a memo key's
  // local ids to ranks)
  if (lane == 0) {
    s.ctl[0] = ~0ull;
    s.ctl[1] = 0;
    s.ctl[2] = 0;
    s.ctl[3] = 0;
  }
  __syncthreads();
  auto room = [&]() { return !p.tau || n_ins - s.ctl[1] < 2 * p.tau; };  // hard bound 2 tau
  bool cur_pruned = false;
  const int32_t* Gdptr = nullptr;
  const int32_t* Gdcol = nullptr;
  const int32_t* Gorig = nullptr;
  const int32_t* Groots = nullptr;
  const u64* Ggw = nullptr;
  const EdgeRec* Gedges = nullptr;
  const u64* Gerows = nullptr;
  int pair = -1;
  int32_t r = 0;
  int d = 0;
  u64 rw = 0;  // weight of the unit's prefix: g(root), or g(u) g(v) for an edge
  for (;;) {
    // ---- 0. next work unit: (root, range of depth-1 children) -------------------
    uint32_t u = 0;
    if (p.chunk > 1) {
      // runs of consecutive units (consecutive roots), so that a shared memo
      // sees neighbouring roots one after another
      const u64 run = s.ctl[2];
      uint32_t u_next = (uint32_t)run, u_end = (uint32_t)(run >> 32);
      if (u_next >= u_end) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(p.cursor, p.chunk);
        b = __shfl(b, 0);
        u_next = b;
        u_end = b + p.chunk;
      }
      u = u_next++;
      __syncthreads();
      if (lane == 0) s.ctl[2] = ((u64)u_end << 32) | u_next;
      __syncthreads();
    } else {
      if (lane == 0) u = atomicAdd(p.cursor, 1u);
      u = __shfl(u, 0);
    }
    if (u >= p.units) break;
    // segment: consecutive roots of one (graph, k) pair, upr units each
    int lo = 0, hi = p.nsegs - 1;  // largest segment with unit_begin <= u
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (p.segs[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
    }
    const BatchSeg sg = p.segs[lo];
    pair = sg.pair;
    const uint32_t off = u - sg.unit_begin;
    const int rel = sg.a + (int)(off / (uint32_t)sg.upr);
    const int upr = sg.upr;
    // a root's units: upr / nsub ranges of depth-1 children, each split into
    // nsub units that take every nsub-th surviving depth-2 child
    const int nsub = sg.sub;
    const int ci = (int)(off % (uint32_t)upr) / nsub;
    const int sub = (int)(off % (uint32_t)upr) % nsub;
    {
      const BatchGraph bgr = p.bg[pair];
      Gdptr = bgr.dptr;
      Gdcol = bgr.dcol;
      Gorig = bgr.orig;
      Groots = bgr.roots;
      Ggw = bgr.gw;
      Gedges = bgr.edges;
      Gerows = bgr.erows;
      k = bgr.k;
      pair_budget = bgr.budget;
      own_clock = bgr.own_clock;
      memo_mode = bgr.memo >= 0 ? bgr.memo : p.memo;
    }
    pair_deadline = 0;
    if (p.pair_t0) {
      // first-unit times of the pair and of the batch; a budget runs from one
      // of them
      u64 tp = 0, tb = 0;
      if (lane == 0) {
        const u64 now = wall_clock64();
        tp = first_time(p.pair_t0 + 1 + pair, now);
        if (pair_budget && !own_clock) tb = first_time(p.pair_t0, now);
      }
      tp = __shfl(tp, 0);
      tb = __shfl(tb, 0);
      if (pair_budget) pair_deadline = (own_clock ? tp : tb) + pair_budget;
    }
    if (p.pair_abort) {
      // a pair out of budget: its remaining units are skipped
      int ab = __hip_atomic_load(p.pair_abort + pair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!ab && pair_deadline && wall_clock64() > pair_deadline) {
        if (lane == 0) atomicOr(p.pair_abort + pair, 1);
        ab = 1;
      }
      if (ab) {
        finish_units(p, pair, 1u + skip_rest(p, sg.pair_end));
        continue;
      }
    }
    if (__hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      aborted = true;
      break;
    }
    if (deadline && wall_clock64() > deadline) {
      if (lane == 0) atomicOr(p.abort_flag, 1);
      aborted = true;
      break;
    }
    const int ridx = rel;
    // one tag per root (its first unit): chunks of a root share memo entries
    const u64 root_tag = tag0 + (u64)sg.unit_begin + (u64)(off / (uint32_t)upr) * (u64)upr;
    ++n_units;
    if (p.tau && (s.ctl[0] == ~0ull || pair != cur_pair || (rel != cur_rel && n_ins - s.ctl[1] > p.tau))) {
      // a new root past the soft bound tau (or a new graph): the shared memo
      // starts empty (entries of earlier clear tags never match)
      __syncthreads();
      if (lane == 0) {
        s.ctl[0] = root_tag;
        s.ctl[1] = n_ins;
      }
      __syncthreads();
    }
    const u64 mtag = p.tau ? s.ctl[0] : root_tag;

    if (rel != cur_rel || pair != cur_pair) {
      cur_rel = rel;
      cur_pair = pair;
      __syncthreads();
      int32_t beg;
      if (Gedges) {
        // an EdgeParallel unit: the vertices of G[N+(u) & N+(v)] from the
        // set bits of its row over N+(u)
        const EdgeRec er = Gedges[Groots[ridx]];
        r = er.u;
        beg = Gdptr[r];
        d = er.d;  // <= 64 * W by the host's bucketing
        rw = FP ? mulp(Ggw[er.u], Ggw[er.v]) : 0;
        const u64* row = Gerows + er.row;
        int nbase = 0;
        for (int w = 0; w < er.wu; ++w) {
          const u64 bw = row[w];
          if ((bw >> lane) & 1ull) s.nb[nbase + __popcll(bw & lanemask_lt())] = Gdcol[beg + w * 64 + lane];
          nbase += __popcll(bw);
        }
      } else {
        r = Groots[ridx];
        beg = Gdptr[r];
        d = Gdptr[r + 1] - beg;  // <= 64 * W by the host's bucketing
        rw = FP ? Ggw[r] : 0;
        for (int i = lane; i < d; i += kWave) s.nb[i] = Gdcol[beg + i];
      }
      if (lane == 0) s.ctl[3] = (u64)(uint32_t)beg;
      __syncthreads();
      ++n_builds;
      // ---- 1. G_u (or G_uv) in LDS ---------------------------------------------
      arcs += build_rows<W>(s, Gdptr, Gdcol, Ggw, Gorig, nullptr, d);
      if (s.wtab) build_weight_table<W>(s, d);

      // ---- 2. soft-embedding bound (Algorithm 5) ---------------------------------
      if (p.soft_only) {
        int rr = soft_embed_levels<W>(s, d, k);
        if (lane == 0) p.soft_out[Gorig[r]] = rr;
        __syncthreads();
        cur_pruned = true;  // nothing to search in this mode
        continue;
      }
      cur_pruned = false;
      if (p.prune && k >= 3) {
        int rr = soft_embed_levels<W>(s, d, k);
        if (rr < k) cur_pruned = true;
      } else {
        for (int i = lane; i < d; i += kWave) s.rcap[i] = 63;
      }
      __syncthreads();
    }
    if (cur_pruned) {
      if (ci == 0 && sub == 0 && !p.soft_only) ++n_pruned;
      finish_units(p, pair, 1u);
      continue;
    }
    // children of frame 0 handled by this unit: local ids [x_lo, x_hi)
    const int ch = (d + upr / nsub - 1) / (upr / nsub);
    const int x_lo = ci * ch < d ? ci * ch : d;
    const int x_hi = x_lo + ch < d ? x_lo + ch : d;
    // with nsub > 1, frame 1 holds only part of its subtree: it neither reads
    // nor writes memo entries, and its closed forms count in sub-unit 0 only
    const int jsplit = nsub > 1 ? 1 : -1;
    // an edge unit's frame 0 (a depth-1 set of its root) takes the closed
    // forms too; all units of the edge reach the same decision, and the
    // first of them counts it
    const bool cf0 = Gedges != nullptr;
    const bool own0 = ci == 0 && sub == 0;

    // ---- 3. depth-first search over candidate bitmaps -----------------------------
    // frame j needs l = k-1-j more vertices from its candidate set stP[j].
    if (lane < W) {
      int lo_bit = lane * 64;
      u64 wv;
      if (d >= lo_bit + 64) wv = ~0ull;
      else if (d <= lo_bit) wv = 0ull;
      else wv = (1ull << (d - lo_bit)) - 1;
      s.stP[lane] = wv;
    }
    __syncthreads();

    int j = 0;
    enum { ENTER, NEXT, FINISH } mode = ENTER;
    u64 r_look = 0, r_hit = 0;  // this root's memo lookups and hits
    const u64 r_ins0 = n_ins;   // and inserts, from here
    // the same test over all of this wave's units so far: the roots of a
    // launch are alike, so a wave whose inserts went unanswered stops early
    bool memo_live = table != nullptr && memo_mode != 0 &&
                     !(n_ins >= kMemoWaveIns && n_hit * kMemoWaveRatio < n_ins);
    u64 res_lo = 0, res_hi = 0, res_fp = 0;
    bool stop = false, unit_cancel = false;
    while (true) {
      if (mode == ENTER) {
        ++n_frames;
        if ((deadline || pair_deadline) && (n_frames & 15) == 0) {
          const u64 now = wall_clock64();
          if (deadline && now > deadline) {
            if (lane == 0) atomicOr(p.abort_flag, 1);
            stop = true;
            break;
          }
          if (pair_deadline && now > pair_deadline && p.pair_abort) {
            if (lane == 0) atomicOr(p.pair_abort + pair, 1);
            unit_cancel = true;
            break;
          }
        }
        const int l = k - 1 - j;
        const u64* P = s.stP + j * W;
        u64 Pr[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Pr[w] = P[w];
        if (l == 1) {
          u64 c = 0;
#pragma unroll
          for (int w = 0; w < W; ++w) c += __popcll(Pr[w]);
          u64 f = 0;
          if (FP) {
            u64 tmpb = 0;
            f = weight_sum_any<W>(Pr, s.gl, s.wtab, tmpb);
            bits += (lane == 0) ? tmpb : 0;
          }
          res_lo = c; res_hi = 0; res_fp = f;
          mode = FINISH;
          continue;
        }
        bool memo_j = false;
        if (memo_mode == 2) memo_j = (l >= 3);
        else if (memo_mode == 1) memo_j = (l >= 3) && j > 0 && s.stMemo[j - 1];
        const u64 tag = (mtag << 8) | (u64)l;
        if (memo_j && memo_live && j > 0 && j != jsplit) {
          ++n_look;
          ++r_look;
          u64 a, b, c;
          if (memo_find<W>(p, table, tag, s.stP + j * W, nullptr, 1, a, b, c, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr) >= 0) {
            ++n_hit;
            ++r_hit;
            res_lo = a; res_hi = b; res_fp = c;
            mode = FINISH;
            continue;
          }
          if ((r_look >= kMemoMinLook && r_hit * kMemoMinRatio < r_look) ||
              (n_ins - r_ins0 >= kMemoMinLook && r_hit * kMemoMinInsRatio < n_ins - r_ins0))
            memo_live = false;
        }
        // members of P
        int np = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          u64 bw = Pr[w];
          if ((bw >> lane) & 1ull) s.mem[np + __popcll(bw & lanemask_lt())] = (uint16_t)(w * 64 + lane);
          np += __popcll(bw);
        }
        __syncthreads();
        if (l == 2 || l == 3) {
          if (j == jsplit && sub != 0) {
            // a leaf frame is not shared out: sub-unit 0 takes all of it
            res_lo = res_hi = res_fp = 0;
            mode = FINISH;
            continue;
          }
          if (l == 3 && (j > 0 || cf0)) {
            // edges of G[P] first: a complete P needs no leaf search
            u64 m = 0;
            for (int i = lane; i < np; i += kWave) {
              const int x = s.mem[i];
              int c = 0;
#pragma unroll
              for (int w = 0; w < W; ++w) c += __popcll(Pr[w] & s.A[x * W + w]);
              m += (u64)c;
            }
            wops += (u64)((np + kWave - 1 - lane) / kWave) * W;
            m = wave_sum(m);
            u64 clo, chi;
            {
              const u64 full = (u64)np * (u64)(np - 1) / 2;
              if (m < full && full - m <= (u64)kNearMissing) {
                const int e = missing_edges<W>(s, Pr, np, s.pos);
                u64 cfp;
                if (e == (int)(full - m) && near_complete<W, FP>(s.pos, e, np, 3, s.mem, s.gl, clo, chi, cfp)) {
                  res_lo = clo;
                  res_hi = chi;
                  res_fp = cfp;
                  if (j == 0 && !own0) res_lo = res_hi = res_fp = 0;
                  if (memo_j && memo_live && j > 0) {
                    memo_put<W>(p, table, tag, s.stP + j * W, -1, res_lo, res_hi, res_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
                    ++n_ins;
                  }
                  __syncthreads();
                  mode = FINISH;
                  continue;
                }
              }
            }
            if (m == (u64)np * (u64)(np - 1) / 2 && binom128(np, 3, clo, chi)) {
              res_lo = clo;
              res_hi = chi;
              res_fp = FP ? esym_members<W>(s.mem, np, s.gl, 3) : 0;
              if (j == 0 && !own0) res_lo = res_hi = res_fp = 0;
              if (memo_j && memo_live && j > 0) {
                memo_put<W>(p, table, tag, s.stP + j * W, -1, res_lo, res_hi, res_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
                ++n_ins;
              }
              __syncthreads();
              mode = FINISH;
              continue;
            }
          }
          u64 c_acc = 0, f_acc = 0;
          for (int base = 0; base < np; base += kWave) {
            int i = base + lane;
            bool act = i < np;
            int x = act ? s.mem[i] : 0;
            if (j == 0 && (x < x_lo || x >= x_hi)) act = false;
            u64 q[W];
            int c = 0;
            if (act) {
#pragma unroll
              for (int w = 0; w < W; ++w) {
                q[w] = Pr[w] & s.A[x * W + w];
                c += __popcll(q[w]);
              }
              wops += W;
              if (l == 2) {
                c_acc += (u64)c;
                if (FP && c) f_acc = addp(f_acc, mulp(s.gl[x], weight_sum_any<W>(q, s.gl, s.wtab, bits)));
              } else if (c >= 2 && s.rcap[x] >= 3) {
                u64 ec = 0, ef = 0;
                edges_in<W>(q, s.A, s.gl, s.wtab, FP, ec, ef, wops, bits);
                c_acc += ec;
                if (FP && ec) f_acc = addp(f_acc, mulp(s.gl[x], ef));
              }
            }
          }
          res_lo = wave_sum(c_acc);
          res_hi = 0;
          res_fp = FP ? wave_sum_p(f_acc) : 0;
          if (memo_j && memo_live && j > 0) memo_put<W>(p, table, tag, s.stP + j * W, -1, res_lo, res_hi, res_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
          if (memo_j && memo_live && j > 0) ++n_ins;
          __syncthreads();
          mode = FINISH;
          continue;
        }
        // l >= 4: evaluate children, collect survivors in stQ[j]
        u64* Q = s.stQ + j * W;
        if (lane < W) Q[lane] = 0;
        __syncthreads();
        u64 m_edges = 0;
        for (int base = 0; base < np; base += kWave) {
          int i = base + lane;
          if (i >= np) continue;
          int x = s.mem[i];
          int c = 0;
#pragma unroll
          for (int w = 0; w < W; ++w) c += __popcll(Pr[w] & s.A[x * W + w]);
          wops += W;
          m_edges += (u64)c;
          if (c >= l - 1 && s.rcap[x] >= l) atomicOr(&Q[x >> 6], 1ull << (x & 63));
        }
        m_edges = wave_sum(m_edges);
        if ((j > 0 || cf0) && m_edges == (u64)np * (u64)(np - 1) / 2) {
          u64 clo, chi;
          if (binom128(np, l, clo, chi)) {
            // at a shared split frame the closed form is sub-unit 0's: the
            // others skip it (and its fingerprint) entirely
            const bool mine = !(j == jsplit && sub != 0) && (j > 0 || own0);
            res_lo = mine ? clo : 0;
            res_hi = mine ? chi : 0;
            res_fp = (FP && mine) ? esym_members<W>(s.mem, np, s.gl, l) : 0;
            __syncthreads();
            mode = FINISH;
            continue;
          }
        }
        {
          const u64 full = (u64)np * (u64)(np - 1) / 2;
          if (j > 0 && j == jsplit && sub != 0 && m_edges < full && full - m_edges <= (u64)kNearMissing &&
              np <= kBinomN && l <= kBinomR && (!FP || l <= kNearFpL)) {
            // a nearly complete split frame whose closed form surely applies
            // (every binomial comes from the table): sub-unit 0's
            res_lo = res_hi = res_fp = 0;
            __syncthreads();
            mode = FINISH;
            continue;
          }
          if ((j > 0 || cf0) && m_edges < full && full - m_edges <= (u64)kNearMissing) {
            const int e = missing_edges<W>(s, Pr, np, s.pos);
            u64 clo, chi, cfp;
            if (e == (int)(full - m_edges) && near_complete<W, FP>(s.pos, e, np, l, s.mem, s.gl, clo, chi, cfp)) {
              res_lo = clo;
              res_hi = chi;
              res_fp = cfp;
              if ((j == jsplit && sub != 0) || (j == 0 && !own0)) res_lo = res_hi = res_fp = 0;
              __syncthreads();
              mode = FINISH;
              continue;
            }
          }
        }
        if (!memo_j && memo_mode == 1 && memo_live) {
          // criterion (1) in integer form: 2 m l > (l - 1) n^2
          u64 lhs = 2ull * m_edges * (u64)l;
          u64 rhs = (u64)(l - 1) * (u64)np * (u64)np;
          if (np >= 2 && lhs > rhs) {
            memo_j = true;
          }
          if (memo_j && j > 0 && j != jsplit) {
            ++n_look;
            ++r_look;
            u64 a, b, c;
            if (memo_find<W>(p, table, tag, s.stP + j * W, nullptr, 1, a, b, c, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr) >= 0) {
              ++n_hit;
              ++r_hit;
              res_lo = a; res_hi = b; res_fp = c;
              __syncthreads();
              mode = FINISH;
              continue;
            }
          }
        }
        u64 acc_lo = 0, acc_hi = 0, acc_fp = 0;
        __syncthreads();
        if (j == 0) {
          // this unit's share of the root's depth-1 children
          if (lane < W) {
            int lo_b = lane * 64;
            u64 m_lo = (x_lo <= lo_b) ? ~0ull : (x_lo >= lo_b + 64 ? 0ull : (~0ull << (x_lo - lo_b)));
            u64 m_hi = (x_hi <= lo_b) ? 0ull : (x_hi >= lo_b + 64 ? ~0ull : ((1ull << (x_hi - lo_b)) - 1));
            Q[lane] &= m_lo & m_hi;
          }
        }
        if (memo_j && memo_live && np >= 2 && j > 0 && j != jsplit) {
          // resume from the longest memoised proper prefix P & [m_i, inf),
          // m_i the i-th smallest member, i = 1..kMemoProbe, all probed at once
          const int ncut = np - 1 < kMemoProbe ? np - 1 : kMemoProbe;
          u64 a = 0, b = 0, c = 0;
          const int hi_ = memo_find<W>(p, table, tag, s.stP + j * W, s.mem + 1, ncut, a, b, c, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr);
          n_look += (u64)ncut;
          r_look += (u64)ncut;
          if (hi_ >= 0) {
            const int best = s.mem[1 + hi_];
            acc_lo = a;
            acc_hi = b;
            acc_fp = c;
            ++n_hit;
            ++r_hit;
            // children >= best are covered by the prefix
            if (lane < W) {
              int lo_b = lane * 64;
              u64 keep = (best <= lo_b) ? 0ull : (best >= lo_b + 64 ? ~0ull : ((1ull << (best - lo_b)) - 1));
              Q[lane] &= keep;
            }
          }
          if ((r_look >= kMemoMinLook && r_hit * kMemoMinRatio < r_look) ||
              (n_ins - r_ins0 >= kMemoMinLook && r_hit * kMemoMinInsRatio < n_ins - r_ins0))
            memo_live = false;
        }
        if (j == jsplit) {
          // this unit's share of frame 1's children: every nsub-th survivor
          // in ascending order, starting at the sub-th
          const int cnt = lane < W ? __popcll(Q[lane]) : 0;
          int incl = cnt;
          for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
          }
          if (lane < W) {
            u64 qw = Q[lane], keep = 0;
            int pos = incl - cnt;
            while (qw) {
              const int b = __ffsll((unsigned long long)qw) - 1;
              qw &= qw - 1;
              if (pos % nsub == sub) keep |= 1ull << b;
              ++pos;
            }
            Q[lane] = keep;
          }
        }
        {
          if (l == 4) {
            // the children are leaf frames (l = 3): counted here, highest
            // first, without a frame push each.  The memo is used exactly as
            // by child frames: a child's set is looked up and stored under
            // l = 3, and after each child the prefix P & [x, inf) under l = 4.
            const bool memo_c = memo_mode == 2 || (memo_mode == 1 && memo_j);
            const u64 ctag = (mtag << 8) | 3ull;
            __syncthreads();
            if (!(memo_j && memo_live && j > 0 && j != jsplit)) {
              // complete and nearly complete child sets first, one child per
              // lane; a frame that stores its prefixes in the memo keeps the
              // order
              const ChildSum cs = complete_children<W, FP>(s, Q, s.stP + j * W, 3, true);
              const u64 nlo = acc_lo + cs.lo;
              acc_hi += cs.hi + (nlo < acc_lo ? 1ull : 0ull);
              acc_lo = nlo;
              if (FP) acc_fp = addp(acc_fp, cs.fp);
              wops += cs.wops;
            }
            while (true) {
              int x = -1;
              for (int w = W - 1; w >= 0; --w) {
                const u64 qw = Q[w];
                if (qw) {
                  x = w * 64 + 63 - __clzll((long long)qw);
                  break;
                }
              }
              if (x < 0) break;
              ++n_frames;
              if ((deadline || pair_deadline) && (n_frames & 15) == 0) {
                const u64 now = wall_clock64();
                if (deadline && now > deadline) {
                  if (lane == 0) atomicOr(p.abort_flag, 1);
                  stop = true;
                  break;
                }
                if (pair_deadline && now > pair_deadline && p.pair_abort) {
                  if (lane == 0) atomicOr(p.pair_abort + pair, 1);
                  unit_cancel = true;
                  break;
                }
              }
              __syncthreads();
              if (lane == 0) Q[x >> 6] &= ~(1ull << (x & 63));
              u64* Pn = s.stP + (j + 1) * W;
              if (lane < W) Pn[lane] = s.stP[j * W + lane] & s.A[x * W + lane];
              __syncthreads();
              u64 clo = 0, chi = 0, cfp = 0;
              bool got = false;
              if (memo_c && memo_live) {
                ++n_look;
                ++r_look;
                if (memo_find<W>(p, table, ctag, Pn, nullptr, 1, clo, chi, cfp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr) >= 0) {
                  ++n_hit;
                  ++r_hit;
                  got = true;
                }
                if ((r_look >= kMemoMinLook && r_hit * kMemoMinRatio < r_look) ||
              (n_ins - r_ins0 >= kMemoMinLook && r_hit * kMemoMinInsRatio < n_ins - r_ins0))
            memo_live = false;
              }
              if (!got) {
                u64 Pc[W];
                int np2 = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                  Pc[w] = Pn[w];
                  const u64 bw = Pc[w];
                  if ((bw >> lane) & 1ull) s.mem[np2 + __popcll(bw & lanemask_lt())] = (uint16_t)(w * 64 + lane);
                  np2 += __popcll(bw);
                }
                __syncthreads();
                if (np2 >= 3) leaf3_count<W, FP>(s, Pc, np2, clo, chi, cfp, wops, bits);
                if (memo_c && memo_live) {
                  memo_put<W>(p, table, ctag, Pn, -1, clo, chi, cfp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
                  ++n_ins;
                }
              }
              const u64 nlo = acc_lo + clo;
              acc_hi += chi + (nlo < acc_lo ? 1ull : 0ull);
              acc_lo = nlo;
              if (FP) acc_fp = addp(acc_fp, mulp(s.gl[x], cfp));
              if (memo_j && memo_live && j > 0 && j != jsplit) {
                // trie node P & [x, inf) is now complete for l = 4
                memo_put<W>(p, table, tag, s.stP + j * W, x, acc_lo, acc_hi, acc_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
                ++n_ins;
              }
              __syncthreads();
            }
            if (stop || unit_cancel) break;
            res_lo = acc_lo;
            res_hi = acc_hi;
            res_fp = acc_fp;
            if (memo_j && memo_live && j > 0 && j != jsplit) {
              memo_put<W>(p, table, tag, s.stP + j * W, -1, res_lo, res_hi, res_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
              ++n_ins;
            }
            __syncthreads();
            mode = FINISH;
            continue;
          }
        }
        if (l - 1 <= kLaneEsymMaxL && !(memo_j && memo_live && j > 0 && j != jsplit)) {
          // complete and nearly complete child sets first, one per lane
          const ChildSum cs = complete_children<W, FP>(s, Q, s.stP + j * W, l - 1, !(j + 1 == jsplit && sub != 0));
          const u64 nlo = acc_lo + cs.lo;
          acc_hi += cs.hi + (nlo < acc_lo ? 1ull : 0ull);
          acc_lo = nlo;
          if (FP) acc_fp = addp(acc_fp, cs.fp);
          wops += cs.wops;
        }
        if (lane == 0) {
          s.stCnt[2 * j] = acc_lo;
          s.stCnt[2 * j + 1] = acc_hi;
          s.stFp[j] = acc_fp;
          s.stMemo[j] = memo_j ? 1 : 0;
        }
        __syncthreads();
        mode = NEXT;
        continue;
      }
      if (mode == NEXT) {
        const int l = k - 1 - j;
        u64* Q = s.stQ + j * W;
        int x = -1;
        for (int w = W - 1; w >= 0; --w) {
          u64 qw = Q[w];
          if (qw) {
            x = w * 64 + 63 - __clzll((long long)qw);
            break;
          }
        }
        __syncthreads();
        if (x < 0) {
          res_lo = s.stCnt[2 * j];
          res_hi = s.stCnt[2 * j + 1];
          res_fp = s.stFp[j];
          if (s.stMemo[j] && memo_live && j > 0 && j != jsplit) {
            u64 Pr[W];
#pragma unroll
            for (int w = 0; w < W; ++w) Pr[w] = s.stP[j * W + w];
            memo_put<W>(p, table, (mtag << 8) | (u64)l, s.stP + j * W, -1, res_lo, res_hi, res_fp, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
            ++n_ins;
          }
          __syncthreads();
          mode = FINISH;
          continue;
        }
        if (lane == 0) {
          Q[x >> 6] &= ~(1ull << (x & 63));
          s.stX[j] = (uint16_t)x;
        }
        if (lane < W) s.stP[(j + 1) * W + lane] = s.stP[j * W + lane] & s.A[x * W + lane];
        __syncthreads();
        ++j;
        mode = ENTER;
        continue;
      }
      // FINISH: hand (res_lo, res_hi, res_fp) to the parent
      if (j == 0) break;
      --j;
      {
        const int l = k - 1 - j;
        int x = s.stX[j];
        u64 lo = s.stCnt[2 * j], hi = s.stCnt[2 * j + 1], f = s.stFp[j];
        u64 nlo = lo + res_lo;
        hi += res_hi + (nlo < lo ? 1ull : 0ull);
        lo = nlo;
        if (FP) f = addp(f, mulp(s.gl[x], res_fp));
        __syncthreads();
        if (lane == 0) {
          s.stCnt[2 * j] = lo;
          s.stCnt[2 * j + 1] = hi;
          s.stFp[j] = f;
        }
        if (s.stMemo[j] && memo_live && j > 0 && j != jsplit) {
          // trie node t_i = P & [x, inf) is now complete for l
          memo_put<W>(p, table, (mtag << 8) | (u64)l, s.stP + j * W, x, lo, hi, f, p.tau ? Gdcol + (int32_t)s.ctl[3] : nullptr, room());
          ++n_ins;
        }
        __syncthreads();
        mode = NEXT;
      }
    }
    if (stop) {
      aborted = true;
      break;
    }
    if (unit_cancel) {  // the pair is reported as cancelled
      finish_units(p, pair, 1u + skip_rest(p, sg.pair_end));
      continue;
    }
    // unit result: cnt, fp times the prefix weight
    u64 rfp = FP ? mulp(rw, res_fp) : 0;
    if (p.pair_out && lane == 0) {
      // plain atomic adds only: many waves finish units of one pair at once
      u64* o = p.pair_out + 4 * (u64)pair;
      atomic_add128(o, res_lo, res_hi);
      if (rfp) atomic_add128(o + 2, rfp, 0);
    }
    u64 nlo = tot_lo + res_lo;
    tot_hi += res_hi + (nlo < tot_lo ? 1ull : 0ull);
    tot_lo = nlo;
    tot_fp = addp(tot_fp, rfp);
    if (p.per_root && lane == 0) {
      // several units may share a root: 128-bit add with carry, fp mod p
      u64* o = p.per_root + 3 * (u64)Gorig[r];
      u64 old = atomicAdd((unsigned long long*)&o[0], (unsigned long long)res_lo);
      u64 carry_in = (old + res_lo < old) ? 1ull : 0ull;
      if (res_hi + carry_in) atomicAdd((unsigned long long*)&o[1], (unsigned long long)(res_hi + carry_in));
      u64 cur = o[2], seen;
      do {
        seen = cur;
        cur = atomicCAS((unsigned long long*)&o[2], seen, addp(seen, rfp));
      } while (cur != seen);
    }
    finish_units(p, pair, 1u);
    __syncthreads();
  }

  // per-wave output
  u64 sw = wave_sum(wops), sb = wave_sum(bits), sa = wave_sum(arcs);
  if (lane == 0) {
    u64* o = p.wave_out + (u64)blockIdx.x * kOutWords;
    o[0] = tot_lo;
    o[1] = tot_hi;
    o[2] = tot_fp;
    o[3] = n_units;
    o[4] = n_pruned;
    o[5] = n_frames;
    o[6] = sw;
    o[7] = sb;
    o[8] = n_look;
    o[9] = n_hit;
    o[10] = n_ins;
    o[11] = sa;
    o[12] = aborted ? 1 : 0;
    o[13] = n_builds;
  }
}

// ---- EdgeParallel set-up (Section VII-D) ----------------------------------------

struct EdgePrep {
  const int32_t* dptr;
  const int32_t* dcol;
  const int32_t* roots;     // heavy roots are roots[0, nh)
  const u64* base;          // per heavy root: first record, first row word
  int32_t first, last;      // this launch's heavy roots
  int k;
  int prune;
  int32_t drows;
  EdgeRec* recs;
  u64* rows;
  unsigned* hist;           // records of each size d (DIST_MAX_OUTDEG + 1 bins)
};

// One wave per heavy root u: G_u is built and pruned exactly as for its own
// search, and each depth-1 child v that passes the search's child test at
// frame 0 (|N+(u) & N+(v)| >= k - 2, soft-embedding bound >= k - 1) gets a
// record whose row is G_u's row of v; the other children and a pruned root
// get d = 0.
template <int W>
__global__ __launch_bounds__(64) void k_edge_rows(EdgePrep p) {
  extern __shared__ __align__(16) char smem[];
  const int lane = lane_id();
  const Lds s = carve<W>(smem, p.k, 0, p.drows);
  for (int32_t i = p.first + (int32_t)blockIdx.x; i < p.last; i += (int32_t)gridDim.x) {
    const int32_t r = p.roots[i];
    const int32_t beg = p.dptr[r];
    const int d = p.dptr[r + 1] - beg;
    __syncthreads();
    build_subgraph<W>(s, p.dptr, p.dcol, nullptr, nullptr, nullptr, beg, d);
    bool dead = false;
    if (p.prune) {
      dead = soft_embed_levels<W>(s, d, p.k) < p.k;
    } else {
      for (int x = lane; x < d; x += kWave) s.rcap[x] = 63;
    }
    __syncthreads();
    const u64 rec0 = p.base[2 * (u64)i], row0 = p.base[2 * (u64)i + 1];
    for (int a = lane; a < d; a += kWave) {
      int c = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) c += __popcll(s.A[a * W + w]);
      const bool ok = !dead && c >= p.k - 2 && s.rcap[a] >= p.k - 1;
      EdgeRec e;
      e.u = r;
      e.v = p.dcol[beg + a];
      e.d = ok ? c : 0;
      e.wu = W;
      e.row = row0 + (u64)a * W;
      p.recs[rec0 + a] = e;
      if (ok) {
#pragma unroll
        for (int w = 0; w < W; ++w) p.rows[e.row + w] = s.A[a * W + w];
        atomicAdd(p.hist + c, 1u);
      }
    }
  }
}

// Records in descending order of size: cur[d] starts at the first slot of
// size d (a counting sort; the order among equal sizes is arbitrary).
__global__ void k_edge_order(const EdgeRec* recs, u64 nrec, unsigned* cur, int32_t* list) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (; i < nrec; i += stride) {
    const int d = recs[i].d;
    if (d > 0) list[atomicAdd(cur + d, 1u)] = (int32_t)i;
  }
}

__global__ void k_zero_u32(unsigned* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero_u64(u64* p, u64 n) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  u64 stride = (u64)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

__global__ void k_sum_weights(const u64* gw, int32_t n, u64* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  u64 s = 0;
  for (; i < n; i += stride) s = addp(s, gw[i]);
  s = wave_sum_p(s);
  if (lane_id() == 0) {
    // mod-p accumulation by compare-and-swap
    u64 old = *out, assumed;
    do {
      assumed = old;
      old = atomicCAS((unsigned long long*)out, assumed, addp(assumed, s));
    } while (old != assumed);
  }
}

// ---- host side ------------------------------------------------------------------

struct Workspace {
  int device = -1;
  int cus = 0;
  u64* wave_out = nullptr;
  size_t wave_out_words = 0;
  unsigned* cursor = nullptr;
  int* abort_flag = nullptr;
  u64* memo = nullptr;
  size_t memo_bytes = 0;
  u64* host_out = nullptr;  // pinned
  size_t host_out_words = 0;
  char* d_plan = nullptr;   // graph descriptor + segments of a single-graph launch
  char* h_plan = nullptr;   // pinned staging for the same
  size_t plan_cap = 0;
  char* edge = nullptr;     // EdgeParallel records, rows, order and histogram
  size_t edge_cap = 0;
};

Workspace g_ws;  // one device per process in this library
std::recursive_mutex g_ws_mu;  // serialises the calls that use g_ws

// Memo keys carry a root tag that is unique over the life of the process,
// so entries left in a table by an earlier launch can never match.
u64 g_tag_next = 1;

// The binomial table of a device is filled once, on a stream of its own,
// before the first search there (never inside a graph capture).
int ensure_binom() {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  DIST_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return DIST_OK;  // the kernels then compute binomials
  std::lock_guard<std::mutex> lock(mu);
  if (done[dev]) return DIST_OK;
  hipStream_t st = nullptr;
  DIST_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipLaunchKernelGGL(k_fill_binom, dim3((kBinomN + 1 + 255) / 256), dim3(256), 0, st);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (e1 != hipSuccess || e2 != hipSuccess) return DIST_E_DEVICE;
  done[dev] = true;
  return DIST_OK;
}

int ws_ensure(size_t wave_words, size_t memo_bytes) {
  int dev = 0;
  DIST_CHECK(hipGetDevice(&dev));
  if (g_ws.device != dev) {
    g_ws = Workspace();
    g_ws.device = dev;
    DIST_CHECK(hipDeviceGetAttribute(&g_ws.cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (dev_alloc((void**)&g_ws.cursor, 64 * sizeof(unsigned))) return DIST_E_NOMEM;
    if (dev_alloc((void**)&g_ws.abort_flag, 64)) return DIST_E_NOMEM;
  }
  if (wave_words > g_ws.wave_out_words) {
    if (g_ws.wave_out) dev_free(g_ws.wave_out);
    if (g_ws.host_out) pinned_free(g_ws.host_out);
    g_ws.wave_out = nullptr;
    g_ws.host_out = nullptr;
    g_ws.wave_out_words = 0;
    if (dev_alloc((void**)&g_ws.wave_out, wave_words * sizeof(u64))) return DIST_E_NOMEM;
    if (pinned_alloc((void**)&g_ws.host_out, wave_words * sizeof(u64)) != DIST_OK) return DIST_E_NOMEM;
    g_ws.wave_out_words = wave_words;
  }
  if (memo_bytes > g_ws.memo_bytes) {
    if (g_ws.memo) dev_free(g_ws.memo);
    g_ws.memo = nullptr;
    g_ws.memo_bytes = 0;
    if (dev_alloc((void**)&g_ws.memo, memo_bytes)) return DIST_E_NOMEM;
    g_ws.memo_bytes = memo_bytes;
  }
  return DIST_OK;
}

// Width classes (words per bitmap row), widest first.  A root goes to the
// narrowest class that holds its out-degree, so little of a row is zero.
constexpr int kClasses = 8;
const int kSlotWidth[kClasses] = {16, 8, 6, 5, 4, 3, 2, 1};

int width_of(int d) {
  for (int c = kClasses - 1; c >= 0; --c)
    if (d <= 64 * kSlotWidth[c]) return kSlotWidth[c];
  return 16;
}

int wslot_of_width(int W) {
  for (int c = 0; c < kClasses; ++c)
    if (kSlotWidth[c] == W) return c;
  return 0;
}

// Index into the per-class statistics (narrowest class first).
int wslot(int W) { return kClasses - 1 - wslot_of_width(W); }

// Calls f(std::integral_constant<int, W>) for a runtime class width W.
template <class F>
auto with_width(int W, F&& f) {
  switch (W) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return f(std::integral_constant<int, 16>{});
  }
}

int ws_plan(size_t bytes) {
  if (bytes <= g_ws.plan_cap) return DIST_OK;
  if (g_ws.d_plan) dev_free(g_ws.d_plan);
  if (g_ws.h_plan) pinned_free(g_ws.h_plan);
  g_ws.d_plan = nullptr;
  g_ws.h_plan = nullptr;
  g_ws.plan_cap = 0;
  if (dev_alloc((void**)&g_ws.d_plan, bytes)) return DIST_E_NOMEM;
  if (pinned_alloc((void**)&g_ws.h_plan, bytes) != DIST_OK) return DIST_E_NOMEM;
  g_ws.plan_cap = bytes;
  return DIST_OK;
}


// Units per range of depth-1 children, for each width class of one count.
// forced > 0 sets it for every class.  Else (automatic) a class is split only
// where its launch would wait on its heaviest unit: a depth-1 subtree costs
// roughly (d/64)^(k-3), the first child of a root about 2^(k-4) times the
// mean over its children, and a launch of W waves ideally takes
// sum(cost) / W; where the heaviest unit exceeds that, each child of a
// single-child unit is shared by up to kMaxSub units.
using DegHist = std::vector<std::pair<int32_t, int64_t>>;

// Calls f(d, a, b) for each run [a, b) of roots of equal out-degree d that
// falls in [first, end) (runs in descending out-degree order, as the roots).
template <class F>
void for_runs(const DegHist& h, int32_t first, int32_t end, F&& f) {
  int64_t a = 0;
  for (const auto& run : h) {
    if (a >= end) break;
    const int64_t b = std::min<int64_t>(a + run.second, end);
    const int64_t lo = std::max<int64_t>(a, first);
    if (b > lo) f((int)run.first, (int32_t)lo, (int32_t)b);
    a += run.second;
  }
}

void split_children(const DegHist& h, int32_t first, int32_t nroots, int k, int cw, int forced,
                    int (&sub_of)[kClasses]) {
  for (int& x : sub_of) x = 1;
  if (k < 6) return;
  if (forced > 0) {
    for (int& x : sub_of) x = forced < kMaxSub ? forced : kMaxSub;
    return;
  }
  double total[kClasses] = {}, heavy[kClasses] = {};
  for_runs(h, first, nroots, [&](int d, int32_t a, int32_t b) {
    const int sl = wslot_of_width(width_of(d));
    const double child = std::pow((double)d / 64.0, (double)(k - 3));
    total[sl] += (double)(b - a) * (double)d * child;
    if (children_per_unit(d, k, cw) == 1 && child > heavy[sl]) heavy[sl] = child;
  });
  const double waves = 8.0 * (g_ws.cus > 0 ? g_ws.cus : 256);
  for (int sl = 0; sl < kClasses; ++sl) {
    if (heavy[sl] <= 0 || total[sl] <= 0) continue;
    const double r = heavy[sl] * std::ldexp(1.0, k - 4) * waves / total[sl];
    if (r <= 1.0) continue;
    int sub = 2;
    while (sub < kMaxSub && sub < 2.0 * r) sub <<= 1;
    sub_of[sl] = sub;
  }
}

void split_children(const dist_graph* g, int32_t nroots, int k, int cw, int forced, int (&sub_of)[kClasses]) {
  split_children(g->deg_hist, 0, nroots, k, cw, forced, sub_of);
}

// The same for EdgeParallel units (clique size k counted from the arc's set,
// i.e. one less than the query's), each one range of children, per set size
// d: a unit costs about d (d/64)^(k-3) on average, but the arcs of equal
// set size differ widely (a dense core's arcs carry most of the work), so a
// run is shared out where 2^(k-2) times that mean (a factor measured on
// power-law graphs with planted cliques, k = 6..8) exceeds the mean load of
// a wave.  sub_d[d] for d <= DIST_MAX_OUTDEG.
void split_edges(const DegHist& h, int32_t n, int k, int forced, std::vector<int>& sub_d) {
  sub_d.assign(DIST_MAX_OUTDEG + 1, 1);
  if (k < 6) return;
  if (forced > 0) {
    for (int& x : sub_d) x = forced < kMaxSub ? forced : kMaxSub;
    return;
  }
  auto unit = [&](int d) { return (double)d * std::pow((double)d / 64.0, (double)(k - 3)); };
  double total[kClasses] = {};
  for_runs(h, 0, n, [&](int d, int32_t a, int32_t b) { total[wslot_of_width(width_of(d))] += (double)(b - a) * unit(d); });
  const double waves = 8.0 * (g_ws.cus > 0 ? g_ws.cus : 256);
  for_runs(h, 0, n, [&](int d, int32_t, int32_t) {
    const double t = total[wslot_of_width(width_of(d))];
    const double r = t > 0 ? unit(d) * std::ldexp(1.0, k - 2) * waves / t : 0.0;
    int sub = 1;
    while (sub < kMaxSub && sub < r) sub <<= 1;
    sub_d[d] = sub;
  });
}

// Appends the work segments of pair `pair` (roots [first, nroots) of a pair
// whose out-degree runs are h, clique size k) to the width classes:
// consecutive roots with the same width and the same split into units form
// one segment.  dmax[c] grows to the widest root put in class c.
// one_range: a root's depth-1 children form one range (units only share
// depth-2 children); sub_d, if set, gives the units sharing a range by
// out-degree instead of by class.
template <class SegList>
void add_segments(const DegHist& h, int pair, int32_t first, int32_t nroots, int k, int cw, bool whole_roots,
                  int min_w, const int (&sub_of)[kClasses], SegList (&segs)[kClasses],
                  uint64_t (&units)[kClasses], int (&kmax)[kClasses], int* dmax = nullptr,
                  bool one_range = false, const int* sub_d = nullptr) {
  // walks the runs of equal out-degree (roots are in descending out-degree
  // order), so planning costs O(distinct degrees), not O(roots)
  int cur_sl = -1, cur_upr = 0, cur_sub = 1;
  int32_t seg_a = 0, last = first;
  size_t first_seg[kClasses];
  for (int b = 0; b < kClasses; ++b) first_seg[b] = segs[b].size();
  auto flush = [&](int32_t end) {
    if (cur_sl < 0 || end <= seg_a) return;
    segs[cur_sl].push_back(BatchSeg{(uint32_t)units[cur_sl], pair, seg_a, cur_upr, 0u, cur_sub});
    units[cur_sl] += (uint64_t)(end - seg_a) * (uint64_t)cur_upr;
    if (k > kmax[cur_sl]) kmax[cur_sl] = k;
  };
  for_runs(h, first, nroots, [&](int d, int32_t a, int32_t b) {
    int W = width_of(d);
    if (W < min_w) W = width_of(64 * min_w);  // the narrowest class of at least min_w words
    const int sl = wslot_of_width(W);
    if (dmax && d > dmax[sl]) dmax[sl] = d;
    const int sub = (whole_roots || k < 6) ? 1 : sub_d ? sub_d[d] : sub_of[sl];
    const int upr = (whole_roots || one_range) ? sub : units_per_root(d, k, cw) * sub;
    if (sl != cur_sl || upr != cur_upr || sub != cur_sub) {
      flush(a);
      cur_sl = sl;
      cur_upr = upr;
      cur_sub = sub;
      seg_a = a;
    }
    last = b;
  });
  flush(last);
  for (int b = 0; b < kClasses; ++b)
    for (size_t i = first_seg[b]; i < segs[b].size(); ++i) segs[b][i].pair_end = (uint32_t)units[b];
}

template <class SegList>
void add_segments(const dist_graph* g, int pair, int32_t nroots, int k, int cw, bool whole_roots, int min_w,
                  const int (&sub_of)[kClasses], SegList (&segs)[kClasses],
                  uint64_t (&units)[kClasses], int (&kmax)[kClasses]) {
  add_segments(g->deg_hist, pair, 0, nroots, k, cw, whole_roots, min_w, sub_of, segs, units, kmax);
}

// The fingerprint switch is a template parameter: a count without
// fingerprints runs a kernel without their registers.
template <int W>
const void* search_kernel(bool fp) {
  return fp ? (const void*)k_search<W, true> : (const void*)k_search<W, false>;
}

template <int W>
int occupancy_blocks(size_t lds, bool fp) {
  int nb = 0;
  hipError_t e = fp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search<W, true>, 64, lds)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search<W, false>, 64, lds);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <int W>
int launch_bucket(Params prm, int grid, size_t lds, hipStream_t s, bool set_attr = true) {
  const bool fp = prm.fingerprint != 0;
  if (set_attr)
    DIST_CHECK(hipFuncSetAttribute(search_kernel<W>(fp), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (fp)
    hipLaunchKernelGGL((k_search<W, true>), dim3(grid), dim3(64), lds, s, prm);
  else
    hipLaunchKernelGGL((k_search<W, false>), dim3(grid), dim3(64), lds, s, prm);
  DIST_CHECK(hipGetLastError());
  return DIST_OK;
}


struct Bucket {
  int W;
  int32_t begin, end;  // range in g->roots
  int D = 0;           // LDS rows (lds_rows of the largest out-degree)
};

// Roots [0, nroots) of g->roots split into width buckets (widest first).
std::vector<Bucket> make_buckets(const dist_graph* g, int32_t nroots) {
  std::vector<Bucket> out;
  int32_t i = 0;
  while (i < nroots) {
    int W = width_of(g->root_deg[i]);
    int32_t j = i;
    while (j < nroots && width_of(g->root_deg[j]) == W) ++j;
    out.push_back({W, i, j, lds_rows(W, g->root_deg[i])});
    i = j;
  }
  return out;
}


// ---- EdgeParallel units (Section VII-D) --------------------------------------------
// The heavy roots' arcs (u, v) become units of their own, each searched over
// G[N+(u) & N+(v)] in the width class of that set: the deep subtrees of a
// wide root then run on rows of a few words instead of the root's.

template <int W>
int launch_edge_rows(const EdgePrep& ep, int32_t count, hipStream_t s) {
  const size_t lds = lds_bytes(W, ep.k, 0, ep.drows);
  DIST_CHECK(hipFuncSetAttribute((const void*)k_edge_rows<W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_edge_rows<W>, 64, lds) != hipSuccess || occ < 1) occ = 1;
  int64_t grid = (int64_t)occ * (g_ws.cus > 0 ? g_ws.cus : 256);
  if (grid > count) grid = count;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_edge_rows<W>, dim3((unsigned)grid), dim3(64), lds, s, ep);
  DIST_CHECK(hipGetLastError());
  return DIST_OK;
}

struct EdgeSet {
  const EdgeRec* recs = nullptr;
  const u64* rows = nullptr;
  const int32_t* list = nullptr;  // record indices, descending size
  DegHist hist;                   // runs (size, records) of the list
  int32_t n = 0;                  // records in the list
};

// Builds the edge units of heavy roots [0, nh) for clique size k (with the
// search's own pruning switch).  Synchronises the stream once (the size
// histogram sets the plan).
int edge_prepare(const dist_graph* g, int32_t nh, int k, int prune, hipStream_t s, EdgeSet* es) {
  constexpr int kBins = DIST_MAX_OUTDEG + 1;
  std::vector<u64> base(2 * (size_t)nh);
  u64 nrec = 0, nwords = 0;
  for (int32_t i = 0; i < nh; ++i) {
    const int d = g->root_deg[i];
    base[2 * (size_t)i] = nrec;
    base[2 * (size_t)i + 1] = nwords;
    nrec += (u64)d;
    nwords += (u64)d * (u64)width_of(d);
  }
  if (nrec >= 0x7fffffffull) return DIST_E_UNSUPPORTED;  // list entries are int32
  const size_t o_rows = align8(nrec * sizeof(EdgeRec));
  const size_t o_base = o_rows + nwords * sizeof(u64);
  const size_t o_list = o_base + base.size() * sizeof(u64);
  const size_t o_hist = align8(o_list + nrec * sizeof(int32_t));
  const size_t o_cur = o_hist + kBins * sizeof(unsigned);
  const size_t bytes = o_cur + kBins * sizeof(unsigned);
  if (bytes > g_ws.edge_cap) {
    if (g_ws.edge) dev_free(g_ws.edge);
    g_ws.edge = nullptr;
    g_ws.edge_cap = 0;
    if (dev_alloc((void**)&g_ws.edge, bytes)) return DIST_E_NOMEM;
    g_ws.edge_cap = bytes;
  }
  char* b = g_ws.edge;
  EdgeRec* recs = (EdgeRec*)b;
  u64* rows = (u64*)(b + o_rows);
  u64* d_base = (u64*)(b + o_base);
  int32_t* list = (int32_t*)(b + o_list);
  unsigned* hist = (unsigned*)(b + o_hist);
  unsigned* cur = (unsigned*)(b + o_cur);
  DIST_CHECK(hipMemcpyAsync(d_base, base.data(), base.size() * sizeof(u64), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero_u32, dim3((kBins + 63) / 64), dim3(64), 0, s, hist, kBins);
  for (const Bucket& bk : make_buckets(g, nh)) {
    EdgePrep ep{g->dptr, g->dcol, g->roots, d_base, bk.begin, bk.end, k, prune, bk.D, recs, rows, hist};
    const int rc = with_width(bk.W, [&](auto w) { return launch_edge_rows<decltype(w)::value>(ep, bk.end - bk.begin, s); });
    if (rc) return rc;
  }
  std::vector<unsigned> h(kBins), c(kBins, 0u);
  DIST_CHECK(hipMemcpyAsync(h.data(), hist, kBins * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  es->hist.clear();
  unsigned off = 0;
  for (int d = kBins - 1; d >= 1; --d) {
    c[d] = off;
    off += h[d];
    if (h[d]) es->hist.push_back({d, (int64_t)h[d]});
  }
  es->n = (int32_t)off;
  es->recs = recs;
  es->rows = rows;
  es->list = list;
  if (off == 0) return DIST_OK;
  DIST_CHECK(hipMemcpyAsync(cur, c.data(), kBins * sizeof(unsigned), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_edge_order, dim3(512), dim3(256), 0, s, recs, nrec, cur, list);
  DIST_CHECK(hipGetLastError());
  // the host vectors are read by the copies above before they go out of scope
  DIST_CHECK(hipStreamSynchronize(s));
  return DIST_OK;
}

// Segments of one graph's count: consecutive roots of equal out-degree fall
// into one segment, so a class holds at most as many segments as there are
// out-degrees (<= DIST_MAX_OUTDEG), and so does the whole plan.  A list of
// fixed capacity over static storage (calls hold g_ws_mu).
constexpr size_t kPlanSegs = DIST_MAX_OUTDEG;
struct SegList {
  BatchSeg* p = nullptr;
  size_t n = 0, cap = 0;
  void push_back(const BatchSeg& x) {
    if (n < cap) p[n] = x;
    ++n;
  }
  size_t size() const { return n < cap ? n : cap; }
  bool overflow() const { return n > cap; }
  BatchSeg& operator[](size_t i) { return p[i]; }
  const BatchSeg& operator[](size_t i) const { return p[i]; }
};
BatchSeg g_seg_store[kClasses][kPlanSegs];

// ---- scratch of the no-allocation entry point -------------------------------
// One fixed block of device memory per GPU holds everything a count needs
// beyond its inputs and outputs: the unit cursors and the abort flag, the
// per-wave results of up to kScratchWaves resident waves (a larger grid is
// clamped: the kernels are persistent) and the launch plan (graph descriptor
// and up to kPlanSegs segments).  Its host-side mirrors are static too.
constexpr int kScratchWaves = 4096;
constexpr size_t kScratchHead = 64;  // words: cursors (words 0..31), abort flag (32..39)
constexpr size_t kScratchPlanBytes = sizeof(BatchGraph) + sizeof(BatchSeg) * (kPlanSegs + 1);
constexpr size_t kScratchWords = kScratchHead + (size_t)kScratchWaves * kOutWords + (kScratchPlanBytes + 7) / 8;
static_assert(kScratchWaves == DIST_NOALLOC_WAVES && kPlanSegs == DIST_NOALLOC_PLAN_SEGS, "dist.h limits");
static __device__ __align__(256) u64 scratch[kScratchWords];
u64 g_scratch_host_out[(size_t)kScratchWaves * kOutWords];
u64 g_scratch_host_plan[(kScratchPlanBytes + 7) / 8];

// The device address of scratch on the current device, looked up once per
// device with that device current (each GPU holds its own copy).
int scratch_base(u64** out) {
  static std::mutex mu;
  static u64* base[64] = {};
  int dev = 0;
  DIST_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return DIST_E_DEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (!base[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DIST_E_DEVICE;
    base[dev] = (u64*)ptr;
  }
  *out = base[dev];
  return DIST_OK;
}

// ensure_binom without a stream of its own: the fill is queued on s, ahead of
// the searches of the same call.
int ensure_binom_on(hipStream_t s) {
  static bool done[64] = {};
  int dev = 0;
  DIST_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return DIST_OK;
  if (done[dev]) return DIST_OK;
  hipLaunchKernelGGL(k_fill_binom, dim3((kBinomN + 1 + 255) / 256), dim3(256), 0, s);
  DIST_CHECK(hipGetLastError());
  DIST_CHECK(hipStreamSynchronize(s));
  done[dev] = true;
  return DIST_OK;
}

// fixed != null: the no-allocation form -- every device buffer is a region of
// the scratch block at `fixed`, host copies go through static buffers, no
// memo table (it is a cache and changes no result) and no timing events.
int run_buckets(const dist_graph* g, Params base, int32_t nroots, const dist_config& cfg, hipStream_t s,
                u64* totals /* 16 */, double* ms_out, dist_stats* bst = nullptr, u64* fixed = nullptr) {
  for (int i = 0; i < kOutWords; ++i) totals[i] = 0;
  if (nroots <= 0) return DIST_OK;
  if (g->root_deg[0] > DIST_MAX_OUTDEG) return DIST_E_UNSUPPORTED;
  if (int rb = fixed ? ensure_binom_on(s) : ensure_binom()) return rb;
  const int cw = base.chunk_work;  // 0: automatic per k
  SegList segs[kClasses];
  for (int sl = 0; sl < kClasses; ++sl) segs[sl] = SegList{g_seg_store[sl], 0, kPlanSegs};
  uint64_t units64[kClasses] = {};
  int kmax[kClasses] = {};
  int sub_of[kClasses];
  int dmax[kClasses] = {};
  // EdgeParallel units for the heavy roots, a prefix of the roots (they are
  // in descending out-degree order); their segments come first in each class
  int32_t nh = 0;
  EdgeSet es;
  // automatic: roots of 4 or more words for k >= 5 (their arcs' sets then
  // still fill one word or more)
  const int ew = cfg.edge_units != 0 ? cfg.edge_units : base.k >= 5 ? 4 : -1;
  if (ew > 0 && !fixed && !base.soft_only && base.tau == 0 && base.k >= 4) {
    while (nh < nroots && width_of(g->root_deg[nh]) >= ew) ++nh;
    if (nh > 0) {
      if (int re = edge_prepare(g, nh, base.k, base.prune, s, &es)) return re;
      std::vector<int> sub_d;
      split_edges(es.hist, es.n, base.k - 1, cfg.sub_units, sub_d);
      add_segments(es.hist, 1, 0, es.n, base.k - 1, cw, false, 1, sub_of, segs, units64, kmax, dmax, true,
                   sub_d.data());
    }
  }
  split_children(g->deg_hist, nh, nroots, base.k, cw, cfg.sub_units, sub_of);
  add_segments(g->deg_hist, 0, nh, nroots, base.k, cw, base.soft_only != 0, 1, sub_of, segs, units64, kmax, dmax);
  const int nbg = nh > 0 ? 2 : 1;
  Bucket buckets[kClasses];
  uint32_t units[kClasses];
  size_t seg_off[kClasses];
  size_t nbk = 0;
  size_t nseg_total = 0;
  for (int sl = 0; sl < kClasses; ++sl) {
    if (segs[sl].overflow()) return DIST_E_UNSUPPORTED;
    if (units64[sl] == 0) continue;
    if (units64[sl] >= 0xffffffffull) return DIST_E_UNSUPPORTED;
    // roots are in descending out-degree order: a class's first root is its widest
    buckets[nbk] = Bucket{kSlotWidth[sl], 0, 0, lds_rows(kSlotWidth[sl], dmax[sl])};
    units[nbk] = (uint32_t)units64[sl];
    seg_off[nbk] = nseg_total;
    ++nbk;
    nseg_total += segs[sl].size();
  }
  if (fixed && nseg_total > kPlanSegs) return DIST_E_SCRATCH;
  {
    int dev = 0, maxlds = 0;
    DIST_CHECK(hipGetDevice(&dev));
    DIST_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    for (size_t b = 0; b < nbk; ++b)
      if (lds_bytes(buckets[b].W, base.k, base.fingerprint, buckets[b].D) > (size_t)maxlds) return DIST_E_UNSUPPORTED;
  }
  // grids and memo sizing
  int maxgrid = 0;
  int grids[kClasses];
  for (size_t b = 0; b < nbk; ++b) {
    int W = buckets[b].W;
    size_t lds = lds_bytes(W, base.k, base.fingerprint, buckets[b].D);
    int occ = 1;
    const bool fp = base.fingerprint != 0;
    occ = with_width(W, [&](auto w) { return occupancy_blocks<decltype(w)::value>(lds, fp); });
    int cus = g_ws.cus > 0 ? g_ws.cus : 256;
    int64_t grid = (int64_t)occ * cus;
    int64_t cnt = units[b];
    if (grid > cnt) grid = cnt;
    if (fixed && grid > kScratchWaves) grid = kScratchWaves;
    if (grid < 1) grid = 1;
    grids[b] = (int)grid;
    if (grids[b] > maxgrid) maxgrid = grids[b];
  }
  bool want_memo = cfg.memo != 0 && base.k >= 4 && !base.soft_only && !fixed;
  size_t memo_total = 0;
  u64 entries = 0;
  if (want_memo) {
    size_t budget = cfg.memo_bytes > 0 ? (size_t)cfg.memo_bytes : ((size_t)16 << 30);
    int maxW = 1;
    for (size_t b = 0; b < nbk; ++b) maxW = buckets[b].W > maxW ? buckets[b].W : maxW;
    size_t es = (size_t)(base.tau ? kShES : maxW + 4) * 8;
    if (cfg.memo_entries > 0) {
      entries = 1;
      while (entries < (u64)cfg.memo_entries) entries <<= 1;
    } else {
      entries = 1 << 16;
      while (entries > 256 && entries * es * (size_t)maxgrid > budget) entries >>= 1;
    }
    memo_total = entries * es * (size_t)maxgrid;
  }
  // device and host buffers: the library's workspace, or regions of scratch
  unsigned* cursor;
  int* abort_flag;
  u64* wave_out;
  u64* host_out;
  char* d_plan;
  char* h_plan;
  const size_t plan_bytes = nbg * sizeof(BatchGraph) + sizeof(BatchSeg) * (nseg_total + 1);
  int rc = DIST_OK;
  if (fixed) {
    cursor = (unsigned*)fixed;
    abort_flag = (int*)(fixed + 32);
    wave_out = fixed + kScratchHead;
    d_plan = (char*)(fixed + kScratchHead + (size_t)kScratchWaves * kOutWords);
    host_out = g_scratch_host_out;
    h_plan = (char*)g_scratch_host_plan;
  } else {
    rc = ws_ensure((size_t)maxgrid * kOutWords, memo_total);
    if (rc) return rc;
    rc = ws_plan(plan_bytes);
    if (rc) return rc;
    cursor = g_ws.cursor;
    abort_flag = g_ws.abort_flag;
    wave_out = g_ws.wave_out;
    host_out = g_ws.host_out;
    d_plan = g_ws.d_plan;
    h_plan = g_ws.h_plan;
  }
  // device plan: the graph descriptors (the roots; the edge units), then the
  // segments of every class
  {
    BatchGraph bgh[2] = {{g->dptr, g->dcol, g->orig, g->roots, g->gw, base.k, 0},
                         {g->dptr, g->dcol, g->orig, es.list, g->gw, base.k - 1, 0}};
    bgh[1].edges = es.recs;
    bgh[1].erows = es.rows;
    memcpy(h_plan, bgh, nbg * sizeof(BatchGraph));
    BatchSeg* hs = (BatchSeg*)(h_plan + nbg * sizeof(BatchGraph));
    size_t o = 0;
    for (int sl = 0; sl < kClasses; ++sl)
      for (size_t i = 0; i < segs[sl].size(); ++i) hs[o++] = segs[sl][i];
    DIST_CHECK(hipMemcpyAsync(d_plan, h_plan, plan_bytes, hipMemcpyHostToDevice, s));
  }
  const BatchGraph* d_bg = (const BatchGraph*)d_plan;
  const BatchSeg* d_segs = (const BatchSeg*)(d_plan + nbg * sizeof(BatchGraph));

  hipEvent_t e0 = nullptr, e1 = nullptr, kb0 = nullptr, kb1 = nullptr;
  if (!fixed) {
    DIST_CHECK(hipEventCreate(&e0));
    DIST_CHECK(hipEventCreate(&e1));
    DIST_CHECK(hipEventCreate(&kb0));
    DIST_CHECK(hipEventCreate(&kb1));
  }
  double kernel_ms = 0;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, cursor, 64);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (unsigned*)abort_flag, 16);
  u64 deadline = 0;
  if (cfg.deadline_ms > 0) {
    // wall_clock64 runs at a fixed rate: query it
    int rate_khz = 0;
    DIST_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, g_ws.device));
    deadline = (u64)cfg.deadline_ms * (u64)rate_khz;  // relative; made absolute on the device
  }
  if (!fixed) DIST_CHECK(hipEventRecord(e0, s));
  for (size_t b = 0; b < nbk; ++b) {
    Params prm = base;
    // light units (k <= 5) in a launch with many of them: a wave takes runs
    // of 8, which spares the cursor (the n = 1e6 graph at k = 5: 58 -> 43 ms);
    // deeper counts keep one unit at a time, since runs of heavy units
    // lengthen the tail (k = 9: 0.74 -> 0.99 s), and so do small launches
    if (!base.tau && base.k <= 5 && (uint64_t)units[b] >= 64ull * (uint64_t)grids[b]) prm.chunk = kShChunk;
    prm.root_deg = g->d_root_deg;
    prm.chunk_work = cw;
    prm.units = units[b];
    prm.bg = d_bg;
    prm.segs = d_segs + seg_off[b];
    prm.nsegs = (int32_t)segs[wslot_of_width(buckets[b].W)].size();
    prm.pair_out = nullptr;
    prm.cursor = cursor + b;  // one counter per bucket (zeroed above; <= 8 buckets)
    prm.wave_out = wave_out;
    prm.abort_flag = abort_flag;
    prm.memo_base = want_memo ? g_ws.memo : nullptr;
    prm.memo_mask = want_memo ? entries - 1 : 0;
    // root tags are unit indices of this launch: reserve the whole range
    prm.tag_base = g_tag_next;
    prm.epoch = nullptr;
    prm.deadline = deadline;
    g_tag_next += (u64)units[b] + 1;
    size_t lds = lds_bytes(buckets[b].W, base.k, base.fingerprint, buckets[b].D);
    prm.drows = buckets[b].D;
    hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, wave_out, (u64)grids[b] * kOutWords);
    if (!fixed) DIST_CHECK(hipEventRecord(kb0, s));
    rc = with_width(buckets[b].W, [&](auto w) { return launch_bucket<decltype(w)::value>(prm, grids[b], lds, s); });
    if (rc) break;
    if (!fixed) DIST_CHECK(hipEventRecord(kb1, s));
    DIST_CHECK(hipMemcpyAsync(host_out, wave_out, (size_t)grids[b] * kOutWords * sizeof(u64),
                              hipMemcpyDeviceToHost, s));
    DIST_CHECK(hipStreamSynchronize(s));
    float kms = 0;
    if (!fixed) DIST_CHECK(hipEventElapsedTime(&kms, kb0, kb1));
    kernel_ms += kms;
    u64 bw = 0, bb = 0, br = 0, ba = 0;
    for (int w = 0; w < grids[b]; ++w) {
      const u64* o = host_out + (size_t)w * kOutWords;
      br += o[3];
      bw += o[6];
      bb += o[7];
      ba += o[11];
    }
    if (bst) {
      int sl = wslot(buckets[b].W);
      bst->bucket_ms[sl] += kms;
      bst->bucket_roots[sl] += br;
      bst->bucket_word_ops[sl] += bw;
      bst->bucket_leaf_bits[sl] += bb;
      bst->bucket_arcs[sl] += ba;
    }
    for (int w = 0; w < grids[b]; ++w) {
      const u64* o = host_out + (size_t)w * kOutWords;
      u64 lo = totals[0] + o[0];
      totals[1] += o[1] + (lo < totals[0] ? 1 : 0);
      totals[0] = lo;
      u64 f = totals[2] + o[2];
      totals[2] = f >= DIST_P61 ? f - DIST_P61 : f;
      for (int i = 3; i < 12; ++i) totals[i] += o[i];
      totals[12] |= o[12];
      totals[13] += o[13];
    }
    if (totals[12]) break;
  }
  if (!fixed) {
    DIST_CHECK(hipEventRecord(e1, s));
    DIST_CHECK(hipEventSynchronize(e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(kb0);
    (void)hipEventDestroy(kb1);
  } else {
    DIST_CHECK(hipStreamSynchronize(s));
  }
  if (ms_out) *ms_out = kernel_ms;
  if (rc) return rc;
  return totals[12] ? DIST_E_CANCELLED : DIST_OK;
}

}  // namespace

int search_count(const SearchLaunch& L, dist_result* out, dist_stats* st, bool no_alloc) {
  std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
  const dist_graph* g = L.g;
  const int k = L.k;
  dist_result res{0, 0, 0};
  dist_stats stats{};
  hipStream_t s = L.stream;
  int rc = DIST_OK;
  u64* fixed = nullptr;
  if (no_alloc) {
    if (L.per_root) return DIST_E_INVALID;
    rc = scratch_base(&fixed);
    if (rc) return rc;
  }
  if (k == 1) {
    res.count_lo = (u64)g->n;
    if (L.cfg.fingerprint && g->n > 0) {
      u64* acc = nullptr;
      if (fixed) {
        acc = fixed + kScratchHead;
      } else {
        int r2 = ws_ensure(kOutWords, 0);
        if (r2) return r2;
        acc = g_ws.wave_out;
      }
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, acc, (u64)1);
      hipLaunchKernelGGL(k_sum_weights, dim3(256), dim3(256), 0, s, g->gw, g->n, acc);
      DIST_CHECK(hipMemcpyAsync(&res.fp, acc, sizeof(u64), hipMemcpyDeviceToHost, s));
      DIST_CHECK(hipStreamSynchronize(s));
    }
    if (L.per_root) {
      // every vertex is the minimum of its own 1-clique
      std::vector<u64> pr(3 * (size_t)g->n);
      std::vector<u64> gw(g->n);
      std::vector<int32_t> orig(g->n);
      DIST_CHECK(hipMemcpy(gw.data(), g->gw, sizeof(u64) * g->n, hipMemcpyDeviceToHost));
      DIST_CHECK(hipMemcpy(orig.data(), g->orig, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost));
      for (int32_t r = 0; r < g->n; ++r) {
        pr[3 * (size_t)orig[r]] = 1;
        pr[3 * (size_t)orig[r] + 2] = L.cfg.fingerprint ? gw[r] : 0;
      }
      DIST_CHECK(hipMemcpy(L.per_root, pr.data(), sizeof(u64) * pr.size(), hipMemcpyHostToDevice));
    }
    *out = res;
    if (st) *st = stats;
    return DIST_OK;
  }
  // roots: out-degree >= k - 1 (a prefix of the sorted roots)
  int32_t lo = 0, hi = g->n;
  while (lo < hi) {
    int32_t mid = (lo + hi) / 2;
    if (g->root_deg[mid] >= k - 1) lo = mid + 1; else hi = mid;
  }
  const int32_t nroots = lo;
  if (L.per_root && g->n > 0)
    hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, L.per_root, (u64)3 * g->n);
  Params prm{};
  prm.dptr = g->dptr;
  prm.dcol = g->dcol;
  prm.gw = g->gw;
  prm.orig = g->orig;
  prm.roots = g->roots;
  prm.k = k;
  prm.prune = L.cfg.prune;
  prm.memo = L.cfg.memo;
  prm.fingerprint = L.cfg.fingerprint;
  prm.soft_only = 0;
  prm.chunk_work = L.cfg.chunk_work;
  prm.per_root = L.per_root;
  prm.tau = (L.cfg.trie_tau > 0 && !fixed) ? (u64)L.cfg.trie_tau : 0;  // no memo without allocation
  prm.chunk = prm.tau ? kShChunk : 1;
  u64 tot[kOutWords];
  double ms = 0;
  rc = run_buckets(g, prm, nroots, L.cfg, s, tot, &ms, &stats, fixed);
  res.count_lo = tot[0];
  res.count_hi = tot[1];
  res.fp = L.cfg.fingerprint ? tot[2] : 0;
  stats.roots = tot[3];
  stats.roots_pruned = tot[4];
  stats.frames = tot[5];
  stats.word_ops = tot[6];
  stats.leaf_bits = tot[7];
  stats.memo_lookups = tot[8];
  stats.memo_hits = tot[9];
  stats.memo_inserts = tot[10];
  stats.subgraph_arcs = tot[11];
  stats.kernel_ms = ms;
  *out = res;
  if (st) *st = stats;
  if (rc == DIST_OK && res.count_hi != 0) rc = DIST_E_OVERFLOW;
  return rc;
}

int search_root_soft_embed(const dist_graph* g, int cap, int32_t* d_out, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
  // every vertex is a root here; vertices with no out-neighbour get r = 1
  std::vector<int32_t> ones;
  Params prm{};
  prm.dptr = g->dptr;
  prm.dcol = g->dcol;
  prm.gw = g->gw;
  prm.orig = g->orig;
  prm.roots = g->roots;
  prm.k = cap;
  prm.prune = 1;
  prm.memo = 0;
  prm.fingerprint = 0;
  prm.soft_only = 1;
  prm.soft_out = d_out;
  dist_config cfg;
  dist_config_init(&cfg);
  cfg.memo = 0;
  u64 tot[kOutWords];
  double ms = 0;
  return run_buckets(g, prm, g->n, cfg, s, tot, &ms);
}

// ---- listing: host side -----------------------------------------------------------
namespace {

u64 addp_host(u64 a, u64 b) {
  const u64 t = a + b;
  return t >= DIST_P61 ? t - DIST_P61 : t;
}

constexpr size_t kListBufBytes = (size_t)512 << 20;    // device record buffer (default)
constexpr size_t kListStageBytes = (size_t)64 << 20;   // pinned host staging
constexpr uint32_t kTrieNodes = 1u << 15;               // trie nodes per wave (default)

__global__ void k_gather_counts(const u64* per_root, const int32_t* orig, const int32_t* roots, int32_t nroots,
                                u64* out, int* wide) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nroots; i += stride) {
    const u64* o = per_root + 3 * (u64)orig[roots[i]];
    out[i] = o[0];
    if (o[1]) atomicOr(wide, 1);
  }
}

// Freed blocks are reused at once, so a buffer is released only after the
// stream's work (also on an error path) has finished.
struct DevBuf {
  hipStream_t s;
  void* p = nullptr;
  explicit DevBuf(hipStream_t st) : s(st) {}
  ~DevBuf() {
    if (p) {
      (void)hipStreamSynchronize(s);
      dev_free(p);
    }
  }
};
struct HostBuf {
  hipStream_t s;
  void* p = nullptr;
  explicit HostBuf(hipStream_t st) : s(st) {}
  ~HostBuf() {
    if (p) {
      (void)hipStreamSynchronize(s);
      pinned_free(p);
    }
  }
};

u64 g_ist_epoch = 1;  // trie epochs: unique over the life of the process

// Clears the hash slots of every wave's trie region (blocks = waves), so no
// stale word of reused memory can pass for a slot of a live epoch.
__global__ void k_zero_trie_hash(char* base, u64 stride, u64 hash_off, u64 hslots) {
  u64* h = (u64*)(base + (u64)blockIdx.x * stride + hash_off);
  for (u64 i = threadIdx.x; i < hslots; i += blockDim.x) h[i] = 0;
}

// Largest listing grid: the per-wave output words of the workspace.
constexpr int kListMaxWaves = 2048;

}  // namespace

// One launch of the trie listing kernel over roots [b0, b1) of g with their
// record offsets and counts (device arrays indexed from b0); see ist.hip.
// With inspect, one root and one retrieval (ret_*) and the wave's totals in
// wave_host.
static int list_launch(const dist_graph* g, int k, const dist_config& cfg, int W, int drows, int32_t b0, int32_t b1,
                       const u64* d_off, const u64* d_cnt, int32_t* d_out, int grid, char* trie, u64 stride,
                       uint32_t node_cap, u64 hslots, size_t lds, hipStream_t s, u64* wave_host, int* err_host,
                       const IstParams* extra) {
  IstParams prm{};
  if (extra) prm = *extra;
  prm.dptr = g->dptr;
  prm.dcol = g->dcol;
  prm.orig = g->orig;
  prm.roots = g->roots;
  prm.gw = g->gw;
  prm.k = k;
  prm.prune = cfg.prune;
  prm.memo = cfg.memo;
  prm.fingerprint = cfg.fingerprint;
  prm.root_begin = b0;
  prm.nroots = b1 - b0;
  prm.cursor = g_ws.cursor;
  prm.rec_off = d_off;
  prm.rec_cnt = d_cnt;
  prm.out = d_out;
  prm.drows = drows;
  prm.trie = trie;
  prm.trie_stride = stride;
  prm.node_cap = node_cap;
  prm.hmask = hslots - 1;
  prm.epoch_base = g_ist_epoch;
  g_ist_epoch += (u64)(b1 - b0) + 1;
  prm.wave_out = g_ws.wave_out;
  prm.err = g_ws.abort_flag;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, g_ws.cursor, 64);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (unsigned*)g_ws.abort_flag, 16);
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, g_ws.wave_out, (u64)grid * kOutWords);
  int rc = ist_list_launch(W, prm, grid, lds, s);
  if (rc) return rc;
  DIST_CHECK(hipMemcpyAsync(wave_host, g_ws.wave_out, (size_t)grid * kOutWords * sizeof(u64), hipMemcpyDeviceToHost,
                            s));
  DIST_CHECK(hipMemcpyAsync(err_host, g_ws.abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  return DIST_OK;
}

int search_list(const dist_graph* g, int k, const dist_config& cfg_in, dist_sink sink, void* user, int flags,
                hipStream_t s, dist_result* out, dist_stats* st_out) {
  std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
  dist_result res{0, 0, 0};
  dist_config cfg = cfg_in;
  dist_stats st{};
  *out = res;
  const bool dev_rows = (flags & DIST_LIST_DEVICE_ROWS) != 0;
  if (k == 1) {
    // every vertex is a 1-clique
    SearchLaunch L{g, 1, cfg, nullptr, s};
    dist_stats st1{};
    int rc = search_count(L, &res, &st1);
    if (rc) return rc;
    std::vector<int32_t> ids(1 << 20);
    DevBuf dids(s);
    if (dev_rows && dev_alloc(&dids.p, sizeof(int32_t) * ids.size())) return DIST_E_NOMEM;
    for (int32_t a = 0; a < g->n; a += (int32_t)ids.size()) {
      int32_t c = g->n - a < (int32_t)ids.size() ? g->n - a : (int32_t)ids.size();
      for (int32_t i = 0; i < c; ++i) ids[i] = a + i;
      const int32_t* rows = ids.data();
      if (dev_rows) {
        DIST_CHECK(hipMemcpyAsync(dids.p, ids.data(), sizeof(int32_t) * c, hipMemcpyHostToDevice, s));
        DIST_CHECK(hipStreamSynchronize(s));
        rows = (const int32_t*)dids.p;
      }
      if (sink(rows, (uint64_t)c, 1, user)) {
        *out = res;
        return DIST_E_CANCELLED;
      }
    }
    *out = res;
    return DIST_OK;
  }
  int32_t lo = 0, hi = g->n;
  while (lo < hi) {
    int32_t mid = (lo + hi) / 2;
    if (g->root_deg[mid] >= k - 1) lo = mid + 1; else hi = mid;
  }
  const int32_t nroots = lo;
  if (nroots == 0) {
    *out = res;
    if (st_out) *st_out = st;
    return DIST_OK;
  }
  if (g->root_deg[0] > DIST_MAX_OUTDEG) return DIST_E_UNSUPPORTED;
  // 1. per-root clique counts (count kernel), gathered in root order
  DevBuf per(s), cnts(s), offs(s), wide(s);
  if (dev_alloc(&per.p, sizeof(u64) * 3 * ((size_t)g->n + 1))) return DIST_E_NOMEM;
  if (dev_alloc(&cnts.p, sizeof(u64) * (size_t)nroots)) return DIST_E_NOMEM;
  if (dev_alloc(&offs.p, sizeof(u64) * (size_t)nroots)) return DIST_E_NOMEM;
  if (dev_alloc(&wide.p, 64)) return DIST_E_NOMEM;
  {
    dist_config cc = cfg;
    cc.fingerprint = 0;
    cc.deadline_ms = 0;
    SearchLaunch L{g, k, cc, (u64*)per.p, s};
    dist_result tmp;
    dist_stats st1{};
    int rc = search_count(L, &tmp, &st1);
    if (rc != DIST_OK && rc != DIST_E_OVERFLOW) return rc;
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (unsigned*)wide.p, 16);
  hipLaunchKernelGGL(k_gather_counts, dim3(256), dim3(256), 0, s, (const u64*)per.p, g->orig, g->roots, nroots,
                     (u64*)cnts.p, (int*)wide.p);
  std::vector<u64> rc_host(nroots);
  int wide_h = 0;
  DIST_CHECK(hipMemcpyAsync(rc_host.data(), cnts.p, sizeof(u64) * nroots, hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipMemcpyAsync(&wide_h, wide.p, sizeof(int), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipStreamSynchronize(s));
  if (wide_h) return DIST_E_UNSUPPORTED;
  const u64 rec_bytes = 4ull * (u64)k;
  u64 total = 0;
  for (u64 c : rc_host) total += c;
  const size_t buf_bytes = cfg.list_bytes > 0 ? (size_t)cfg.list_bytes : kListBufBytes;
  u64 cap = buf_bytes / rec_bytes;
  if (cap == 0) return DIST_E_UNSUPPORTED;
  for (u64 c : rc_host)
    if (c > cap) return DIST_E_UNSUPPORTED;  // one root's output exceeds the buffer
  if (total < cap) cap = total > 0 ? total : 1;
  // 2. buffers: records, host staging, per-wave tries
  DevBuf obuf(s), trie(s);
  HostBuf stage(s);
  if (dev_alloc(&obuf.p, cap * rec_bytes)) return DIST_E_NOMEM;
  size_t stage_bytes = 0;
  if (!dev_rows) {
    stage_bytes = cap * rec_bytes < kListStageBytes ? cap * rec_bytes : kListStageBytes;
    stage_bytes = stage_bytes / rec_bytes * rec_bytes;
    if (stage_bytes == 0) stage_bytes = rec_bytes;
    if (pinned_alloc(&stage.p, stage_bytes) != DIST_OK) return DIST_E_NOMEM;
  }
  std::vector<Bucket> buckets = make_buckets(g, nroots);
  int maxlds = 0;
  DIST_CHECK(hipGetDevice(&g_ws.device));
  DIST_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, g_ws.device));
  int cus = 0;
  DIST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g_ws.device));
  const bool use_trie = cfg.memo != 0;
  uint32_t node_cap = cfg.trie_nodes > 0 ? (uint32_t)std::min<int64_t>(cfg.trie_nodes, (1 << 24) - 1) : kTrieNodes;
  if (!use_trie) node_cap = 1;
  u64 hslots = 1;
  while (hslots < 2ull * node_cap) hslots <<= 1;
  // grids and the trie region (the largest any bucket needs)
  std::vector<int> grids(buckets.size());
  size_t trie_bytes = 0;
  for (size_t b = 0; b < buckets.size(); ++b) {
    const size_t lds = ist_lds_bytes(buckets[b].W, k, cfg.fingerprint, buckets[b].D);
    if (lds > (size_t)maxlds) return DIST_E_UNSUPPORTED;
    int64_t grid = (int64_t)ist_occupancy(buckets[b].W, lds) * cus;
    if (grid > kListMaxWaves) grid = kListMaxWaves;
    if (grid > buckets[b].end - buckets[b].begin) grid = buckets[b].end - buckets[b].begin;
    if (grid < 1) grid = 1;
    grids[b] = (int)grid;
    const IstLayout L = ist_layout(buckets[b].W, k, node_cap, hslots, buckets[b].D);
    trie_bytes = std::max(trie_bytes, (size_t)grid * L.total);
  }
  if (dev_alloc(&trie.p, trie_bytes)) return DIST_E_NOMEM;
  int rc = ws_ensure(kListMaxWaves * kOutWords, 0);
  if (rc) return rc;
  std::vector<u64> offs_h(nroots);
  u64 tot_lo = 0, tot_hi = 0, tot_fp = 0;
  bool cancelled = false;
  for (size_t bi = 0; bi < buckets.size() && !cancelled; ++bi) {
    const Bucket& bk = buckets[bi];
    const int W = bk.W;
    const size_t lds = ist_lds_bytes(W, k, cfg.fingerprint, bk.D);
    const IstLayout L = ist_layout(W, k, node_cap, hslots, bk.D);
    int32_t b0 = bk.begin;
    while (b0 < bk.end && !cancelled) {
      // batch [b0, b1): records within the buffer, each root at its offset
      u64 sum = 0;
      int32_t b1 = b0;
      while (b1 < bk.end && sum + rc_host[b1] <= cap) {
        offs_h[b1] = sum;
        sum += rc_host[b1++];
      }
      DIST_CHECK(hipMemcpyAsync((u64*)offs.p + b0, offs_h.data() + b0, sizeof(u64) * (size_t)(b1 - b0),
                                hipMemcpyHostToDevice, s));
      const int grid = std::min<int>(grids[bi], b1 - b0);
      if (use_trie)
        hipLaunchKernelGGL(k_zero_trie_hash, dim3(grid), dim3(256), 0, s, (char*)trie.p, (u64)L.total, (u64)L.hash,
                           hslots);
      std::vector<u64> wh((size_t)grid * kOutWords);
      int err = 0;
      rc = list_launch(g, k, cfg, W, bk.D, b0, b1, (const u64*)offs.p + b0, (const u64*)cnts.p + b0,
                       (int32_t*)obuf.p, grid, (char*)trie.p, L.total, node_cap, hslots, lds, s, wh.data(), &err,
                       nullptr);
      if (rc) return rc;
      if (err) return DIST_E_DEVICE;  // records disagree with the counts
      u64 b_cnt = 0, b_fp = 0;
      for (int w = 0; w < grid; ++w) {
        const u64* o = wh.data() + (size_t)w * kOutWords;
        b_cnt += o[0];
        b_fp = addp_host(b_fp, o[2]);
        st.roots += o[3];
        st.roots_pruned += o[4];
        st.frames += o[5];
        st.memo_inserts += o[7];   // trie nodes created
        st.memo_lookups += o[6];   // ListingDense frames
        st.memo_hits += o[9];      // retrievals from l-memoised nodes
        st.leaf_bits += o[10];     // cliques delivered by retrieval
      }
      if (b_cnt != sum) return DIST_E_DEVICE;
      // 3. hand the records to the sink
      if (dev_rows) {
        if (sum && sink((const int32_t*)obuf.p, sum, k, user)) cancelled = true;
      } else {
        const u64 per_stage = stage_bytes / rec_bytes;
        for (u64 a = 0; a < sum; a += per_stage) {
          u64 c = sum - a < per_stage ? sum - a : per_stage;
          DIST_CHECK(hipMemcpyAsync(stage.p, (char*)obuf.p + a * rec_bytes, c * rec_bytes, hipMemcpyDeviceToHost,
                                    s));
          DIST_CHECK(hipStreamSynchronize(s));
          if (sink((const int32_t*)stage.p, c, k, user)) {
            cancelled = true;
            break;
          }
        }
      }
      if (!cancelled) {
        u64 nl = tot_lo + b_cnt;
        tot_hi += (nl < tot_lo ? 1 : 0);
        tot_lo = nl;
        tot_fp = addp_host(tot_fp, b_fp);
      }
      b0 = b1;
    }
  }
  res.count_lo = tot_lo;
  res.count_hi = tot_hi;
  res.fp = cfg.fingerprint ? tot_fp : 0;
  *out = res;
  if (st_out) *st_out = st;
  if (cancelled) return DIST_E_CANCELLED;
  return res.count_hi ? DIST_E_OVERFLOW : DIST_OK;
}

// The trie of one root (inspection; see dist_ist_inspect).
int search_ist_inspect(const dist_graph* g, int k, int32_t root_id, const dist_config& cfg, const uint64_t* ret_set,
                       int ret_l, int32_t cap, int32_t* local_ids, int32_t* d_out, uint64_t* sets, uint64_t* marked,
                       uint32_t* lc, uint32_t* ls, int32_t* n_nodes, int32_t* rows, int64_t rows_cap,
                       int64_t* n_rows, int64_t* n_ret, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
  if (root_id < 0 || root_id >= g->n || k < 3 || cap < 1) return DIST_E_INVALID;
  if (ret_set && ret_l != k - 1) return DIST_E_INVALID;  // retrieved records are k-cliques
  // the root's rank, out-degree and clique count
  int32_t r = 0;
  DIST_CHECK(hipMemcpy(&r, g->rank + root_id, sizeof(int32_t), hipMemcpyDeviceToHost));
  int32_t pr[2];
  DIST_CHECK(hipMemcpy(pr, g->dptr + r, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
  const int d = pr[1] - pr[0];
  *d_out = d;
  if (d > DIST_MAX_OUTDEG) return DIST_E_UNSUPPORTED;
  std::vector<int32_t> nb(d);
  std::vector<int32_t> orig_all;
  if (d) DIST_CHECK(hipMemcpy(nb.data(), g->dcol + pr[0], sizeof(int32_t) * d, hipMemcpyDeviceToHost));
  for (int i = 0; i < d; ++i) DIST_CHECK(hipMemcpy(local_ids + i, g->orig + nb[i], sizeof(int32_t), hipMemcpyDeviceToHost));
  DevBuf per(s), dr(s), doff(s), dcnt(s), obuf(s), trie(s);
  if (dev_alloc(&per.p, sizeof(u64) * 3 * ((size_t)g->n + 1))) return DIST_E_NOMEM;
  {
    dist_config cc = cfg;
    cc.fingerprint = 0;
    SearchLaunch L{g, k, cc, (u64*)per.p, s};
    dist_result tmp;
    dist_stats st1{};
    int rc = search_count(L, &tmp, &st1);
    if (rc != DIST_OK && rc != DIST_E_OVERFLOW) return rc;
  }
  u64 rcnt[3];
  DIST_CHECK(hipMemcpy(rcnt, (u64*)per.p + 3 * (size_t)root_id, sizeof(rcnt), hipMemcpyDeviceToHost));
  if (rcnt[1]) return DIST_E_UNSUPPORTED;
  // rows holds rows_cap records in all: the root's, then the retrieval's
  if (rows && (rows_cap < 0 || (u64)rows_cap < rcnt[0])) return DIST_E_UNSUPPORTED;
  const u64 ret_cap = rows ? (u64)rows_cap - rcnt[0] : 0;
  const u64 total_rows = rcnt[0] + ret_cap;
  if (dev_alloc(&dr.p, sizeof(int32_t) * 2)) return DIST_E_NOMEM;
  if (dev_alloc(&doff.p, sizeof(u64))) return DIST_E_NOMEM;
  if (dev_alloc(&dcnt.p, sizeof(u64))) return DIST_E_NOMEM;
  if (dev_alloc(&obuf.p, 4ull * k * std::max<u64>(total_rows, 1))) return DIST_E_NOMEM;
  const int W = width_of(d < 1 ? 1 : d);
  const int D = lds_rows(W, d < 1 ? 1 : d);
  const uint32_t node_cap = (uint32_t)cap + 1;
  u64 hslots = 1;
  while (hslots < 2ull * node_cap) hslots <<= 1;
  const IstLayout L = ist_layout(W, k, node_cap, hslots, D);
  if (dev_alloc(&trie.p, L.total)) return DIST_E_NOMEM;
  hipLaunchKernelGGL(k_zero_trie_hash, dim3(1), dim3(256), 0, s, (char*)trie.p, (u64)L.total, (u64)L.hash, hslots);
  const u64 zero = 0;
  DIST_CHECK(hipMemcpy(dr.p, &r, sizeof(int32_t), hipMemcpyHostToDevice));
  DIST_CHECK(hipMemcpy(doff.p, &zero, sizeof(u64), hipMemcpyHostToDevice));
  DIST_CHECK(hipMemcpy(dcnt.p, &rcnt[0], sizeof(u64), hipMemcpyHostToDevice));
  int rc = ws_ensure(16 * kOutWords, 0);
  if (rc) return rc;
  IstParams extra{};
  extra.inspect = 1;
  extra.ret_l = ret_l;
  for (int w = 0; w < 16; ++w) extra.ret_key[w] = ret_set ? ret_set[w] : 0;
  extra.ret_off = rcnt[0];
  extra.ret_cap = ret_cap;
  // a plan whose roots array is the single root
  dist_graph one = *g;
  one.roots = (int32_t*)dr.p;
  u64 wh[kOutWords];
  int err = 0;
  const size_t lds = ist_lds_bytes(W, k, cfg.fingerprint, D);
  rc = list_launch(&one, k, cfg, W, D, 0, 1, (const u64*)doff.p, (const u64*)dcnt.p, (int32_t*)obuf.p, 1,
                   (char*)trie.p, L.total, node_cap, hslots, lds, s, wh, &err, &extra);
  if (rc) return rc;
  if (err || wh[14]) return DIST_E_DEVICE;
  const u64 nn = wh[11];
  *n_nodes = (int32_t)nn;
  *n_rows = (int64_t)rcnt[0];
  *n_ret = (int64_t)wh[13];
  if (nn > (u64)cap + 1) return DIST_E_UNSUPPORTED;
  std::vector<u64> keys(nn * W), mk(nn);
  std::vector<uint32_t> lcv(nn * k), lsv(nn * k);
  char* base = (char*)trie.p;
  DIST_CHECK(hipMemcpy(keys.data(), base + L.keys, sizeof(u64) * nn * W, hipMemcpyDeviceToHost));
  DIST_CHECK(hipMemcpy(mk.data(), base + L.marked, sizeof(u64) * nn, hipMemcpyDeviceToHost));
  DIST_CHECK(hipMemcpy(lcv.data(), base + L.lc, sizeof(uint32_t) * nn * k, hipMemcpyDeviceToHost));
  DIST_CHECK(hipMemcpy(lsv.data(), base + L.ls, sizeof(uint32_t) * nn * k, hipMemcpyDeviceToHost));
  for (u64 t = 0; t < nn; ++t) {
    for (int w = 0; w < 16; ++w) sets[t * 16 + w] = (t > 0 && w < W) ? keys[t * W + w] : 0;
    marked[t] = t > 0 ? mk[t] : ~0ull;
    for (int l = 0; l < k; ++l) {
      lc[t * k + l] = t > 0 ? lcv[t * k + l] : 0;
      ls[t * k + l] = t > 0 ? lsv[t * k + l] : 0;
    }
  }
  if (rows) {
    const u64 nr = rcnt[0] + wh[13];
    if (nr > (u64)rows_cap) return DIST_E_UNSUPPORTED;
    DIST_CHECK(hipMemcpy(rows, obuf.p, 4ull * k * nr, hipMemcpyDeviceToHost));
  }
  return DIST_OK;
}

// ---- pivot-based counting, every k at once (pivot.hip) ---------------------------

// The device address of the binomial table, filled first if needed.
static int binom_table(const u64** out) {
  if (int rc = ensure_binom()) return rc;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_binom)) != hipSuccess || !ptr) return DIST_E_DEVICE;
  *out = (const u64*)ptr;
  return DIST_OK;
}

int search_count_all(const dist_graph* g, int kmax, const dist_config& cfg, u64* per_root, int per_root_k,
                     hipStream_t s, dist_result* out, dist_stats* st_out) {
  std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
  constexpr int kPivWords = 256;   // per-wave output words of the pivot kernel
  constexpr int kPivMaxWaves = 2048;
  for (int k = 0; k <= kmax; ++k) out[k] = dist_result{0, 0, 0};
  dist_stats st{};
  const bool fp = cfg.fingerprint != 0;
  int rc = ws_ensure((size_t)kPivMaxWaves * kPivWords, 0);
  if (rc) return rc;
  if (per_root && g->n > 0) hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, per_root, (u64)3 * g->n);
  // k = 1: every vertex
  if (kmax >= 1) {
    out[1].count_lo = (u64)g->n;
    if (fp && g->n > 0) {
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, g_ws.wave_out, (u64)1);
      hipLaunchKernelGGL(k_sum_weights, dim3(256), dim3(256), 0, s, g->gw, g->n, g_ws.wave_out);
      DIST_CHECK(hipMemcpyAsync(&out[1].fp, g_ws.wave_out, sizeof(u64), hipMemcpyDeviceToHost, s));
      DIST_CHECK(hipStreamSynchronize(s));
    }
  }
  if (kmax < 2) {
    if (st_out) *st_out = st;
    return DIST_OK;
  }
  // roots with at least one out-neighbour (a prefix of the sorted roots)
  int32_t lo = 0, hi = g->n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) / 2;
    if (g->root_deg[mid] >= 1) lo = mid + 1; else hi = mid;
  }
  const int32_t nroots = lo;
  if (nroots == 0) {
    if (st_out) *st_out = st;
    return DIST_OK;
  }
  if (g->root_deg[0] > DIST_MAX_OUTDEG) return DIST_E_UNSUPPORTED;
  const u64* binom = nullptr;
  rc = binom_table(&binom);
  if (rc) return rc;
  std::vector<Bucket> buckets = make_buckets(g, nroots);
  int maxlds = 0, cus = 0;
  DIST_CHECK(hipGetDevice(&g_ws.device));
  DIST_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, g_ws.device));
  DIST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g_ws.device));
  std::vector<int> grids(buckets.size()), nsubs(buckets.size()), sdepth(buckets.size());
  size_t stack_words = 0;
  for (size_t b = 0; b < buckets.size(); ++b) {
    const size_t lds = pivot_lds_bytes(buckets[b].W, cfg.fingerprint, buckets[b].D);
    if (lds > (size_t)maxlds) return DIST_E_UNSUPPORTED;
    int64_t grid = (int64_t)pivot_occupancy(buckets[b].W, lds) * cus;
    if (grid > kPivMaxWaves) grid = kPivMaxWaves;
    // units per root: a launch with fewer than 8 roots per wave shares each
    // root among up to 64 units (a power of two), so that its few heavy
    // roots do not hold the launch; cfg.sub_units forces a count.  The units
    // part ways at depth 2 of the tree, at depth 24 where the launch has
    // fewer roots than waves, and at depth 32 where it has fewer than one
    // per 8 waves: a pivot tree keeps most of its nodes under the chain of
    // pivot children, so a shallow split leaves one unit most of a heavy root
    // (on the 10^6-vertex Chung-Lu graph, all k <= 9: one unit held 5.6M of a
    // root's nodes and the whole 11 s of its launch at depth 2).  The walk
    // above the split is repeated by every unit, so the depth grows only as
    // the roots per wave shrink (there, 708 roots: 2.2 s at depth 24, 3.1 s
    // at 32; 51 roots: 3.4 s at 24, 2.3 s at 32).
    const int64_t nr = buckets[b].end - buckets[b].begin;
    sdepth[b] = nr * 8 < grid ? 32 : (nr < grid ? 24 : 2);
    int nsub = 1;
    if (cfg.sub_units > 0) {
      nsub = std::min(cfg.sub_units, 64);
    } else {
      while (nsub < 64 && (int64_t)nsub * nr < 8 * grid) nsub *= 2;
    }
    while (nsub > 1 && nr * nsub > (int64_t)UINT32_MAX) nsub /= 2;  // unit numbers are 32-bit
    nsubs[b] = nsub;
    if (grid > nr * nsub) grid = nr * nsub;
    if (grid < 1) grid = 1;
    grids[b] = (int)grid;
    stack_words = std::max(stack_words, (size_t)grid * pivot_stack_words(buckets[b].W, kmax, buckets[b].D));
  }
  DevBuf stack(s);
  if (dev_alloc(&stack.p, stack_words * sizeof(u64))) return DIST_E_NOMEM;
  u64 deadline = 0;
  if (cfg.deadline_ms > 0) {
    int rate_khz = 0;
    DIST_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, g_ws.device));
    deadline = (u64)cfg.deadline_ms * (u64)rate_khz;
  }
  hipEvent_t e0, e1;
  DIST_CHECK(hipEventCreate(&e0));
  DIST_CHECK(hipEventCreate(&e1));
  std::vector<u64> wh((size_t)kPivMaxWaves * kPivWords);
  std::vector<u64> c_lo(kmax + 1, 0), c_hi(kmax + 1, 0), c_fp(kmax + 1, 0);
  bool aborted = false;
  double kernel_ms = 0;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (unsigned*)g_ws.abort_flag, 16);
  for (size_t b = 0; b < buckets.size() && !aborted; ++b) {
    const Bucket& bk = buckets[b];
    PivParams prm{};
    prm.dptr = g->dptr;
    prm.dcol = g->dcol;
    prm.orig = g->orig;
    prm.roots = g->roots + bk.begin;
    prm.gw = g->gw;
    prm.kmax = kmax;
    prm.fingerprint = cfg.fingerprint;
    prm.nroots = bk.end - bk.begin;
    prm.drows = bk.D;
    prm.cursor = g_ws.cursor;
    prm.stack = (u64*)stack.p;
    prm.binom = binom;
    prm.wave_out = g_ws.wave_out;
    prm.abort_flag = g_ws.abort_flag;
    prm.deadline = deadline;
    prm.per_root = per_root;
    prm.per_root_k = per_root ? per_root_k : -1;
    prm.nsub = nsubs[b];
    prm.split_depth = sdepth[b];
    const size_t lds = pivot_lds_bytes(bk.W, cfg.fingerprint, bk.D);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, g_ws.cursor, 64);
    hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, g_ws.wave_out, (u64)grids[b] * kPivWords);
    DIST_CHECK(hipEventRecord(e0, s));
    rc = pivot_launch(bk.W, prm, grids[b], lds, s);
    if (rc) break;
    DIST_CHECK(hipEventRecord(e1, s));
    DIST_CHECK(hipMemcpyAsync(wh.data(), g_ws.wave_out, (size_t)grids[b] * kPivWords * sizeof(u64),
                              hipMemcpyDeviceToHost, s));
    DIST_CHECK(hipStreamSynchronize(s));
    float kms = 0;
    DIST_CHECK(hipEventElapsedTime(&kms, e0, e1));
    kernel_ms += kms;
    st.bucket_ms[wslot(bk.W)] += kms;
    for (int w = 0; w < grids[b]; ++w) {
      const u64* o = wh.data() + (size_t)w * kPivWords;
      for (int k = 2; k <= kmax; ++k) {
        const u64 nl = c_lo[k] + o[3 * k];
        c_hi[k] += o[3 * k + 1] + (nl < c_lo[k] ? 1 : 0);
        c_lo[k] = nl;
        c_fp[k] = addp_host(c_fp[k], o[3 * k + 2]);
      }
      st.frames += o[192];
      st.leaf_bits += o[193];
      st.roots += o[194];
      st.subgraph_arcs += o[195];
      st.bucket_roots[wslot(bk.W)] += o[194];
      if (o[196]) aborted = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st.kernel_ms = kernel_ms;
  if (st_out) *st_out = st;
  if (rc) return rc;
  bool wide = false;
  for (int k = 2; k <= kmax; ++k) {
    out[k].count_lo = c_lo[k];
    out[k].count_hi = c_hi[k];
    out[k].fp = fp ? c_fp[k] : 0;
    wide = wide || c_hi[k] != 0;
  }
  if (aborted) return DIST_E_CANCELLED;
  return wide ? DIST_E_OVERFLOW : DIST_OK;
}

// ---- batched counting ----------------------------------------------------------
// Many (graph, k) pairs in one persistent launch per bitmap width: the work
// units of all pairs are laid end to end as segments of consecutive roots;
// every unit adds its root's result into its pair's slot.  Each HIP stream
// has its own batch workspace, so batches on different streams (issued from
// different host threads) run concurrently on the device.  With use_graph
// the launch sequence is captured as a hipGraph and replayed while the same
// batch is submitted again on that stream; every run starts a fresh range of
// memo root tags, so no run reuses what an earlier one stored.
namespace {

__global__ void k_bump_epoch(u64* e, u64 by) { *e += by; }

__global__ void k_zero_i32(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// cost tiers of a streamed batch (the cursor array holds 64 launch cursors)
constexpr int kTiers = 8;
constexpr double kTierDecades = 2.0;
static_assert(kTiers * kClasses <= 64, "one cursor per launch");

struct BatchLaunch {
  int W;
  int grid;
  size_t lds;
  Params prm;
};

template <class T>
int grow_dev(T** p, size_t& cap, size_t need) {
  if (need <= cap && *p) return DIST_OK;
  if (*p) dev_free(*p);
  *p = nullptr;
  cap = 0;
  if (dev_alloc((void**)p, need * sizeof(T))) return DIST_E_NOMEM;
  cap = need;
  return DIST_OK;
}

struct BatchWs {
  int device = -1;
  BatchGraph* d_bg = nullptr;
  size_t cap_bg = 0;
  BatchSeg* d_segs = nullptr;
  size_t cap_segs = 0;
  u64* d_pair_out = nullptr;  // 4 per pair, then one word: the launch abort flag
  size_t cap_out = 0;
  int* d_pair_abort = nullptr;
  size_t cap_pab = 0;
  unsigned* d_pair_rem = nullptr;       // per run: units left per pair
  unsigned* d_pair_rem_init = nullptr;  // units per pair
  size_t cap_rem = 0, cap_rem_init = 0;
  unsigned long long* d_pair_t0 = nullptr;
  size_t cap_t0 = 0;
  u64* h_pair_host = nullptr;           // pinned, device-visible: {flag, lo, hi, fp} per pair
  u64* d_pair_host = nullptr;           // its device address
  size_t cap_ph = 0;
  bool stream_done = false;             // publish per-pair completions
  u64* h_out = nullptr;       // pinned: pair_out, abort word, pair abort flags
  size_t cap_h = 0;
  unsigned* d_cursor = nullptr;
  int* d_abort = nullptr;
  u64* d_epoch = nullptr;
  u64* d_wave_out = nullptr;
  size_t cap_wave = 0;
  u64* d_memo = nullptr;
  size_t cap_memo = 0;
  // the batch held by this workspace
  int n = 0;
  std::vector<u64> serials;
  std::vector<int> ks;
  std::vector<int64_t> dls;
  dist_config cfg{};
  std::vector<dist_pair_switches> sw;  // per-pair switches (empty: none)
  std::vector<int> status;
  std::vector<uint32_t> units;          // units per pair
  std::vector<BatchLaunch> launches;
  u64 units_total = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    serials.clear();
  }
  ~BatchWs() {
    drop_graph();
    dev_free(d_bg);
    dev_free(d_segs);
    dev_free(d_pair_out);
    dev_free(d_pair_abort);
    dev_free(d_cursor);
    dev_free(d_abort);
    dev_free(d_epoch);
    dev_free(d_wave_out);
    dev_free(d_memo);
    dev_free(d_pair_rem);
    dev_free(d_pair_rem_init);
    dev_free(d_pair_t0);
    if (h_out) pinned_free(h_out);
    if (h_pair_host) pinned_free(h_pair_host);
  }
};

std::mutex g_batch_mu;
std::map<hipStream_t, BatchWs*> g_batch;

bool same_cfg(const dist_config& a, const dist_config& b) { return memcmp(&a, &b, sizeof(a)) == 0; }

int occupancy_any(int W, size_t lds, bool fp) {
  return with_width(W, [&](auto w) { return occupancy_blocks<decltype(w)::value>(lds, fp); });
}

const void* kernel_of(int W, bool fp) {
  return with_width(W, [&](auto w) { return search_kernel<decltype(w)::value>(fp); });
}

int launch_any(int W, const Params& prm, int grid, size_t lds, hipStream_t s) {
  // attributes were set before any capture began
  return with_width(W, [&](auto w) { return launch_bucket<decltype(w)::value>(prm, grid, lds, s, false); });
}

// Lays out the batch in ws and uploads its descriptors (synchronous on s).
u64 fold_p_host(u64 hi, u64 lo) {
  const unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;
  return (u64)(v % (unsigned __int128)DIST_P61);
}

int plan_batch(BatchWs* P, const dist_graph* const* gs, const int* ks, const int64_t* dls, int n,
               const dist_config& cfg, hipStream_t s, bool stream_done, const double* pair_cost,
               const dist_pair_switches* sw) {
  P->drop_graph();
  P->launches.clear();
  P->status.assign(n, DIST_OK);
  P->units_total = 0;
  int dev = 0, maxlds = 0, cus = 0, rate_khz = 0;
  DIST_CHECK(hipGetDevice(&dev));
  DIST_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  DIST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  DIST_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  std::vector<BatchGraph> bg(n);
  // Launch groups: tier-major, then width class.  A plain batch has one
  // tier.  When pairs are reported as they finish, or have budgets, pairs go
  // into tiers by predicted cost (kTierDecades decades each) and are taken
  // cheapest first, so a cheap pair never waits for the launch of an
  // expensive one.
  std::vector<BatchSeg> segs[kTiers][kClasses];
  uint64_t units64[kTiers][kClasses] = {};
  int kmax[kTiers][kClasses] = {};
  const int min_w = cfg.min_width > 1 ? cfg.min_width : 1;
  // batches split depth-1 children only on request: their graphs are small
  int sub_of[kClasses];
  for (int& x : sub_of) x = cfg.sub_units > 0 ? std::min(cfg.sub_units, kMaxSub) : 1;
  const int cw = cfg.chunk_work;  // 0: automatic per pair's k
  std::vector<int> order(n), tier(n, 0);
  for (int i = 0; i < n; ++i) order[i] = i;
  const bool own_clock = cfg.budget_from_pair_start != 0;
  bool by_cost = stream_done || pair_cost;
  for (int i = 0; i < n && dls && !by_cost; ++i) by_cost = dls[i] > 0;
  if (by_cost) {
    // With budgets that run from each pair's own start, a pair that waits
    // loses nothing: one tier.  With budgets from the batch start, a cheap
    // pair must not wait for the launch of an expensive one: cost tiers.
    std::vector<double> est(n);
    for (int i = 0; i < n; ++i) {
      est[i] = pair_cost ? pair_cost[i] : estimate_cost(gs[i], ks[i]);
      int t = (!own_clock && est[i] > 1) ? (int)(std::log10(est[i]) / kTierDecades) : 0;
      tier[i] = t < kTiers - 1 ? t : kTiers - 1;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return est[a] < est[b]; });
  }
  std::vector<uint32_t> rem_init(n > 0 ? n : 1, 0);
  bool any_memo = false;
  for (int oi = 0; oi < n; ++oi) {
    const int i = order[oi];
    const int t = tier[i];
    const dist_graph* g = gs[i];
    const int k = ks[i];
    u64 budget = (dls && dls[i] > 0) ? (u64)dls[i] * (u64)rate_khz : 0;
    bg[i] = BatchGraph{g->dptr, g->dcol, g->orig, g->roots, g->gw, k, own_clock ? 1 : 0, budget};
    // this pair's switches (< 0: the batch's)
    const int pmw = (sw && sw[i].min_width > 0) ? sw[i].min_width : min_w;
    const int pcw = (sw && sw[i].chunk_work >= 0) ? sw[i].chunk_work : cw;
    if (sw && sw[i].memo >= 0) bg[i].memo = sw[i].memo;
    if ((sw && sw[i].memo >= 0 ? sw[i].memo : cfg.memo) != 0) any_memo = true;
    if (k < 2) continue;  // k = 1 is answered on the host side
    int32_t lo = 0, hi = g->n;
    while (lo < hi) {
      int32_t mid = (lo + hi) / 2;
      if (g->root_deg[mid] >= k - 1) lo = mid + 1; else hi = mid;
    }
    const int32_t nroots = lo;
    if (nroots > 0 && g->root_deg[0] > DIST_MAX_OUTDEG) {
      P->status[i] = DIST_E_UNSUPPORTED;
      continue;
    }
    uint64_t* u = units64[t];
    uint64_t before = 0;
    for (int c = 0; c < kClasses; ++c) before += u[c];
    add_segments(g, i, nroots, k, pcw, false, pmw, sub_of, segs[t], units64[t], kmax[t]);
    uint64_t after = 0;
    for (int c = 0; c < kClasses; ++c) after += u[c];
    rem_init[i] = (uint32_t)(after - before);
  }
  std::vector<BatchSeg> all;
  size_t seg_off[kTiers][kClasses];
  for (int t = 0; t < kTiers; ++t)
    for (int b = 0; b < kClasses; ++b) {
      if (units64[t][b] >= 0xffffffffull) return DIST_E_UNSUPPORTED;
      seg_off[t][b] = all.size();
      all.insert(all.end(), segs[t][b].begin(), segs[t][b].end());
    }
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int rc = DIST_OK;
  if ((rc = grow_dev(&P->d_bg, P->cap_bg, nn))) return rc;
  if ((rc = grow_dev(&P->d_segs, P->cap_segs, all.size() + 1))) return rc;
  if ((rc = grow_dev(&P->d_pair_out, P->cap_out, 4 * nn + 1))) return rc;
  if ((rc = grow_dev(&P->d_pair_abort, P->cap_pab, nn))) return rc;
  if ((rc = grow_dev(&P->d_pair_rem, P->cap_rem, nn))) return rc;
  if ((rc = grow_dev(&P->d_pair_rem_init, P->cap_rem_init, nn))) return rc;
  if ((rc = grow_dev(&P->d_pair_t0, P->cap_t0, nn + 1))) return rc;
  if (6 * nn > P->cap_ph) {
    if (P->h_pair_host) pinned_free(P->h_pair_host);
    P->h_pair_host = nullptr;
    P->cap_ph = 0;
    if (pinned_alloc((void**)&P->h_pair_host, 6 * nn * sizeof(u64), hipHostMallocMapped | hipHostMallocCoherent) !=
        DIST_OK)
      return DIST_E_NOMEM;
    DIST_CHECK(hipHostGetDevicePointer((void**)&P->d_pair_host, P->h_pair_host, 0));
    P->cap_ph = 6 * nn;
  }
  DIST_CHECK(hipMemcpyAsync(P->d_pair_rem_init, rem_init.data(), sizeof(uint32_t) * nn, hipMemcpyHostToDevice, s));
  P->stream_done = stream_done;
  P->units.assign(rem_init.begin(), rem_init.begin() + n);
  if (!P->d_cursor && dev_alloc((void**)&P->d_cursor, 64 * sizeof(unsigned))) return DIST_E_NOMEM;
  if (!P->d_abort && dev_alloc((void**)&P->d_abort, 64)) return DIST_E_NOMEM;
  if (!P->d_epoch) {
    if (dev_alloc((void**)&P->d_epoch, 64)) return DIST_E_NOMEM;
    // a private range of root tags for this workspace
    u64 base;
    {
      std::lock_guard<std::recursive_mutex> lock(g_ws_mu);
      base = g_tag_next;
      g_tag_next += (u64)1 << 44;
    }
    DIST_CHECK(hipMemcpyAsync(P->d_epoch, &base, sizeof(u64), hipMemcpyHostToDevice, s));
    DIST_CHECK(hipStreamSynchronize(s));
  }
  const size_t hneed = 4 * nn + 1 + nn;  // pair_out, abort word, pair aborts (as u64 slots)
  if (hneed > P->cap_h) {
    if (P->h_out) pinned_free(P->h_out);
    P->h_out = nullptr;
    P->cap_h = 0;
    if (pinned_alloc((void**)&P->h_out, hneed * sizeof(u64)) != DIST_OK) return DIST_E_NOMEM;
    P->cap_h = hneed;
  }
  if (n) DIST_CHECK(hipMemcpyAsync(P->d_bg, bg.data(), sizeof(BatchGraph) * n, hipMemcpyHostToDevice, s));
  if (!all.empty())
    DIST_CHECK(hipMemcpyAsync(P->d_segs, all.data(), sizeof(BatchSeg) * all.size(), hipMemcpyHostToDevice, s));
  DIST_CHECK(hipStreamSynchronize(s));  // bg and all are host locals
  int maxgrid = 0, maxW = 1;
  for (int t = 0; t < kTiers; ++t)
  for (int b = 0; b < kClasses; ++b) {
    if (units64[t][b] == 0) continue;
    BatchLaunch L{};
    L.W = kSlotWidth[b];
    int dmax = 1;  // widest root of the launch: each segment's first root is its widest
    for (const auto& sg : segs[t][b]) dmax = std::max(dmax, (int)gs[sg.pair]->root_deg[sg.a]);
    const int drows = lds_rows(L.W, dmax);
    L.lds = lds_bytes(L.W, kmax[t][b], cfg.fingerprint, drows);
    if (L.lds > (size_t)maxlds) {
      for (auto& sg : segs[t][b]) P->status[sg.pair] = DIST_E_UNSUPPORTED;
      continue;
    }
    int occ = occupancy_any(L.W, L.lds, cfg.fingerprint != 0);
    int64_t grid = (int64_t)occ * (cus > 0 ? cus : 256);
    if (cfg.grid_pct > 0 && cfg.grid_pct < 100) grid = grid * cfg.grid_pct / 100;
    if (grid > (int64_t)units64[t][b]) grid = (int64_t)units64[t][b];
    L.grid = (int)(grid < 1 ? 1 : grid);
    Params& prm = L.prm;
    prm = Params{};
    prm.k = kmax[t][b];
    prm.drows = drows;
    prm.prune = cfg.prune;
    prm.memo = cfg.memo;
    prm.fingerprint = cfg.fingerprint;
    prm.tau = cfg.trie_tau > 0 ? (u64)cfg.trie_tau : 0;
    // runs of units only for the shared trie: runs of 8 took the 4,096-graph
    // batch from 118 to 107 ms, but they hold small serving batches back
    // (p50 18 -> 63 ms), where a few waves would take all the units
    prm.chunk = prm.tau ? kShChunk : 1;
    prm.cursor = P->d_cursor + (t * kClasses + b);
    prm.units = (uint32_t)units64[t][b];
    prm.chunk_work = cw;
    prm.bg = P->d_bg;
    prm.segs = P->d_segs + seg_off[t][b];
    prm.nsegs = (int32_t)segs[t][b].size();
    prm.pair_out = P->d_pair_out;
    prm.pair_abort = P->d_pair_abort;
    prm.pair_rem = stream_done ? P->d_pair_rem : nullptr;
    prm.pair_t0 = P->d_pair_t0;
    prm.pair_host = stream_done ? P->d_pair_host : nullptr;
    prm.abort_flag = P->d_abort;
    prm.epoch = P->d_epoch;
    prm.tag_base = P->units_total;  // units of earlier launches come first
    if (cfg.deadline_ms > 0) prm.deadline = (u64)cfg.deadline_ms * (u64)rate_khz;
    P->units_total += units64[t][b];
    P->launches.push_back(L);
    if (L.grid > maxgrid) maxgrid = L.grid;
    if (L.W > maxW) maxW = L.W;
  }
  if ((rc = grow_dev(&P->d_wave_out, P->cap_wave, (size_t)(maxgrid > 0 ? maxgrid : 1) * kOutWords))) return rc;
  u64 entries = 0;
  size_t memo_bytes = 0;
  if (any_memo && maxgrid > 0) {
    size_t budget = cfg.memo_bytes > 0 ? (size_t)cfg.memo_bytes : ((size_t)16 << 30);
    size_t es = (size_t)(cfg.trie_tau > 0 ? kShES : maxW + 4) * 8;
    entries = cfg.memo_entries > 0 ? 1 : (1 << 16);
    if (cfg.memo_entries > 0)
      while (entries < (u64)cfg.memo_entries) entries <<= 1;
    else
      while (entries > 256 && entries * es * (size_t)maxgrid > budget) entries >>= 1;
    memo_bytes = entries * es * (size_t)maxgrid;
    if ((rc = grow_dev((char**)&P->d_memo, P->cap_memo, memo_bytes))) return rc;
  }
  for (auto& L : P->launches) {
    L.prm.wave_out = P->d_wave_out;
    L.prm.memo_base = memo_bytes ? P->d_memo : nullptr;
    L.prm.memo_mask = memo_bytes ? entries - 1 : 0;
    DIST_CHECK(hipFuncSetAttribute(kernel_of(L.W, L.prm.fingerprint != 0), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)L.lds));
  }
  P->n = n;
  P->ks.assign(ks, ks + n);
  P->dls.assign(n, 0);
  if (dls) P->dls.assign(dls, dls + n);
  P->cfg = cfg;
  P->sw.clear();
  if (sw) P->sw.assign(sw, sw + n);
  P->serials.clear();
  for (int i = 0; i < n; ++i) P->serials.push_back(gs[i]->serial);
  return DIST_OK;
}

int enqueue_batch(BatchWs* P, hipStream_t s) {
  const int n = P->n;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  // fresh root tags for this run: memo entries of an earlier run never match
  hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(1), 0, s, P->d_epoch, P->units_total + 1);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, P->d_cursor, 64);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (unsigned*)P->d_abort, 16);
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, P->d_pair_out, (u64)(4 * nn));
  hipLaunchKernelGGL(k_zero_i32, dim3(64), dim3(256), 0, s, P->d_pair_abort, (int)nn);
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, (u64*)P->d_pair_t0, (u64)(nn + 1));
  if (P->stream_done)
    DIST_CHECK(hipMemcpyAsync(P->d_pair_rem, P->d_pair_rem_init, sizeof(unsigned) * nn, hipMemcpyDeviceToDevice, s));
  for (const auto& L : P->launches) {
    hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, P->d_wave_out, (u64)L.grid * kOutWords);
    int rc = launch_any(L.W, L.prm, L.grid, L.lds, s);
    if (rc) return rc;
  }
  DIST_CHECK(hipMemcpyAsync(P->h_out, P->d_pair_out, sizeof(u64) * 4 * nn, hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipMemcpyAsync(P->h_out + 4 * nn, P->d_abort, sizeof(int), hipMemcpyDeviceToHost, s));
  DIST_CHECK(hipMemcpyAsync(P->h_out + 4 * nn + 1, P->d_pair_abort, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
  return DIST_OK;
}

}  // namespace

int search_count_batch(const dist_graph* const* gs, const int* ks, int n, const dist_config& cfg, int use_graph,
                       const int64_t* dls, hipStream_t s, dist_result* out, int* pair_status, double* ms,
                       dist_pair_done on_done, void* user, const double* pair_cost, const dist_pair_switches* sw) {
  if (on_done) use_graph = 0;
  for (int i = 0; i < n; ++i)
    if (!gs[i] || ks[i] < 1 || ks[i] > DIST_K_MAX) return gs[i] ? DIST_E_K : DIST_E_INVALID;
  if (int rb = ensure_binom()) return rb;
  int dev = 0;
  DIST_CHECK(hipGetDevice(&dev));
  if (use_graph && s == nullptr) {
    // the legacy default stream cannot be captured: use a library stream
    static hipStream_t own = nullptr;
    static int own_dev = -1;
    {
      std::lock_guard<std::mutex> lock(g_batch_mu);
      if (own_dev != dev) {
        DIST_CHECK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        own_dev = dev;
      }
    }
    DIST_CHECK(hipDeviceSynchronize());
    int rc2 = search_count_batch(gs, ks, n, cfg, use_graph, dls, own, out, pair_status, ms, on_done, user,
                                 pair_cost, sw);
    DIST_CHECK(hipStreamSynchronize(own));
    return rc2;
  }
  BatchWs* P = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    BatchWs*& slot = g_batch[s];
    if (slot && slot->device != dev) {
      delete slot;
      slot = nullptr;
    }
    if (!slot) {
      slot = new BatchWs();
      slot->device = dev;
    }
    P = slot;
  }
  bool reuse = use_graph && P->exec && P->n == n && same_cfg(P->cfg, cfg) &&
               std::equal(P->ks.begin(), P->ks.end(), ks) && (int)P->serials.size() == n;
  for (int i = 0; i < n && reuse; ++i) reuse = P->serials[i] == gs[i]->serial && P->dls[i] == (dls ? dls[i] : 0);
  if (reuse) reuse = sw ? (P->sw.size() == (size_t)n && memcmp(P->sw.data(), sw, sizeof(*sw) * n) == 0) : P->sw.empty();
  hipEvent_t e0, e1;
  DIST_CHECK(hipEventCreate(&e0));
  DIST_CHECK(hipEventCreate(&e1));
  int rc = DIST_OK;
  if (!reuse) {
    rc = plan_batch(P, gs, ks, dls, n, cfg, s, on_done != nullptr, pair_cost, sw);
    if (rc) {
      P->drop_graph();
      return rc;
    }
    if (use_graph) {
      DIST_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      int erc = enqueue_batch(P, s);
      hipGraph_t gr = nullptr;
      hipError_t ce = hipStreamEndCapture(s, &gr);
      if (erc || ce != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        P->drop_graph();
        return erc ? erc : DIST_E_DEVICE;
      }
      P->graph = gr;
      if (hipGraphInstantiate(&P->exec, gr, nullptr, nullptr, 0) != hipSuccess) {
        P->drop_graph();
        return DIST_E_DEVICE;
      }
    }
  }
  const size_t nn0 = (size_t)(n > 0 ? n : 1);
  std::vector<char> reported;
  double ticks_per_ms = 1.0;
  if (on_done) {
    int rate_khz = 0;
    DIST_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    ticks_per_ms = rate_khz > 0 ? (double)rate_khz : 1.0;
    memset(P->h_pair_host, 0, 6 * nn0 * sizeof(u64));
    reported.assign(n, 0);
    // pairs with no work (no root deep enough) are done before the launch
    for (int i = 0; i < n; ++i)
      if (ks[i] >= 2 && P->status[i] == DIST_OK && P->units[i] == 0) {
        dist_result r{0, 0, 0};
        reported[i] = 1;
        out[i] = r;
        on_done(i, &r, DIST_OK, 0.0, user);
      }
  }
  DIST_CHECK(hipEventRecord(e0, s));
  if (P->exec) {
    DIST_CHECK(hipGraphLaunch(P->exec, s));
  } else {
    rc = enqueue_batch(P, s);
    if (rc) return rc;
  }
  DIST_CHECK(hipEventRecord(e1, s));
  if (on_done) {
    // report pairs as the device finishes them
    for (;;) {
      bool finished = hipEventQuery(e1) == hipSuccess;
      for (int i = 0; i < n; ++i) {
        if (reported[i] || ks[i] < 2 || P->status[i] != DIST_OK) continue;
        const u64* h = P->h_pair_host + 6 * i;
        u64 flag = __atomic_load_n(h, __ATOMIC_ACQUIRE);
        if (!flag) continue;
        dist_result r{h[1], h[2], cfg.fingerprint ? h[3] : 0};
        int st = flag == 2 ? DIST_E_CANCELLED : (r.count_hi ? DIST_E_OVERFLOW : DIST_OK);
        double dms = h[5] > h[4] ? (double)(h[5] - h[4]) / ticks_per_ms : 0.0;
        reported[i] = 1;
        on_done(i, &r, st, dms, user);
      }
      if (finished) break;
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  }
  DIST_CHECK(hipEventSynchronize(e1));
  float t = 0;
  DIST_CHECK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms) *ms = t;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const bool aborted = (P->h_out[4 * nn] & 0xffffffffull) != 0;
  const int* pab = (const int*)(P->h_out + 4 * nn + 1);
  int first = aborted ? DIST_E_CANCELLED : DIST_OK;
  for (int i = 0; i < n; ++i) {
    dist_result r{P->h_out[4 * i], P->h_out[4 * i + 1],
                  cfg.fingerprint ? fold_p_host(P->h_out[4 * i + 3], P->h_out[4 * i + 2]) : 0};
    int st = P->status[i];
    if (st == DIST_OK && (aborted || pab[i])) st = DIST_E_CANCELLED;
    if (ks[i] == 1 && st == DIST_OK) {
      SearchLaunch L{gs[i], 1, cfg, nullptr, s};
      dist_stats dummy{};
      st = search_count(L, &r, &dummy);
    }
    if (st == DIST_OK && r.count_hi) st = DIST_E_OVERFLOW;
    out[i] = r;
    if (pair_status) pair_status[i] = st;
    if (on_done && !reported[i]) on_done(i, &r, st, -1.0, user);
    if (st != DIST_OK && first == DIST_OK) first = st;
  }
  if (!use_graph) P->serials.clear();  // nothing captured to replay
  return first;
}

void batch_forget(const dist_graph* g) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (auto& kv : g_batch) {
    BatchWs* P = kv.second;
    for (u64 sr : P->serials)
      if (sr == g->serial) {
        P->drop_graph();
        break;
      }
  }
}

double estimate_cost(const dist_graph* g, int k) {
  if (k <= 1) return (double)g->n;
  const int r = k - 1;
  double total = 0;
  for (const auto& dc : g->deg_hist) {
    if (dc.first < r) continue;
    double lc = std::lgamma((double)dc.first + 1) - std::lgamma((double)r + 1) - std::lgamma((double)(dc.first - r) + 1);
    total += (double)dc.second * std::exp(lc);
  }
  return total;
}
