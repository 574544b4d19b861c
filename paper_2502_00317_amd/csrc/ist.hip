// ist.hip -- k-clique listing with the Induced Subgraph Trie (Section IV;
// Algorithms 2, 3 and 4), one wavefront per root.
//
// A root u's search runs on its 1-induced subgraph G_u, built in LDS as
// bitmap rows over local ids (the rank order of N+(u)).  Frames follow
// Algorithm 2's Listing and Algorithm 3's ListingDense:
//
//  * a Listing frame (candidate set P, l vertices still needed) extends the
//    clique by every member x of P whose branch survives the pruning test
//    (|P & A[x]| >= l - 1 and the soft-embedding bound r(x) >= l, Lemma 1);
//    the child runs as ListingDense when criterion (1) holds for it (only if
//    it needs at least 4 vertices), else as Listing; l = 2 reports the edges
//    of G[P], l = 3 (Listing only) the triangles, lane-parallel;
//  * a ListingDense frame inserts the identifying string of P (its members,
//    highest first) into the trie and walks the path t_1 .. t_|P|: for
//    t_i with Marked[l] it retrieves the inclusive set of t_i through the
//    trie (ListingIST below); otherwise it sets the l-sibling link of t_i,
//    lists the child G[P & A[x_i]] recursively (or takes the root as its
//    l-child link when the branch is pruned), sets the l-child link and
//    marks t_i.  l = 2 reports the edges of G[P] and links every t_i to the
//    node of the string of its out-neighbourhood;
//  * ListingIST(t, l, C) walks t's l-child link for the cliques containing
//    l(t) and its l-sibling link for the rest, down to l = 1, where the
//    cliques are C plus each vertex of the node's set (a 1-sibling link leads
//    to the parent, so the 1-level walk visits exactly the node's members).
//
// Trie nodes.  A node is identified by its identifying string, i.e. by its
// vertex set (a prefix of a string of members in descending order is the set
// of the largest ones).  Within one root every set is a bitmap over local
// ids, so the trie is kept as a hash table from bitmap to node: the nodes of
// all prefixes of a string are found or created at once, one lane each, and
// a node's parent is the node of the next shorter prefix.  Per node: its set
// (W words), Marked[l] as one bit per l, and the l-child and l-sibling links
// for l < k.  The trie of a root lives in a per-wave region of device memory
// and is discarded (by an epoch tag on the hash slots) when the wave moves on
// to its next root.  If the node pool of a wave fills up, a ListingDense
// frame that cannot insert its string runs as Listing instead, and a node is
// marked only when its links lead to memoised nodes, so every result stays
// exact.
//
// Records: each clique is written once as k input ids in ascending order, at
// the root's own offset (prefix sums of the per-root counts of a counting
// pass), so no atomic is needed; a root that writes a different number of
// records than counted raises the error flag.
#include "device_common.h"
#include "ist.h"

namespace {

constexpr uint32_t kTrieRoot = 0;
constexpr u64 kEpochMask = (1ull << 40) - 1;  // hash slot: epoch (40 bits) | node (24 bits)
constexpr int kOutW = 16;

struct Trie {
  u64* keys;        // node_cap * W
  u64* marked;      // node_cap
  uint32_t* lc;     // node_cap * k   (index l, 1 <= l < k)
  uint32_t* ls;     // node_cap * k
  uint32_t* label;  // node_cap
  u64* hash;        // hmask + 1 slots
  uint32_t* path;   // k * drows: node of P & [x, inf) for member x of the frame at depth j
};

template <int W>
__device__ Trie trie_view(const IstParams& p) {
  char* b = p.trie + (u64)blockIdx.x * p.trie_stride;
  const IstLayout L = ist_layout(W, p.k, p.node_cap, p.hmask + 1, p.drows);
  Trie t;
  t.keys = (u64*)(b + L.keys);
  t.marked = (u64*)(b + L.marked);
  t.lc = (uint32_t*)(b + L.lc);
  t.ls = (uint32_t*)(b + L.ls);
  t.label = (uint32_t*)(b + L.label);
  t.hash = (u64*)(b + L.hash);
  t.path = (uint32_t*)(b + L.path);
  return t;
}

// trie metadata is read and written by lane 0 only (wave-private memory)
__device__ __forceinline__ uint32_t tget32(const uint32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void tput32(uint32_t* a, uint32_t v) {
  __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void tput64(u64* a, u64 v) {
  __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t bcast32(uint32_t v) { return (uint32_t)__shfl((int)v, 0); }
__device__ __forceinline__ u64 bcast64(u64 v) { return __shfl(v, 0); }

// Wave-uniform reads of a node's fields (lane 0 loads, every lane gets it).
__device__ __forceinline__ u64 node_marked(const Trie& T, uint32_t t) {
  u64 v = 0;
  if (lane_id() == 0) v = ld_wave(T.marked + t);
  return bcast64(v);
}
__device__ __forceinline__ uint32_t node_lc(const Trie& T, int k, uint32_t t, int l) {
  uint32_t v = 0;
  if (lane_id() == 0) v = tget32(T.lc + (u64)t * k + l);
  return bcast32(v);
}
__device__ __forceinline__ uint32_t node_ls(const Trie& T, int k, uint32_t t, int l) {
  uint32_t v = 0;
  if (lane_id() == 0) v = tget32(T.ls + (u64)t * k + l);
  return bcast32(v);
}
__device__ __forceinline__ void set_links(const Trie& T, int k, uint32_t t, int l, uint32_t lc, uint32_t ls) {
  if (lane_id() == 0) {
    tput32(T.lc + (u64)t * k + l, lc);
    tput32(T.ls + (u64)t * k + l, ls);
  }
}
__device__ __forceinline__ void set_lc(const Trie& T, int k, uint32_t t, int l, uint32_t lc) {
  if (lane_id() == 0) tput32(T.lc + (u64)t * k + l, lc);
}
__device__ __forceinline__ void set_ls(const Trie& T, int k, uint32_t t, int l, uint32_t ls) {
  if (lane_id() == 0) tput32(T.ls + (u64)t * k + l, ls);
}
// The root of the trie is l-memoised for every l; a node is 1-memoised (its
// 1-child link is the root and its 1-sibling link its parent).
__device__ __forceinline__ bool memoised(const Trie& T, uint32_t t, int l) {
  if (t == kTrieRoot || l <= 1) return true;
  return (node_marked(T, t) >> l) & 1ull;
}
__device__ __forceinline__ void set_marked(const Trie& T, uint32_t t, int l) {
  if (lane_id() == 0) {
    const u64 m = ld_wave(T.marked + t);
    tput64(T.marked + t, m | (1ull << l));
  }
}

template <int W>
__device__ __forceinline__ u64 set_hash(const u64 (&key)[W]) {
  u64 h = 0x51ED270B27E4A6D1ull;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    h ^= key[w];
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  return h ^ (h >> 29);
}

__device__ __forceinline__ u64 cutm(int x, int w) {
  const int lo_b = w * 64;
  return (x <= lo_b) ? ~0ull : (x >= lo_b + 64 ? 0ull : (~0ull << (x - lo_b)));
}

// Wave-collective: inserts the identifying string of the set S into the trie
// (Algorithm 3, first line): for every member y of S the node of the prefix
// S & [y, inf) is found or created, and path[y] receives it.  Lanes take the
// members; each hashes its prefix set and probes linearly, creating the node
// in the first free slot of this epoch (node ids from the wave's counter).
// Returns false, with path incomplete, if the node pool is full.
template <int W>
__device__ bool trie_insert(const Trie& T, const u64 (&S)[W], uint16_t* scratch, uint32_t* path, u64 epoch,
                            uint32_t& nnodes, uint32_t cap, u64 hmask, u64& created) {
  const int lane = lane_id();
  int ns = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 b = S[w];
    if ((b >> lane) & 1ull) scratch[ns + __popcll(b & lanemask_lt())] = (uint16_t)(w * 64 + lane);
    ns += __popcll(b);
  }
  __syncthreads();
  const u64 tag = (epoch & kEpochMask) << 24;
  bool ok = true;
  for (int base = 0; base < ns && ok; base += kWave) {
    const int i = base + lane;
    const bool act = i < ns;
    const int y = act ? (int)scratch[i] : 0;
    u64 key[W];
#pragma unroll
    for (int w = 0; w < W; ++w) key[w] = act ? (S[w] & cutm(y, w)) : 0ull;
    u64 h = set_hash<W>(key);
    uint32_t node = 0, mine = 0;
    bool done = !act;
    while (__any(!done)) {
      bool need = false;
      u64 slot = 0;
      if (!done) {
        slot = ld_wave(T.hash + (h & hmask));
        if ((slot & ~0xFFFFFFull) == tag) {
          const uint32_t nd = (uint32_t)(slot & 0xFFFFFFull);
          bool eq = true;
#pragma unroll
          for (int w = 0; w < W; ++w) eq = eq && (ld_wave(T.keys + (u64)nd * W + w) == key[w]);
          if (eq) {
            node = nd;
            done = true;
          } else {
            ++h;
          }
        } else {
          need = true;  // a free slot (empty, or left by an earlier root)
        }
      }
      // a node id for every lane that will claim a slot and has none yet
      const u64 fresh = __ballot(need && mine == 0);
      if (fresh) {
        const uint32_t first = nnodes;
        nnodes += (uint32_t)__popcll(fresh);
        if (nnodes > cap) {
          ok = false;
          break;
        }
        if (need && mine == 0) {
          mine = first + (uint32_t)__popcll(fresh & lanemask_lt());
#pragma unroll
          for (int w = 0; w < W; ++w) T.keys[(u64)mine * W + w] = key[w];
          T.marked[mine] = 0;
          T.label[mine] = (uint32_t)y;
          created += 1;
        }
        wave_fence();
      }
      if (need) {
        const u64 old = atomicCAS((unsigned long long*)(T.hash + (h & hmask)), (unsigned long long)slot,
                                  (unsigned long long)(tag | mine));
        if (old == slot) {
          node = mine;
          done = true;
        }
        // else another lane took the slot for another prefix: read it again
      }
    }
    if (ok && act) path[y] = node;
  }
  wave_fence();
  __syncthreads();
  return ok;
}

// ---- records ---------------------------------------------------------------

// The sorted input ids (and weight product) of the clique chosen so far.
struct Prefix {
  int32_t* ids;   // sorted, n entries
  int n;
  u64 prod;       // product of g over them (fingerprints), uniform
};

// Builds the sorted prefix from `n` input ids with weights (lane 0), into dst.
__device__ void make_prefix(const int32_t* ids, const u64* wts, int n, int32_t* dst, bool fp, Prefix& P) {
  if (lane_id() == 0) {
    for (int i = 0; i < n; ++i) {
      const int32_t v = ids[i];
      int q = i;
      while (q > 0 && dst[q - 1] > v) {
        dst[q] = dst[q - 1];
        --q;
      }
      dst[q] = v;
    }
  }
  u64 pr = 1;
  if (fp && lane_id() == 0)
    for (int i = 0; i < n; ++i) pr = mulp(pr, wts[i]);
  P.ids = dst;
  P.n = n;
  P.prod = bcast64(pr);
  __syncthreads();
}

// Writes the record prefix + {a} (+ {b}) in ascending order.
__device__ __forceinline__ void put_record(int32_t* dst, const Prefix& P, int nl, int32_t a, int32_t b) {
  int pa = 0, pb = 0;
  for (int q = 0; q < P.n; ++q) {
    const int32_t v = P.ids[q];
    pa += v < a;
    if (nl > 1) pb += v < b;
    dst[q + (a < v) + (nl > 1 && b < v)] = v;
  }
  dst[pa + (nl > 1 && b < a)] = a;
  if (nl > 1) dst[pb + (a < b)] = b;
}

// Emission state of the current root: next record slot and its end.
struct Out {
  u64 cur, end;
  bool bad;
};

// Reserves, for every lane, cnt consecutive record slots (prefix sum over the
// wave); returns the lane's first slot.  Marks the root bad (no write) past
// its end.
__device__ __forceinline__ u64 take_slots(Out& o, u64 cnt, bool& ok) {
  const int lane = lane_id();
  u64 incl = cnt;
  for (int off = 1; off < kWave; off <<= 1) {
    const u64 t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  const u64 total = __shfl(incl, kWave - 1);
  const u64 first = o.cur + incl - cnt;
  o.cur += total;
  ok = o.cur <= o.end;
  if (!ok) o.bad = true;
  return first;
}

// Every clique prefix + {v}, v in S (a set of local ids).
template <int W>
__device__ void emit_set(const IstParams& p, const Lds& s, const int32_t* oid, const u64 (&S)[W], const Prefix& P,
                         Out& o, u64& cnt, u64& fpacc) {
  const int lane = lane_id();
  const int k = p.k;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 b = S[w];
    if (!b) continue;
    const bool in = (b >> lane) & 1ull;
    bool ok;
    const u64 slot = take_slots(o, in ? 1ull : 0ull, ok);
    cnt += in ? 1ull : 0ull;
    if (in) {
      const int x = w * 64 + lane;
      if (ok) put_record(p.out + slot * (u64)k, P, 1, oid[x], 0);
      if (p.fingerprint) fpacc = addp(fpacc, mulp(P.prod, s.gl[x]));
    }
  }
}

// Every edge (x, y) of G[P], as prefix + {x, y} (Algorithm 2 / 3 at l = 2).
template <int W>
__device__ void emit_edges(const IstParams& p, const Lds& s, const int32_t* oid, const u64 (&Pr)[W], int np,
                           const Prefix& P, Out& o, u64& cnt, u64& fpacc) {
  const int lane = lane_id();
  const int k = p.k;
  for (int base = 0; base < np; base += kWave) {
    const int i = base + lane;
    u64 q[W];
    int c = 0;
    int x = 0;
    if (i < np) {
      x = s.mem[i];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        q[w] = Pr[w] & s.A[x * W + w];
        c += __popcll(q[w]);
      }
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) q[w] = 0;
    }
    bool ok;
    u64 slot = take_slots(o, (u64)c, ok);
    cnt += (u64)c;
    if (c) {
      u64 f = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 b = q[w];
        while (b) {
          const int t = __ffsll((unsigned long long)b) - 1;
          b &= b - 1;
          const int y = w * 64 + t;
          if (ok) put_record(p.out + slot * (u64)k, P, 2, oid[x], oid[y]);
          ++slot;
          if (p.fingerprint) f = addp(f, s.gl[y]);
        }
      }
      if (p.fingerprint) fpacc = addp(fpacc, mulp(P.prod, mulp(s.gl[x], f)));
    }
  }
}

// Every triangle of G[P], as prefix + {x, y, z} (Listing at l = 3).
template <int W>
__device__ void emit_triangles(const IstParams& p, const Lds& s, const int32_t* oid, const u64 (&Pr)[W], int np,
                               const Prefix& P, int32_t* pre2, Out& o, u64& cnt, u64& fpacc) {
  // per member x: the edges of G[P & A[x]] with prefix + {x}
  const int lane = lane_id();
  const int k = p.k;
  for (int base = 0; base < np; base += kWave) {
    const int i = base + lane;
    u64 q[W];
    int x = 0;
    u64 c = 0;
    if (i < np) {
      x = s.mem[i];
#pragma unroll
      for (int w = 0; w < W; ++w) q[w] = Pr[w] & s.A[x * W + w];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 b = q[w];
        while (b) {
          const int t = __ffsll((unsigned long long)b) - 1;
          b &= b - 1;
          const int y = w * 64 + t;
#pragma unroll
          for (int v = 0; v < W; ++v) c += (u64)__popcll(q[v] & s.A[y * W + v]);
        }
      }
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) q[w] = 0;
    }
    bool ok;
    u64 slot = take_slots(o, c, ok);
    cnt += c;
    if (c) {
      u64 f = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        u64 b = q[w];
        while (b) {
          const int t = __ffsll((unsigned long long)b) - 1;
          b &= b - 1;
          const int y = w * 64 + t;
          u64 fz = 0;
#pragma unroll
          for (int v = 0; v < W; ++v) {
            u64 bz = q[v] & s.A[y * W + v];
            while (bz) {
              const int tz = __ffsll((unsigned long long)bz) - 1;
              bz &= bz - 1;
              const int z = v * 64 + tz;
              if (ok) {
                // prefix + {x, y, z}: y, z into the record after placing x
                int32_t* dst = p.out + slot * (u64)k;
                const int32_t ids[3] = {oid[x], oid[y], oid[z]};
                int pos[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a) {
                  for (int q2 = 0; q2 < P.n; ++q2) pos[a] += P.ids[q2] < ids[a];
                  for (int b2 = 0; b2 < 3; ++b2) pos[a] += ids[b2] < ids[a];
                }
                for (int q2 = 0; q2 < P.n; ++q2) {
                  const int32_t v2 = P.ids[q2];
                  dst[q2 + (ids[0] < v2) + (ids[1] < v2) + (ids[2] < v2)] = v2;
                }
                for (int a = 0; a < 3; ++a) dst[pos[a]] = ids[a];
              }
              ++slot;
              if (p.fingerprint) fz = addp(fz, s.gl[z]);
            }
          }
          if (p.fingerprint) f = addp(f, mulp(s.gl[y], fz));
        }
      }
      if (p.fingerprint) fpacc = addp(fpacc, mulp(P.prod, mulp(s.gl[x], f)));
    }
  }
  (void)pre2;
}

// ---- per-wave LDS beyond the search layout ----------------------------------
struct IstLds {
  int32_t* oid;     // drows: input id of each local vertex
  int32_t* cid;     // k + 1: input ids of the chosen vertices (depth order)
  u64* cw;          // k + 1: their weights
  int32_t* pre;     // k + 1: sorted prefix of records
  uint32_t* cur_t;  // k: node t_i being expanded at depth j (dense frames)
  uint32_t* sib;    // k: current l-sibling target at depth j
  u64* recs;        // k: record cursor when the child of depth j was pushed
  uint8_t* kind;    // k: 1 = ListingDense
  uint32_t* rs_t;   // k + 1: ListingIST walk: chain position per level
  uint8_t* rs_l;    // k + 1
  int32_t* rs_lab;  // k + 1: label (input id) taken at each level
  u64* rs_w;        // k + 1: its weight
};

__device__ IstLds carve_ist(char* base, int k, int drows) {
  IstLds x;
  char* c = base;
  auto take = [&](size_t bytes) {
    char* r = c;
    c += align8(bytes);
    return r;
  };
  x.oid = (int32_t*)take(4 * (size_t)drows);
  x.cid = (int32_t*)take(4 * (size_t)(k + 1));
  x.cw = (u64*)take(8 * (size_t)(k + 1));
  x.pre = (int32_t*)take(4 * (size_t)(k + 1));
  x.cur_t = (uint32_t*)take(4 * (size_t)k);
  x.sib = (uint32_t*)take(4 * (size_t)k);
  x.recs = (u64*)take(8 * (size_t)k);
  x.kind = (uint8_t*)take((size_t)k);
  x.rs_t = (uint32_t*)take(4 * (size_t)(k + 1));
  x.rs_l = (uint8_t*)take((size_t)(k + 1));
  x.rs_lab = (int32_t*)take(4 * (size_t)(k + 1));
  x.rs_w = (u64*)take(8 * (size_t)(k + 1));
  return x;
}

// ListingIST(t, l, C) (Algorithm 4), C = the nc chosen vertices in x.cid:
// emits every l-clique of the node's subgraph with C, walking l-child links
// (cliques with the node's label) and l-sibling links (the rest) down to
// l = 1, where a node's cliques are its members.
template <int W>
__device__ void listing_ist(const IstParams& p, const Lds& s, const IstLds& x, const Trie& T, uint32_t t0, int l0,
                            int nc, Out& o, u64& cnt, u64& fpacc, u64& retrieved) {
  const int k = p.k;
  const bool fp = p.fingerprint != 0;
  if (t0 == kTrieRoot) return;
  u64 key[W];
  Prefix P;
  const u64 before = cnt;
  if (l0 == 1) {
#pragma unroll
    for (int w = 0; w < W; ++w) key[w] = ld_wave(T.keys + (u64)t0 * W + w);
    make_prefix(x.cid, x.cw, nc, x.pre, fp, P);
    emit_set<W>(p, s, x.oid, key, P, o, cnt, fpacc);
    retrieved += cnt - before;
    return;
  }
  int dep = 0;
  if (lane_id() == 0) {
    x.rs_t[0] = t0;
    x.rs_l[0] = (uint8_t)l0;
  }
  __syncthreads();
  while (dep >= 0) {
    const uint32_t t = x.rs_t[dep];
    const int l = x.rs_l[dep];
    __syncthreads();
    if (t == kTrieRoot) {
      --dep;
      continue;
    }
    uint32_t lab = 0;
    if (lane_id() == 0) lab = tget32(T.label + t);
    lab = bcast32(lab);
    const uint32_t child = node_lc(T, k, t, l);
    const uint32_t next = node_ls(T, k, t, l);
    if (lane_id() == 0) {
      x.rs_t[dep] = next;
      x.rs_lab[dep] = x.oid[lab];
      x.rs_w[dep] = fp ? s.gl[lab] : 0ull;
    }
    __syncthreads();
    if (child == kTrieRoot) continue;
    if (l - 1 == 1) {
      // C + the labels taken at levels 0..dep + each member of the child
      if (lane_id() == 0) {
        for (int q = 0; q <= dep; ++q) {
          x.cid[nc + q] = x.rs_lab[q];
          x.cw[nc + q] = x.rs_w[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < W; ++w) key[w] = ld_wave(T.keys + (u64)child * W + w);
      make_prefix(x.cid, x.cw, nc + dep + 1, x.pre, fp, P);
      emit_set<W>(p, s, x.oid, key, P, o, cnt, fpacc);
    } else {
      if (lane_id() == 0) {
        x.rs_t[dep + 1] = child;
        x.rs_l[dep + 1] = (uint8_t)(l - 1);
      }
      __syncthreads();
      ++dep;
    }
  }
  retrieved += cnt - before;
}

// Criterion (1) for a child frame needing l vertices from P (n members, e
// edges): ListingDense when l >= 4 and 2 e l > (l - 1) n^2; memo = 2 takes
// ListingDense wherever l >= 2, memo = 0 never.
__device__ __forceinline__ bool dense_frame(int memo, int l, u64 n, u64 e) {
  if (memo == 2) return l >= 2;
  if (memo != 1 || l < 4 || n < 2) return false;
  return 2ull * e * (u64)l > (u64)(l - 1) * n * n;
}

template <int W>
__device__ __forceinline__ u64 edges_of(const Lds& s, const u64 (&Pr)[W], int np) {
  u64 m = 0;
  for (int i = lane_id(); i < np; i += kWave) {
    const int y = s.mem[i];
#pragma unroll
    for (int w = 0; w < W; ++w) m += (u64)__popcll(Pr[w] & s.A[y * W + w]);
  }
  return wave_sum(m);
}

template <int W>
__device__ __forceinline__ int members_of(const Lds& s, const u64 (&Pr)[W]) {
  const int lane = lane_id();
  int np = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const u64 bw = Pr[w];
    if ((bw >> lane) & 1ull) s.mem[np + __popcll(bw & lanemask_lt())] = (uint16_t)(w * 64 + lane);
    np += __popcll(bw);
  }
  __syncthreads();
  return np;
}

template <int W>
__device__ __forceinline__ int lowest(const u64 (&Pr)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (Pr[w]) return w * 64 + __ffsll((unsigned long long)Pr[w]) - 1;
  return -1;
}

template <int W>
__global__ __launch_bounds__(64, 1) void k_list_ist(IstParams p) {
  extern __shared__ __align__(16) char smem[];
  const int lane = lane_id();
  const int k = p.k;
  const bool fp = p.fingerprint != 0;
  const Lds s = carve<W>(smem, k, p.fingerprint, p.drows);
  const IstLds x = carve_ist(smem + lds_bytes(W, k, p.fingerprint, p.drows), k, p.drows);
  const Trie T = trie_view<W>(p);
  const int D = p.drows;
  u64 tot_cnt = 0, tot_fp = 0, n_frames = 0, n_dense = 0, n_nodes = 0, n_full = 0, n_hits = 0, n_retr = 0;
  u64 n_roots = 0, n_pruned = 0;
  for (;;) {
    uint32_t ri = 0;
    if (lane == 0) ri = atomicAdd(p.cursor, 1u);
    ri = bcast32(ri);
    if (ri >= (uint32_t)p.nroots) break;
    const int32_t r = p.roots[p.root_begin + (int32_t)ri];
    const int32_t beg = p.dptr[r];
    const int d = p.dptr[r + 1] - beg;
    ++n_roots;
    build_subgraph<W>(s, p.dptr, p.dcol, p.gw, p.orig, x.oid, beg, d);
    if (p.prune && k >= 3) {
      const int rr = soft_embed_levels<W>(s, d, k);
      __syncthreads();
      if (rr < k) {
        ++n_pruned;
        if (p.rec_cnt[ri] != 0 && lane == 0) atomicOr(p.err, 1);
        continue;
      }
    } else {
      for (int i = lane; i < d; i += kWave) s.rcap[i] = 63;
      __syncthreads();
    }
    Out o{p.rec_off[ri], p.rec_off[ri] + p.rec_cnt[ri], false};
    u64 cnt = 0, fpacc = 0;
    const u64 epoch = p.epoch_base + (u64)ri;
    uint32_t nnodes = 1;  // node 0: the root of the trie
    // frame 0: G_u, l = k - 1, C = {u}
    if (lane == 0) {
      x.cid[0] = p.orig[r];
      x.cw[0] = fp ? p.gw[r] : 0ull;
    }
    if (lane < W) {
      const int lo_b = lane * 64;
      s.stP[lane] = d >= lo_b + 64 ? ~0ull : (d <= lo_b ? 0ull : ((1ull << (d - lo_b)) - 1));
    }
    __syncthreads();
    {
      u64 P0[W];
#pragma unroll
      for (int w = 0; w < W; ++w) P0[w] = s.stP[w];
      const int np0 = members_of<W>(s, P0);
      const u64 e0 = (p.memo == 1 && k - 1 >= 4) ? edges_of<W>(s, P0, np0) : 0;
      if (lane == 0) x.kind[0] = dense_frame(p.memo, k - 1, (u64)np0, e0) ? 1 : 0;
    }
    __syncthreads();
    int j = 0;
    enum { ENTER, NEXT, FINISH } mode = ENTER;
    while (true) {
      const int l = k - 1 - j;
      if (mode == ENTER) {
        ++n_frames;
        u64 Pr[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Pr[w] = s.stP[j * W + w];
        Prefix P;
        if (l == 1) {  // k = 2: C + each vertex
          make_prefix(x.cid, x.cw, j + 1, x.pre, fp, P);
          emit_set<W>(p, s, x.oid, Pr, P, o, cnt, fpacc);
          mode = FINISH;
          continue;
        }
        bool dense = x.kind[j] != 0;
        __syncthreads();
        if (dense) {
          u64 made = 0;
          const bool ok = trie_insert<W>(T, Pr, s.pos, T.path + (u64)j * D, epoch, nnodes, p.node_cap, p.hmask, made);
          n_nodes += made;
          if (!ok) {
            dense = false;
            ++n_full;
            if (lane == 0) x.kind[j] = 0;
          } else {
            ++n_dense;
          }
          __syncthreads();
        }
        const int np = members_of<W>(s, Pr);
        if (l == 2 || (l == 3 && !dense)) {
          make_prefix(x.cid, x.cw, j + 1, x.pre, fp, P);
          if (l == 2) emit_edges<W>(p, s, x.oid, Pr, np, P, o, cnt, fpacc);
          else emit_triangles<W>(p, s, x.oid, Pr, np, P, x.pre, o, cnt, fpacc);
          if (l == 2 && dense) {
            // Algorithm 3 at l = 2: link every unmarked t_i of P's path to
            // the node of the string of x_i's out-neighbours in P
            uint32_t sib = kTrieRoot;
            for (int i = np - 1; i >= 0; --i) {
              const int xi = s.mem[i];
              uint32_t t = 0;
              if (lane == 0) t = tget32(T.path + (u64)j * D + xi);
              t = bcast32(t);
              u64 Q[W];
              int c = 0;
#pragma unroll
              for (int w = 0; w < W; ++w) {
                Q[w] = Pr[w] & s.A[xi * W + w];
                c += __popcll(Q[w]);
              }
              if (memoised(T, t, 2)) {
                if (node_lc(T, k, t, 2) != kTrieRoot) sib = t;
                continue;
              }
              set_ls(T, k, t, 2, sib);
              const bool sib_ok = memoised(T, sib, 2);
              if (c == 0) {
                set_lc(T, k, t, 2, kTrieRoot);
                if (sib_ok) set_marked(T, t, 2);
                continue;
              }
              // the string of G_{x_i} (path kept in the next depth's row)
              u64 made = 0;
              const bool ok = j + 1 < k ? trie_insert<W>(T, Q, s.pos, T.path + (u64)(j + 1) * D, epoch, nnodes,
                                                          p.node_cap, p.hmask, made)
                                        : false;
              n_nodes += made;
              // trie_insert reused s.pos; the members of P are still in s.mem
              if (ok) {
                const int lo = lowest<W>(Q);
                uint32_t tstar = 0;
                if (lane == 0) tstar = tget32(T.path + (u64)(j + 1) * D + lo);
                tstar = bcast32(tstar);
                set_lc(T, k, t, 2, tstar);
                if (sib_ok) set_marked(T, t, 2);
              } else {
                ++n_full;
              }
              sib = t;  // x_i has an out-neighbour in t_i: I(G[t_i], 2) is not empty
            }
          }
          mode = FINISH;
          continue;
        }
        if (lane < W) s.stQ[j * W + lane] = Pr[lane];
        if (lane == 0) x.sib[j] = kTrieRoot;
        __syncthreads();
        mode = NEXT;
        continue;
      }
      if (mode == NEXT) {
        // the next member of P, highest first
        int xv = -1;
        for (int w = W - 1; w >= 0; --w) {
          const u64 qw = s.stQ[j * W + w];
          if (qw) {
            xv = w * 64 + 63 - __clzll((long long)qw);
            break;
          }
        }
        __syncthreads();
        if (xv < 0) {
          mode = FINISH;
          continue;
        }
        if (lane == 0) s.stQ[j * W + (xv >> 6)] &= ~(1ull << (xv & 63));
        u64 Pn[W];
        int c = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          Pn[w] = s.stP[j * W + w] & s.A[xv * W + w];
          c += __popcll(Pn[w]);
        }
        const bool viable = c >= l - 1 && s.rcap[xv] >= l;
        const bool dense = x.kind[j] != 0;
        __syncthreads();
        if (dense) {
          uint32_t t = 0;
          if (lane == 0) t = tget32(T.path + (u64)j * D + xv);
          t = bcast32(t);
          if (memoised(T, t, l)) {
            // Algorithm 3: t_i is l-memoised -- retrieve I(G[t_i], l)
            const uint32_t lc = node_lc(T, k, t, l);
            if (lane == 0) {
              x.cid[j + 1] = x.oid[xv];
              x.cw[j + 1] = fp ? s.gl[xv] : 0ull;
            }
            __syncthreads();
            ++n_hits;
            listing_ist<W>(p, s, x, T, lc, l - 1, j + 2, o, cnt, fpacc, n_retr);
            if (lc != kTrieRoot && lane == 0) x.sib[j] = t;
            __syncthreads();
            continue;
          }
          const uint32_t sib = x.sib[j];
          __syncthreads();
          set_ls(T, k, t, l, sib);
          if (!viable) {
            // the branch is pruned: no (l-1)-clique in G_{x_i}
            set_lc(T, k, t, l, kTrieRoot);
            if (memoised(T, sib, l)) set_marked(T, t, l);
            continue;
          }
          if (lane == 0) x.cur_t[j] = t;
        } else if (!viable) {
          continue;
        }
        // push the child G[P & A[x]]
        const int np2 = members_of<W>(s, Pn);
        const u64 e2 = (p.memo == 1 && l - 1 >= 4) ? edges_of<W>(s, Pn, np2) : 0;
        const bool child_dense = dense || dense_frame(p.memo, l - 1, (u64)np2, e2);
        if (lane == 0) {
          s.stX[j] = (uint16_t)xv;
          x.cid[j + 1] = x.oid[xv];
          x.cw[j + 1] = fp ? s.gl[xv] : 0ull;
          x.kind[j + 1] = child_dense ? 1 : 0;
          x.recs[j] = o.cur;
        }
        if (lane < W) s.stP[(j + 1) * W + lane] = Pn[lane];
        __syncthreads();
        ++j;
        mode = ENTER;
        continue;
      }
      // FINISH: back to the parent frame
      if (j == 0) break;
      const bool child_dense = x.kind[j] != 0;
      const int lowc = [&] {
        u64 Pc[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Pc[w] = s.stP[j * W + w];
        return lowest<W>(Pc);
      }();
      const int cj = j;
      --j;
      const int lp = k - 1 - j;
      if (x.kind[j]) {
        const uint32_t t = x.cur_t[j];
        __syncthreads();
        if (child_dense && lowc >= 0) {
          // l-child link from the node t'_d of the child's whole string
          uint32_t td = 0;
          if (lane == 0) td = tget32(T.path + (u64)cj * D + lowc);
          td = bcast32(td);
          const uint32_t lc_td = node_lc(T, k, td, lp - 1);
          const uint32_t lct = (lp - 1 == 1 || lc_td != kTrieRoot) ? td : node_ls(T, k, td, lp - 1);
          set_lc(T, k, t, lp, lct);
          const uint32_t lst = node_ls(T, k, t, lp);
          if (memoised(T, td, lp - 1) && memoised(T, lst, lp)) set_marked(T, t, lp);
          if (lct != kTrieRoot && lane == 0) x.sib[j] = t;
        } else {
          // the child ran as Listing: t stays unmarked
          if (o.cur > x.recs[j] && lane == 0) x.sib[j] = t;
        }
        __syncthreads();
      }
      mode = NEXT;
    }
    if (o.cur != o.end || o.bad) {
      if (lane == 0) atomicOr(p.err, 1);
    }
    tot_cnt += cnt;
    tot_fp = addp(tot_fp, fpacc);
    if (p.inspect) {
      // ListingIST(t, ret_l, {root}) for the node t whose set is ret_key
      u64 key[W];
#pragma unroll
      for (int w = 0; w < W; ++w) key[w] = p.ret_key[w];
      uint32_t node = 0;
      bool any = false;
#pragma unroll
      for (int w = 0; w < W; ++w) any = any || key[w] != 0;
      if (any && lane == 0) {
        const u64 tag = (epoch & kEpochMask) << 24;
        u64 h = set_hash<W>(key);
        for (uint32_t probe = 0; probe <= (uint32_t)p.hmask; ++probe, ++h) {
          const u64 slot = ld_wave(T.hash + (h & p.hmask));
          if ((slot & ~0xFFFFFFull) != tag) break;
          const uint32_t nd = (uint32_t)(slot & 0xFFFFFFull);
          bool eq = true;
          for (int w = 0; w < W; ++w) eq = eq && ld_wave(T.keys + (u64)nd * W + w) == key[w];
          if (eq) {
            node = nd;
            break;
          }
        }
      }
      node = bcast32(node);
      Out ro{p.ret_off, p.ret_off + p.ret_cap, false};
      u64 rc = 0, rf = 0, rr = 0;
      if (node != kTrieRoot) listing_ist<W>(p, s, x, T, node, p.ret_l, 1, ro, rc, rf, rr);
      if (lane == 0) {
        u64* w = p.wave_out + (u64)blockIdx.x * kOutW;
        w[11] = nnodes;
        w[12] = node;
        w[13] = ro.cur - p.ret_off;
        w[14] = ro.bad ? 1 : 0;
      }
    }
  }
  const u64 c_all = wave_sum(tot_cnt);
  const u64 f_all = wave_sum_p(tot_fp);
  const u64 nodes = wave_sum(n_nodes);
  n_retr = wave_sum(n_retr);
  if (lane == 0) {
    u64* w = p.wave_out + (u64)blockIdx.x * kOutW;
    w[0] = c_all;
    w[1] = 0;
    w[2] = f_all;
    w[3] = n_roots;
    w[4] = n_pruned;
    w[5] = n_frames;
    w[6] = n_dense;
    w[7] = nodes;
    w[8] = n_full;
    w[9] = n_hits;
    w[10] = n_retr;
  }
}

}  // namespace

int ist_list_launch(int W, const IstParams& prm, int grid, size_t lds, hipStream_t s) {
  const void* fn = nullptr;
  switch (W) {
    case 1: fn = (const void*)k_list_ist<1>; break;
    case 2: fn = (const void*)k_list_ist<2>; break;
    case 3: fn = (const void*)k_list_ist<3>; break;
    case 4: fn = (const void*)k_list_ist<4>; break;
    case 5: fn = (const void*)k_list_ist<5>; break;
    case 6: fn = (const void*)k_list_ist<6>; break;
    case 8: fn = (const void*)k_list_ist<8>; break;
    default: fn = (const void*)k_list_ist<16>; break;
  }
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return DIST_E_DEVICE;
  IstParams p = prm;
  void* args[] = {&p};
  if (hipLaunchKernel(fn, dim3(grid), dim3(64), args, lds, s) != hipSuccess) return DIST_E_DEVICE;
  return hipGetLastError() == hipSuccess ? DIST_OK : DIST_E_DEVICE;
}

int ist_occupancy(int W, size_t lds) {
  const void* fn = nullptr;
  switch (W) {
    case 1: fn = (const void*)k_list_ist<1>; break;
    case 2: fn = (const void*)k_list_ist<2>; break;
    case 3: fn = (const void*)k_list_ist<3>; break;
    case 4: fn = (const void*)k_list_ist<4>; break;
    case 5: fn = (const void*)k_list_ist<5>; break;
    case 6: fn = (const void*)k_list_ist<6>; break;
    case 8: fn = (const void*)k_list_ist<8>; break;
    default: fn = (const void*)k_list_ist<16>; break;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, lds) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

size_t ist_lds_bytes(int W, int k, int fp, int drows) {
  size_t b = lds_bytes(W, k, fp, drows);
  auto a8 = [](size_t v) { return (v + 7) & ~(size_t)7; };
  b += a8(4 * (size_t)drows) + a8(4 * (size_t)(k + 1)) + a8(8 * (size_t)(k + 1)) + a8(4 * (size_t)(k + 1)) +
       a8(4 * (size_t)k) + a8(4 * (size_t)k) + a8(8 * (size_t)k) + a8((size_t)k) + a8(4 * (size_t)(k + 1)) +
       a8((size_t)(k + 1)) + a8(4 * (size_t)(k + 1)) + a8(8 * (size_t)(k + 1));
  return b;
}
