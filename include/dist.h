/*
 * dist.h -- C ABI of libdist: k-clique counting and listing on one AMD
 * Instinct MI355X (gfx950), after DIST (Nam, Jang, Park, Yang, Long:
 * "DIST: Efficient k-Clique Listing via Induced Subgraph Trie").
 *
 * The problem (Section II-A, Definition "k-clique listing"): given a simple
 * undirected graph G and an integer k, list all k-subsets of V whose
 * members are pairwise adjacent.  The library follows the paper's method:
 *
 *   1. orient G into a DAG by a total order (Section II-A; degeneracy order
 *      as in Algorithm 2, or degree order);
 *   2. for every root vertex u, build the subgraph induced by its
 *      out-neighbours (the 1-induced subgraph of Section IV) -- here as
 *      adjacency bitmaps in LDS;
 *   3. search it recursively for (k-1)-cliques (Algorithms 1 and 2),
 *      pruning a branch u when the soft-embedding bound r_{G'}(u) of
 *      Algorithm 5 on G' = G[N(u) u {u}] is below the clique size still
 *      needed (Section V, Lemma 1, Theorem 2);
 *   4. on dense branches (criterion (1) of Section IV) memoise the number
 *      of l-cliques of every identifying-string prefix met (the nodes of
 *      the Induced Subgraph Trie, Algorithm 3) and reuse it instead of
 *      recomputing (the retrieval of Algorithm 4, in counting form).
 *
 * Results.  count = |K_k(G)| as an unsigned 128-bit integer (count_hi:
 * count_lo); fp = sum over k-cliques C of prod_{v in C} g(v) mod (2^61-1),
 * g(v) = 1 + (splitmix64_next(0x44495354 ^ v) mod (2^61 - 2)) where v is the
 * vertex's id in the caller's input and splitmix64_next is one step of
 * SplitMix64 (Steele, Lea, Flood 2014).  fp does not depend on the order in
 * which cliques are found, and any change of the clique set changes it
 * except with probability <= k / (2^61 - 2).
 *
 * Threading: every call is synchronous on the given HIP stream (NULL = the
 * default stream) and returns when its results are in host memory.  Calls
 * that share a dist_graph may run concurrently on different host threads
 * only if they also use different streams.  Errors are returned as status
 * codes; no call aborts the process.
 */
#ifndef DIST_H
#define DIST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DIST_OK 0
#define DIST_E_INVALID 1     /* malformed CSR: unsorted row, duplicate, self-loop,
                                asymmetric, id out of range, n or nnz >= 2^31,
                                NULL pointer where one is required */
#define DIST_E_K 2           /* k < 1 or k > DIST_K_MAX */
#define DIST_E_NOMEM 3       /* device or host allocation failed */
#define DIST_E_DEVICE 4      /* a HIP runtime call failed */
#define DIST_E_OVERFLOW 5    /* count_hi != 0: the 128-bit result is still exact
                                but does not fit the low word */
#define DIST_E_CANCELLED 6   /* the sink returned nonzero, or the deadline in
                                dist_config.deadline_ms passed; results partial */
#define DIST_E_UNSUPPORTED 7 /* a root's out-degree exceeds DIST_MAX_OUTDEG */
#define DIST_E_SCRATCH 8     /* dist_count_noalloc: the call's launch plan exceeds
                                DIST_NOALLOC_PLAN_SEGS segments */

#define DIST_K_MAX 64
#define DIST_MAX_OUTDEG 1024  /* widest per-root subgraph (16 words per bitmap row) */
/* A root's subgraph rows take the narrowest of these widths (64-bit words)
 * that holds its out-degree. */
#define DIST_WIDTH_CLASSES 8
#define DIST_WIDTHS {1, 2, 3, 4, 5, 6, 8, 16}

/* ---- types --------------------------------------------------------------- */

/* Opaque device-resident oriented graph, owned by the library. */
typedef struct dist_graph dist_graph;

/* Order used by dist_orient (Section II-A). */
#define DIST_ORDER_DEGREE 0      /* (degree, id) ascending */
#define DIST_ORDER_DEGENERACY 1  /* bulk minimum-degree peeling: (round, id) ascending;
                                    every out-degree is at most the degeneracy */
#define DIST_ORDER_INPUT 2       /* the caller's numbering: id ascending (an order
                                    computed elsewhere, e.g. the worked example's) */

/* Switches of the search.  All of them leave count and fp unchanged (the
 * paper's Theorem 1, Lemma 1 and Theorem 2); they only change the work. */
typedef struct {
  int32_t memo;          /* 1 (default): memoise dense branches (Section IV);
                            0: plain search everywhere (Algorithm 1);
                            2: memoise every branch that still needs >= 3
                               vertices, ignoring criterion (1) */
  int32_t prune;         /* 1 (default): soft-embedding pruning (Section V);
                            0: off */
  int32_t fingerprint;   /* 1 (default): compute fp; 0: fp reported as 0 */
  int32_t memo_entries;  /* memo table entries per wave (power of two); 0 = auto */
  int64_t memo_bytes;    /* total memo budget in bytes; 0 = auto (16 GiB) */
  int64_t deadline_ms;   /* stop after this many milliseconds of kernel time
                            and return DIST_E_CANCELLED; 0 = no deadline */
  int32_t chunk_work;    /* work-unit size for roots with more than 64
                            out-neighbours: such a root is split into ranges of
                            max(1, chunk_work / d) depth-1 children that
                            different wavefronts take; 0 = auto (k <= 6: as
                            1024; deeper: ranges worth about
                            512 / (d/64)^(k-3) children, so light roots stay
                            whole and heavy ones split per child) */
  int32_t grid_pct;      /* batches: percent of the full persistent grid a
                            launch may use (so that batches of several streams
                            share the device); 0 = 100 */
  int32_t budget_from_pair_start; /* batches: 1 = a pair's deadline runs from
                            the moment its first work unit starts on the
                            device; 0 (default) = from the batch start */
  int32_t min_width;     /* smallest bitmap width in words (one of DIST_WIDTHS)
                            used for a root; a larger value merges the small
                            width classes of a batch into fewer launches;
                            0 = 1 */
  int32_t sub_units;     /* k >= 6: each unit of depth-1 children is shared by
                            this many work units, each taking every
                            sub_units-th surviving depth-2 child (results do
                            not depend on it); 0 = auto (more for wide roots
                            at large k, up to 32); larger values count as 32 */
  int32_t trie_nodes;    /* listing: nodes of the Induced Subgraph Trie per
                            wavefront (< 2^24); 0 = auto (32,768).  A frame
                            whose string does not fit lists without the trie
                            (results do not depend on it) */
  int64_t list_bytes;    /* listing: device record buffer in bytes; 0 = auto
                            (512 MiB).  Roots are listed in batches whose
                            records fit it; one root's records must fit */
  int64_t trie_tau;      /* counting with memo != 0: 0 = each root keeps its
                            own memo entries (keyed by the root's local ids);
                            tau > 0 = the Induced Subgraph Trie is shared by
                            the consecutive roots a wavefront takes (it takes
                            runs of 8 work units), Section VI: nodes are
                            keyed by their vertex sets as global ranks (sets
                            of up to 60 vertices), the table is cleared before
                            the next root once more than tau nodes were
                            inserted since the last clear (soft bound), and
                            no node is inserted past 2 tau (hard bound).
                            Results do not depend on it */
  int32_t edge_units;    /* dist_count / dist_count_ex: EdgeParallel work
                            units (Section VII-D).  W in DIST_WIDTHS: every
                            root whose subgraph takes at least W words is
                            searched as one unit per arc (u, v), over
                            G[N+(u) & N+(v)] for (k - 2)-cliques, each unit
                            in the width class of its own set (a pre-pass
                            builds G_u once to find the sets); 0 = auto
                            (W = 4 for k >= 5, off for k < 5); -1 = off.  Ignored with trie_tau > 0,
                            k < 4 and by dist_count_noalloc, dist_count_all
                            and the batched calls.  Results do not depend
                            on it; work counters count the arcs as roots */
  int32_t reserved;      /* must be 0 */
} dist_config;

typedef struct {
  uint64_t count_lo, count_hi; /* number of k-cliques, 128-bit */
  uint64_t fp;                 /* fingerprint in [0, 2^61 - 1) */
} dist_result;

/* Work counters of the last dist_count / dist_count_ex on this graph. */
typedef struct {
  uint64_t roots;         /* roots searched (out-degree >= k - 1) */
  uint64_t roots_pruned;  /* roots dropped by the soft-embedding test */
  uint64_t frames;        /* search-tree nodes expanded */
  uint64_t word_ops;      /* 64-bit AND+popcount operations on bitmap words */
  uint64_t leaf_bits;     /* set bits visited to form fingerprint sums */
  uint64_t memo_lookups, memo_hits, memo_inserts;
  uint64_t subgraph_arcs; /* arcs read from HBM to build per-root bitmaps */
  double kernel_ms;       /* device time of the search launches */
  /* the same, split by bitmap width class: W = 1, 2, 3, 4, 5, 6, 8, 16 words
     (DIST_WIDTHS) */
  double bucket_ms[DIST_WIDTH_CLASSES];
  uint64_t bucket_roots[DIST_WIDTH_CLASSES];
  uint64_t bucket_word_ops[DIST_WIDTH_CLASSES];
  uint64_t bucket_leaf_bits[DIST_WIDTH_CLASSES];
  uint64_t bucket_arcs[DIST_WIDTH_CLASSES];
} dist_stats;

typedef struct {
  int32_t n;
  int64_t m;              /* undirected edges = DAG arcs */
  int32_t order_mode;
  int32_t max_outdeg;
  int32_t order_bound;    /* degeneracy mode: largest peeling level reached
                             (= degeneracy); degree mode: max out-degree */
  double orient_ms;       /* device time of dist_orient */
} dist_graph_info;

/* Receives listed cliques: n_cliques rows of k input ids, each row in
 * ascending order.  The buffer is valid only during the call.  Return 0 to
 * continue, nonzero to stop (dist_list then returns DIST_E_CANCELLED). */
typedef int (*dist_sink)(const int32_t* cliques, uint64_t n_cliques, int k,
                         void* user);

/* ---- entry points -------------------------------------------------------- */

/* Default switches: memo 1, prune 1, fingerprint 1, auto memo sizes, no
 * deadline. */
void dist_config_init(dist_config* cfg);

/* Orient the graph (Section II-A; Algorithm 2, first line).
 * row_ptr: int32[n+1], col: int32[nnz]; host or device memory (detected);
 * the rows must be strictly increasing, symmetric, without self-loops.
 * nnz = row_ptr[n] = 2|E|.  The input is copied; the caller keeps
 * ownership.  order_mode: DIST_ORDER_DEGREE, DIST_ORDER_DEGENERACY or
 * DIST_ORDER_INPUT.
 * cfg: switches stored with the graph (NULL = defaults).  On success *out
 * owns a device-resident DAG (ranks, out-lists sorted by rank, per-vertex
 * fingerprint weights, roots sorted by out-degree descending) until
 * dist_graph_free.  Errors: DIST_E_INVALID (checked on the device),
 * DIST_E_NOMEM, DIST_E_DEVICE. */
int dist_orient(const int32_t* row_ptr, const int32_t* col, int32_t n,
                int64_t nnz, int order_mode, const dist_config* cfg,
                void* hip_stream, dist_graph** out);

/* Count the k-cliques of g (Algorithms 2-5 in counting form).  Writes *out
 * (host memory).  Returns DIST_OK, DIST_E_OVERFLOW (result still exact),
 * DIST_E_K, DIST_E_UNSUPPORTED, DIST_E_CANCELLED or DIST_E_DEVICE.
 * Edge cases: k = 1 gives n, k = 2 gives |E|, k above the clique number 0. */
int dist_count(const dist_graph* g, int k, void* hip_stream, dist_result* out);

/* dist_count with per-call switches (cfg NULL = the graph's) and an
 * optional per-root breakdown: if per_root is non-NULL (device or host
 * memory, 3*n uint64 words), per_root[3v..3v+2] receives {count_lo,
 * count_hi, fp} of the k-cliques whose minimum vertex under g's order is
 * input vertex v (zero for vertices that are not roots). */
int dist_count_ex(const dist_graph* g, int k, const dist_config* cfg,
                  uint64_t* per_root, void* hip_stream, dist_result* out);

/* Every clique size at once, by pivoting (the exact pivot-based counter the
 * paper cites among related work, Section II-B: Jain and Seshadhri, "The
 * Power of Pivoting for Exact Clique Counting").  For each root u the
 * cliques of G[N+(u)] are represented once each in a tree of (held, pivot)
 * vertex sets; a leaf with held set H (u included) and pivot set Q holds,
 * for every k, C(|Q|, k - |H|) k-cliques with fingerprint sum
 * prod_{v in H} g(v) * e_{k-|H|}(g(Q)).  No clique is enumerated, so dense
 * cores count in time near their tree size rather than their clique count.
 * out[k] (host memory, kmax + 1 entries) receives the count and fp of the
 * k-cliques for k = 0 .. kmax (out[0] = 0, out[1] = n, out[2] = |E|);
 * 1 <= kmax <= DIST_ALL_K_MAX (so every C(|Q|, j) is exact in 128 bits).  per_root (optional, host or device, 3 * n
 * words) receives, for k = per_root_k (2 .. kmax), each root's count and fp
 * as in dist_count_ex.  cfg (NULL = the graph's): fingerprint and
 * deadline_ms apply, and sub_units > 0 sets how many work units share each
 * root (0 = auto: launches with few roots per wavefront split them, up to
 * 64; results do not depend on it).  Returns DIST_OK, DIST_E_OVERFLOW (some count >= 2^64;
 * results exact), DIST_E_CANCELLED (deadline; results partial), DIST_E_K,
 * DIST_E_UNSUPPORTED, DIST_E_NOMEM or DIST_E_DEVICE. */
#define DIST_ALL_K_MAX 16
int dist_count_all(const dist_graph* g, int kmax, const dist_config* cfg,
                   uint64_t* per_root, int per_root_k, void* hip_stream,
                   dist_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dist_count
 * that allocates nothing.  It calls no hipMalloc, hipFree, pinned-memory or
 * other allocating routine; everything the kernels need beyond the graph and
 * *out (unit cursors, abort flag, per-wave results of up to
 * DIST_NOALLOC_WAVES resident waves -- a larger grid is clamped -- and the
 * launch plan of up to DIST_NOALLOC_PLAN_SEGS segments) lives in one static
 * device block of 0.55 MB per GPU, held until the process ends.  The
 * memo table is not used (cfg->memo is ignored: it is a cache and changes no
 * result) and there is no per-root output; every other switch of cfg (NULL =
 * the graph's) applies.  Results and statuses are those of dist_count_ex
 * with the same switches; the device time is not measured (the kernel_ms of
 * dist_stats_get is 0).  Every call on a GPU shares that GPU's block, which
 * keeps the last call's contents (each call clears what must start at zero):
 * two calls overlapping on one GPU would race on it, so the library makes
 * its calls from several host threads take turns (each returns only after
 * its work on the stream is done).  Returns DIST_E_SCRATCH if the plan would
 * not fit (for one graph it always fits: its segments are at most its
 * distinct out-degrees, <= DIST_MAX_OUTDEG). */
#define DIST_NOALLOC_WAVES 4096
#define DIST_NOALLOC_PLAN_SEGS 1024
int dist_count_noalloc(const dist_graph* g, int k, const dist_config* cfg,
                       void* hip_stream, dist_result* out);

/* List the k-cliques of g (Definition "k-clique listing"): every clique is
 * delivered once to sink as k ascending input ids, in chunks; the order of
 * cliques is unspecified.  *out receives the count and fp of the cliques
 * delivered.  Returns DIST_E_CANCELLED if sink stopped the run.
 *
 * The search is Algorithm 2's Listing; a branch whose subgraph satisfies
 * criterion (1) of Section IV (and still needs at least 4 vertices) runs as
 * Algorithm 3's ListingDense on a per-root Induced Subgraph Trie: the
 * identifying string of each dense subgraph is inserted, its path nodes get
 * l-child and l-sibling links and Marked[l], and an l-memoised node's
 * cliques are retrieved by Algorithm 4's ListingIST instead of being
 * recomputed.  cfg->memo (dist_list_ex) selects: 1 criterion (1), 2 every
 * branch that still needs >= 2 vertices, 0 no trie (Listing only).  Counters
 * of the last run (dist_stats_get): memo_lookups = ListingDense frames,
 * memo_inserts = trie nodes created, memo_hits = retrievals from l-memoised
 * nodes, leaf_bits = cliques delivered by retrieval. */
int dist_list(const dist_graph* g, int k, dist_sink sink, void* user,
              void* hip_stream, dist_result* out);

/* dist_list with per-call switches (cfg NULL = the graph's) and flags:
 * DIST_LIST_DEVICE_ROWS hands sink device pointers (rows in device memory,
 * valid during the call) instead of copying them to the host first. */
#define DIST_LIST_DEVICE_ROWS 1
int dist_list_ex(const dist_graph* g, int k, const dist_config* cfg, int flags,
                 dist_sink sink, void* user, void* hip_stream,
                 dist_result* out);

/* Inspection of the Induced Subgraph Trie (Section IV, Definitions of the
 * l-child and l-sibling links, Algorithms 3 and 4) for one root: lists the
 * k-cliques whose minimum vertex under g's order is input vertex `root`
 * (k >= 3) with switches cfg, then runs ListingIST(t, ret_l, {root}) for the
 * trie node t whose vertex set is ret_set (a bitmap over the root's local
 * ids, 16 words; NULL or empty: no retrieval; ret_l must be k - 1, so that
 * the retrieved cliques are k-cliques).  Outputs (host memory):
 * local_ids[i] (i < *d, capacity DIST_MAX_OUTDEG): input id of local vertex
 * i (the i-th out-neighbour of root in g's order); *n_nodes trie nodes
 * (node 0 is the trie's root), at most cap + 1; per node t: sets[16 t ..]
 * its vertex set over local ids, marked[t] bit l = Marked[l], lc[k t + l]
 * and ls[k t + l] its l-child and l-sibling links (node ids; valid where
 * Marked[l]); rows (may be NULL; room for rows_cap records): the root's
 * *n_rows cliques followed by the *n_ret cliques of the retrieval, k
 * ascending input ids each.  Errors: DIST_E_INVALID, DIST_E_UNSUPPORTED (trie or rows beyond the
 * capacities), DIST_E_DEVICE. */
int dist_ist_inspect(const dist_graph* g, int k, int32_t root,
                     const dist_config* cfg, const uint64_t* ret_set, int ret_l,
                     int32_t cap, int32_t* local_ids, int32_t* d,
                     uint64_t* sets, uint64_t* marked, uint32_t* lc,
                     uint32_t* ls, int32_t* n_nodes, int32_t* rows,
                     int64_t rows_cap, int64_t* n_rows, int64_t* n_ret,
                     void* hip_stream);

/* Count many (graph, k) pairs in one persistent launch per bitmap width
 * class (at most DIST_WIDTH_CLASSES launches for the whole batch; with
 * per-pair budgets, one such set per cost tier).  gs[i], ks[i] for
 * i < n (the same graph may appear with several k); out[i] receives the
 * result of pair i.  The launch sequence is captured as a HIP graph and
 * replayed when the same batch (same graphs, ks and switches) is submitted
 * again.  Returns the first non-OK status of any pair (DIST_E_OVERFLOW is
 * reported but every result is still written). */
int dist_count_batch(const dist_graph* const* gs, const int* ks, int n,
                     void* hip_stream, dist_result* out);

/* dist_count_batch with switches (cfg NULL = defaults; memo, prune,
 * fingerprint, memo sizes, chunk_work and min_width apply to every pair),
 * use_graph = 0 to launch without graph capture, and per-pair time budgets:
 * pair_deadline_ms[i] > 0 (array may be NULL) stops pair i once that many
 * milliseconds have passed since the batch started on the device, without
 * stopping the other pairs; pair_status[i] (array may be NULL) receives DIST_OK,
 * DIST_E_OVERFLOW, DIST_E_CANCELLED (budget spent; out[i] is partial) or
 * DIST_E_UNSUPPORTED.  *ms (may be NULL) receives the device time of the
 * batch.  Batches on different streams may be issued concurrently from
 * different host threads; each stream keeps its own workspace. */
int dist_count_batch_ex(const dist_graph* const* gs, const int* ks, int n,
                        const dist_config* cfg, int use_graph,
                        const int64_t* pair_deadline_ms, void* hip_stream,
                        dist_result* out, int* pair_status, double* ms);

/* Per-pair switches of dist_count_batch_tuned; a negative field (or, for
 * min_width, 0) takes the value of the batch's cfg.  min_width: smallest
 * bitmap width in words given to the pair's roots (one of DIST_WIDTHS;
 * larger values put the pair's narrow roots into wider launches);
 * chunk_work: the pair's work-unit size (as dist_config.chunk_work; 0 =
 * automatic); memo: 0, 1 or 2 as dist_config.memo.  None of them changes a
 * result. */
typedef struct dist_pair_switches {
  int32_t min_width;
  int32_t chunk_work;
  int32_t memo;
  int32_t reserved;  /* 0 */
} dist_pair_switches;

/* dist_count_batch_ex with switches chosen per pair (sw[i] for pair i; sw
 * NULL = dist_count_batch_ex): an autotuner that picks the switches per
 * size bucket of a batch still runs the whole batch as one launch per width
 * class, captured and replayed like dist_count_batch_ex (a replay requires
 * the same switches too).  Returns DIST_E_INVALID for a switch out of range;
 * otherwise as dist_count_batch_ex. */
int dist_count_batch_tuned(const dist_graph* const* gs, const int* ks, int n,
                           const dist_config* cfg,
                           const dist_pair_switches* sw, int use_graph,
                           const int64_t* pair_deadline_ms, void* hip_stream,
                           dist_result* out, int* pair_status, double* ms);

/* Called from the thread of dist_count_batch_stream as soon as pair `pair`
 * is finished on the device (or cut off by its budget), while the rest of
 * the batch may still run.  res and status as in dist_count_batch_ex;
 * device_ms: time from the pair's first work unit starting to its last one
 * ending (the pair's service time), or -1 when the pair is reported only at
 * the end of the batch. */
typedef void (*dist_pair_done)(int pair, const dist_result* res, int status,
                               double device_ms, void* user);

/* dist_count_batch_ex without graph capture that reports every pair through
 * on_done as it completes.  Pairs are scheduled in ascending order of
 * pair_cost[i] (array may be NULL: dist_estimate_cost is used), so light
 * queries of a mixed batch finish early; with budgets from the batch start
 * (cfg->budget_from_pair_start = 0), pairs whose costs differ by more than
 * two decades go to separate launches, cheapest first.  Returns when the
 * whole batch is done; out and pair_status are filled as in
 * dist_count_batch_ex. */
int dist_count_batch_stream(const dist_graph* const* gs, const int* ks, int n,
                            const dist_config* cfg,
                            const int64_t* pair_deadline_ms,
                            const double* pair_cost, void* hip_stream,
                            dist_result* out, int* pair_status,
                            dist_pair_done on_done, void* user);

/* Upper bound on the search of (g, k): the sum over roots u of C(d+(u), k-1),
 * the number of (k-1)-subsets of each out-neighbourhood.  Used to order and
 * route queries; never changes a result. */
int dist_estimate_cost(const dist_graph* g, int k, double* out);

/* r_{G'}(u) of Algorithm 5 on G' = G[N+(u) u {u}] for every vertex u, the
 * value the top-level pruning test compares with k (Section V).  Values
 * are capped at cap (>= 1): r_out[v] = min(r_{G'}(v), cap) for input id v.
 * r_out: host or device int32[n]. */
int dist_root_soft_embed(const dist_graph* g, int cap, int32_t* r_out,
                         void* hip_stream);

/* Copy g's order to r_out (host or device int32[n]): r_out[v] = position
 * of input vertex v in the total order. */
int dist_graph_ranks(const dist_graph* g, int32_t* r_out, void* hip_stream);

int dist_graph_info_get(const dist_graph* g, dist_graph_info* out);
int dist_stats_get(const dist_graph* g, dist_stats* out);

/* Releases g (NULL is ignored).  No call using g may still be running on
 * any stream: its memory is reused at once by later allocations. */
void dist_graph_free(dist_graph* g);

const char* dist_strerror(int status);

/* Memory.  The library keeps the device and pinned host blocks it frees
 * (graphs, workspaces, staging) in a per-device cache and reuses them, so
 * that no free waits for work that other streams have in flight.
 * dist_mem_cached reports the bytes held in the cache; dist_mem_trim returns
 * them to the runtime (this waits for the device). */
int dist_mem_cached(int64_t* device_bytes, int64_t* host_bytes);
int dist_mem_trim(void);

#ifdef __cplusplus
}
#endif
#endif
