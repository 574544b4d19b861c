/*
 * oracle.h -- plain CPU reference for k-clique counting and listing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * What it computes is the plain definition of the problem (Section II-A,
 * Definition "k-clique listing"): the set of all k-subsets of V whose
 * members are pairwise adjacent.  It follows the ordering-based recursive
 * framework (Algorithm 1): orient the graph by a total order, then for every
 * vertex u extend cliques inside the out-neighbourhood of u.  There is no
 * pruning, no trie and no bitmap: out-lists are sorted arrays intersected by
 * merging, so every step can be checked against the definition by eye.
 *
 * Reported values (identical on the HIP side by construction of the
 * definition, not by shared code):
 *   count = |K_k(G)| as an unsigned 128-bit integer (lo, hi words);
 *   fp    = sum over k-cliques C of prod_{v in C} g(v)  mod p, p = 2^61 - 1;
 *   g(v)  = 1 + (splitmix64_next(0x44495354 ^ v) mod (p - 1)), v = input id,
 *           where splitmix64_next is one step of Steele/Lea/Flood's SplitMix64
 *           generator (state += 0x9E3779B97F4A7C15, then the 30/27/31
 *           xor-shift-multiply finaliser).
 *
 * Parity pins (tests/): brute force over k-subsets, C(n,k) and e_k(g) on K_n,
 * the Turan-graph closed forms, the worked example of Figure 2 / Table 2,
 * invariants on every listed clique, triangle count by trace(A^3)/6.
 */
#ifndef DIST_ORACLE_H
#define DIST_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 0 if row_ptr/col is a simple undirected graph in CSR form (rows strictly
 * increasing, no self-loops, ids in range, symmetric), nonzero otherwise. */
int oracle_validate(int32_t n, const int32_t* row_ptr, const int32_t* col);

/* The fingerprint weight g(v) defined above. */
uint64_t oracle_weight(int64_t v);

/* Count all k-cliques.  out[0] = count low 64 bits, out[1] = count high 64
 * bits, out[2] = fp.  nthreads <= 0 uses the OpenMP default.  Returns 0, or
 * nonzero on invalid input / k < 1. */
int oracle_count(int32_t n, const int32_t* row_ptr, const int32_t* col, int k,
                 int nthreads, uint64_t out[3]);

/* Per-root counts: for each roots[i], the k-cliques whose minimum vertex
 * under the total order (degree, id) ascending is roots[i].  out has
 * 3 * nroots words laid out as out[3i..3i+2] = {count lo, count hi, fp}. */
int oracle_count_roots(int32_t n, const int32_t* row_ptr, const int32_t* col,
                       int k, const int32_t* roots, int64_t nroots,
                       int nthreads, uint64_t* out);

/* List all k-cliques, each as k input ids in ascending order, rows in
 * lexicographic order.  Writes at most cap rows into out (k*cap int32) and
 * returns the total number of k-cliques (or -1 on error). */
int64_t oracle_list(int32_t n, const int32_t* row_ptr, const int32_t* col,
                    int k, int32_t* out, int64_t cap);

/* Algorithm 5 (ComputeSoftEmbeddings) on a DAG whose vertices are 0..n-1 in
 * the total order (vertex i precedes vertex j iff i < j) and whose arcs are
 * dag_ptr/dag_col (out-lists, any order).  Writes r(u) for every u. */
int oracle_soft_embed(int32_t n, const int32_t* dag_ptr, const int32_t* dag_col,
                      int32_t* r);

/* r_{G'}(u) with G' = G[N+(u) u {u}] for every vertex u of the DAG obtained
 * from the undirected CSR by the (degree, id) order: the value the pruning
 * test (Section V, applied at the top level of Algorithm 2) compares with
 * k.  Indexed by input id. */
int oracle_root_soft_embed(int32_t n, const int32_t* row_ptr,
                           const int32_t* col, int32_t* r);

/* Exact degeneracy by repeated removal of a minimum-degree vertex (ties to
 * the smallest id), Section II-A.  Writes order[i] = i-th removed vertex
 * (may be NULL) and returns the degeneracy, or -1 on error. */
int32_t oracle_degeneracy(int32_t n, const int32_t* row_ptr, const int32_t* col,
                          int32_t* order);

/* The (degree, id) rank of every vertex: rank[v] = position of v when the
 * vertices are sorted by (degree ascending, id ascending). */
int oracle_degree_rank(int32_t n, const int32_t* row_ptr, int32_t* rank);

/* Secondary reference: the same per-root results as oracle_count_roots
 * (cliques whose minimum under the (degree, id) order is roots[i]), computed
 * by pivoting instead of enumeration (Jain and Seshadhri, "The Power of
 * Pivoting for Exact Clique Counting", WSDM 2020 -- the pivot-based exact
 * counter the paper cites among related work).  Each clique of a root's
 * out-neighbourhood is represented once in a tree of (held, pivot) sets, so
 * dense neighbourhoods are counted in closed form: a leaf with h held and q
 * pivot vertices holds C(q, k - h) k-cliques, whose fingerprint sum is
 * prod(g(held)) * e_{k-h}(g(pivots)).  Used where enumeration cannot finish
 * (dense cores at k = 7, 9); pinned against oracle_count_roots, brute force
 * and closed forms.  k must be in 1..16. */
int oracle_pivot_count_roots(int32_t n, const int32_t* row_ptr, const int32_t* col,
                             int k, const int32_t* roots, int64_t nroots,
                             int nthreads, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif
