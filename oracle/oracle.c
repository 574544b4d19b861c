/*
 * oracle.c -- plain CPU reference for k-clique counting and listing.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C, OpenMP over roots.
 *
 * Method: the general framework of Algorithm 1.  The graph is oriented by
 * the total order (degree, id) ascending (Section II-A: a DAG by a total
 * order keeps the arc u->v iff u precedes v); then for every vertex u the
 * (k-1)-cliques inside the out-neighbourhood of u are found by recursive
 * extension, each step intersecting two sorted out-lists by merging.  Every
 * k-clique has exactly one minimum vertex under the order, so each is found
 * exactly once.
 */
#include "oracle.h"

#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define P61 ((uint64_t)0x1FFFFFFFFFFFFFFFull) /* 2^61 - 1 */

static uint64_t add_p(uint64_t a, uint64_t b) {
  uint64_t s = a + b; /* a, b < 2^61: no overflow */
  return s >= P61 ? s - P61 : s;
}

static uint64_t mul_p(uint64_t a, uint64_t b) {
  return (uint64_t)(((u128)a * (u128)b) % P61);
}

uint64_t oracle_weight(int64_t v) {
  /* One step of SplitMix64 from state (0x44495354 xor v). */
  uint64_t z = (0x44495354ull ^ (uint64_t)v) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 1 + z % (P61 - 1);
}

int oracle_validate(int32_t n, const int32_t* row_ptr, const int32_t* col) {
  if (n < 0 || !row_ptr) return 1;
  if (row_ptr[0] != 0) return 1;
  for (int32_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return 1;
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (v < 0 || v >= n || v == u) return 1;
      if (e > row_ptr[u] && col[e - 1] >= v) return 1; /* sorted, no dups */
      /* symmetric: u must appear in the row of v (binary search) */
      int32_t lo = row_ptr[v], hi = row_ptr[v + 1];
      while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (col[mid] < u) lo = mid + 1; else hi = mid;
      }
      if (lo >= row_ptr[v + 1] || col[lo] != u) return 1;
    }
  }
  return 0;
}

/* ---- orientation by (degree, id) ------------------------------------- */

typedef struct {
  int32_t n;
  int32_t* rank;     /* rank[v]: position of input vertex v in the order */
  int32_t* orig;     /* orig[r]: input vertex at rank r */
  int64_t* optr;     /* out-lists in rank space, sorted ascending */
  int32_t* ocol;
  uint64_t* gw;      /* gw[r] = g(orig[r]) */
} dag_t;

static int32_t* g_sort_deg; /* qsort context (single-threaded setup only) */

static int cmp_deg_id(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  int32_t dx = g_sort_deg[x], dy = g_sort_deg[y];
  if (dx != dy) return dx < dy ? -1 : 1;
  return x < y ? -1 : (x > y);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return x < y ? -1 : (x > y);
}

static int build_dag(int32_t n, const int32_t* row_ptr, const int32_t* col,
                     dag_t* d) {
  memset(d, 0, sizeof(*d));
  d->n = n;
  d->rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  d->orig = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  d->optr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  d->gw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!d->rank || !d->orig || !d->optr || !d->gw || !deg) return 1;
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = row_ptr[v + 1] - row_ptr[v];
    d->orig[v] = v;
  }
  g_sort_deg = deg;
  qsort(d->orig, (size_t)n, sizeof(int32_t), cmp_deg_id);
  for (int32_t r = 0; r < n; ++r) d->rank[d->orig[r]] = r;
  /* out-degree in rank space: neighbours of higher rank */
  for (int32_t r = 0; r < n; ++r) {
    int32_t v = d->orig[r];
    int64_t c = 0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (d->rank[col[e]] > r) ++c;
    d->optr[r + 1] = d->optr[r] + c;
  }
  d->ocol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(d->optr[n] + 1));
  if (!d->ocol) return 1;
  for (int32_t r = 0; r < n; ++r) {
    int32_t v = d->orig[r];
    int64_t p = d->optr[r];
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (d->rank[col[e]] > r) d->ocol[p++] = d->rank[col[e]];
    qsort(d->ocol + d->optr[r], (size_t)(d->optr[r + 1] - d->optr[r]),
          sizeof(int32_t), cmp_i32);
    d->gw[r] = oracle_weight(v);
  }
  free(deg);
  return 0;
}

static void free_dag(dag_t* d) {
  free(d->rank); free(d->orig); free(d->optr); free(d->ocol); free(d->gw);
}

int oracle_degree_rank(int32_t n, const int32_t* row_ptr, int32_t* rank) {
  if (n < 0) return 1;
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* ord = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!deg || !ord) { free(deg); free(ord); return 1; }
  for (int32_t v = 0; v < n; ++v) { deg[v] = row_ptr[v + 1] - row_ptr[v]; ord[v] = v; }
  g_sort_deg = deg;
  qsort(ord, (size_t)n, sizeof(int32_t), cmp_deg_id);
  for (int32_t r = 0; r < n; ++r) rank[ord[r]] = r;
  free(deg); free(ord);
  return 0;
}

/* ---- recursive extension (Algorithm 1, Listing) ---------------------- */

typedef struct {
  const dag_t* d;
  int k;
  /* per-level candidate buffers: cand[j] holds the candidate set after j+1
   * clique vertices have been chosen */
  int32_t** cand;
  int32_t* clique;   /* ranks of the chosen vertices */
  u128 count;
  uint64_t fp;
  /* listing */
  int32_t* out;
  int64_t cap;
  int64_t written;
} walk_t;

/* P (size np) holds the common out-neighbours of the |C| = depth chosen
 * vertices; l more vertices are needed; pi = prod g over C mod p. */
static void extend(walk_t* w, const int32_t* P, int32_t np, int l, int depth,
                   uint64_t pi) {
  const dag_t* d = w->d;
  if (l == 1) {
    for (int32_t i = 0; i < np; ++i) {
      w->count += 1;
      w->fp = add_p(w->fp, mul_p(pi, d->gw[P[i]]));
      if (w->out) {
        if (w->written < w->cap) {
          int32_t* row = w->out + (size_t)w->written * (size_t)w->k;
          for (int j = 0; j < depth; ++j) row[j] = d->orig[w->clique[j]];
          row[depth] = d->orig[P[i]];
          qsort(row, (size_t)w->k, sizeof(int32_t), cmp_i32);
        }
        w->written += 1;
      }
    }
    return;
  }
  int32_t* next = w->cand[depth];
  for (int32_t i = 0; i < np; ++i) {
    int32_t v = P[i];
    /* next = P intersect N+(v), by merging two sorted lists */
    int32_t nn = 0;
    int64_t a = 0, ae = np, b = d->optr[v], be = d->optr[v + 1];
    while (a < ae && b < be) {
      if (P[a] < d->ocol[b]) ++a;
      else if (P[a] > d->ocol[b]) ++b;
      else { next[nn++] = P[a]; ++a; ++b; }
    }
    if (nn < l - 1) continue;
    w->clique[depth] = v;
    extend(w, next, nn, l - 1, depth + 1, mul_p(pi, d->gw[v]));
  }
}

static int32_t max_outdeg(const dag_t* d) {
  int64_t m = 0;
  for (int32_t r = 0; r < d->n; ++r)
    if (d->optr[r + 1] - d->optr[r] > m) m = d->optr[r + 1] - d->optr[r];
  return (int32_t)m;
}

static int walk_init(walk_t* w, const dag_t* d, int k) {
  memset(w, 0, sizeof(*w));
  w->d = d;
  w->k = k;
  int32_t md = max_outdeg(d) + 1;
  w->cand = (int32_t**)calloc((size_t)k + 1, sizeof(int32_t*));
  w->clique = (int32_t*)calloc((size_t)k + 1, sizeof(int32_t));
  if (!w->cand || !w->clique) return 1;
  for (int j = 0; j <= k; ++j) {
    w->cand[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)md);
    if (!w->cand[j]) return 1;
  }
  return 0;
}

static void walk_free(walk_t* w) {
  if (w->cand)
    for (int j = 0; j <= w->k; ++j) free(w->cand[j]);
  free(w->cand);
  free(w->clique);
}

/* All k-cliques whose minimum vertex (in rank space) is r. */
static void root_task(walk_t* w, int32_t r) {
  const dag_t* d = w->d;
  w->clique[0] = r;
  if (w->k == 1) {
    int32_t one[1] = {r};
    /* the single 1-clique {r}: reuse the l == 1 branch with P = {r} */
    extend(w, one, 1, 1, 0, 1);
    return;
  }
  int32_t deg = (int32_t)(d->optr[r + 1] - d->optr[r]);
  if (deg < w->k - 1) return;
  extend(w, d->ocol + d->optr[r], deg, w->k - 1, 1, d->gw[r]);
}

int oracle_count(int32_t n, const int32_t* row_ptr, const int32_t* col, int k,
                 int nthreads, uint64_t out[3]) {
  if (k < 1 || n < 0 || !out) return 1;
  if (oracle_validate(n, row_ptr, col)) return 1;
  dag_t d;
  if (build_dag(n, row_ptr, col, &d)) { free_dag(&d); return 1; }
  u128 total = 0;
  uint64_t fp = 0;
  int err = 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
  {
    walk_t w;
    int bad = walk_init(&w, &d, k);
    if (!bad) {
#pragma omp for schedule(dynamic, 64)
      for (int32_t r = 0; r < n; ++r) root_task(&w, r);
    }
#pragma omp critical
    {
      if (bad) err = 1;
      total += w.count;
      fp = add_p(fp, w.fp);
    }
    walk_free(&w);
  }
  free_dag(&d);
  if (err) return 1;
  out[0] = (uint64_t)total;
  out[1] = (uint64_t)(total >> 64);
  out[2] = fp;
  return 0;
}

int oracle_count_roots(int32_t n, const int32_t* row_ptr, const int32_t* col,
                       int k, const int32_t* roots, int64_t nroots,
                       int nthreads, uint64_t* out) {
  if (k < 1 || n < 0 || !out || nroots < 0) return 1;
  if (oracle_validate(n, row_ptr, col)) return 1;
  for (int64_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return 1;
  dag_t d;
  if (build_dag(n, row_ptr, col, &d)) { free_dag(&d); return 1; }
  int err = 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
  {
    walk_t w;
    int bad = walk_init(&w, &d, k);
    if (!bad) {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < nroots; ++i) {
        w.count = 0;
        w.fp = 0;
        root_task(&w, d.rank[roots[i]]);
        out[3 * i + 0] = (uint64_t)w.count;
        out[3 * i + 1] = (uint64_t)(w.count >> 64);
        out[3 * i + 2] = w.fp;
      }
    }
#pragma omp critical
    { if (bad) err = 1; }
    walk_free(&w);
  }
  free_dag(&d);
  return err;
}

static int g_list_k;
static int cmp_row(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  for (int j = 0; j < g_list_k; ++j)
    if (x[j] != y[j]) return x[j] < y[j] ? -1 : 1;
  return 0;
}

int64_t oracle_list(int32_t n, const int32_t* row_ptr, const int32_t* col,
                    int k, int32_t* out, int64_t cap) {
  if (k < 1 || n < 0 || cap < 0) return -1;
  if (oracle_validate(n, row_ptr, col)) return -1;
  dag_t d;
  if (build_dag(n, row_ptr, col, &d)) { free_dag(&d); return -1; }
  walk_t w;
  if (walk_init(&w, &d, k)) { walk_free(&w); free_dag(&d); return -1; }
  w.out = out;
  w.cap = out ? cap : 0;
  for (int32_t r = 0; r < n; ++r) root_task(&w, r);
  int64_t total = (int64_t)w.count;
  if (out && total <= cap) {
    g_list_k = k;
    qsort(out, (size_t)total, sizeof(int32_t) * (size_t)k, cmp_row);
  }
  walk_free(&w);
  free_dag(&d);
  return total;
}

/* ---- Algorithm 5 ------------------------------------------------------ */

int oracle_soft_embed(int32_t n, const int32_t* dag_ptr, const int32_t* dag_col,
                      int32_t* r) {
  if (n < 0) return 1;
  int32_t maxd = 0;
  for (int32_t u = 0; u < n; ++u)
    if (dag_ptr[u + 1] - dag_ptr[u] > maxd) maxd = dag_ptr[u + 1] - dag_ptr[u];
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd + 1));
  if (!nb) return 1;
  /* vertices in descending order of the total order */
  for (int32_t u = n - 1; u >= 0; --u) {
    int32_t d = dag_ptr[u + 1] - dag_ptr[u];
    for (int32_t i = 0; i < d; ++i) {
      int32_t v = dag_col[dag_ptr[u] + i];
      if (v <= u || v >= n) { free(nb); return 1; } /* not a DAG in this order */
      nb[i] = v;
    }
    qsort(nb, (size_t)d, sizeof(int32_t), cmp_i32); /* u_1 < ... < u_d */
    r[u] = 1;
    for (int32_t i = d - 1; i >= 0; --i)   /* i := d down to 1 */
      if (r[u] <= r[nb[i]]) r[u] += 1;
  }
  free(nb);
  return 0;
}

int oracle_root_soft_embed(int32_t n, const int32_t* row_ptr,
                           const int32_t* col, int32_t* r_out) {
  if (oracle_validate(n, row_ptr, col)) return 1;
  dag_t d;
  if (build_dag(n, row_ptr, col, &d)) { free_dag(&d); return 1; }
  int32_t md = max_outdeg(&d) + 1;
  /* local DAG G' = G[N+(u) u {u}] with local ids 0 = u, 1..deg = N+(u) in
   * rank order; arcs keep their direction because ranks are preserved */
  int32_t* lptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(md + 2));
  int32_t* lcol = NULL;
  int32_t* lr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(md + 2));
  int err = (!lptr || !lr);
  for (int32_t u = 0; u < n && !err; ++u) {
    const int32_t* N = d.ocol + d.optr[u];
    int32_t deg = (int32_t)(d.optr[u + 1] - d.optr[u]);
    /* count arcs inside G' */
    int64_t arcs = deg;
    for (int32_t i = 0; i < deg; ++i) {
      int32_t v = N[i];
      for (int64_t e = d.optr[v]; e < d.optr[v + 1]; ++e) {
        int32_t x = d.ocol[e];
        int32_t lo = 0, hi = deg;
        while (lo < hi) { int32_t m = (lo + hi) / 2; if (N[m] < x) lo = m + 1; else hi = m; }
        if (lo < deg && N[lo] == x) ++arcs;
      }
    }
    free(lcol);
    lcol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs + 1));
    if (!lcol) { err = 1; break; }
    int32_t p = 0;
    lptr[0] = 0;
    for (int32_t i = 0; i < deg; ++i) lcol[p++] = i + 1;
    lptr[1] = p;
    for (int32_t i = 0; i < deg; ++i) {
      int32_t v = N[i];
      for (int64_t e = d.optr[v]; e < d.optr[v + 1]; ++e) {
        int32_t x = d.ocol[e];
        int32_t lo = 0, hi = deg;
        while (lo < hi) { int32_t m = (lo + hi) / 2; if (N[m] < x) lo = m + 1; else hi = m; }
        if (lo < deg && N[lo] == x) lcol[p++] = lo + 1;
      }
      lptr[i + 2] = p;
    }
    if (oracle_soft_embed(deg + 1, lptr, lcol, lr)) { err = 1; break; }
    r_out[d.orig[u]] = lr[0];
  }
  free(lptr); free(lcol); free(lr);
  free_dag(&d);
  return err;
}

/* ---- degeneracy ------------------------------------------------------- */

/* binary min-heap of 64-bit keys (degree << 32 | id), lazy deletion */
static void heap_push(uint64_t* h, int64_t* sz, uint64_t key) {
  int64_t i = (*sz)++;
  h[i] = key;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p] <= h[i]) break;
    uint64_t t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static uint64_t heap_pop(uint64_t* h, int64_t* sz) {
  uint64_t top = h[0];
  h[0] = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t a = 2 * i + 1, b = a + 1, m = i;
    if (a < *sz && h[a] < h[m]) m = a;
    if (b < *sz && h[b] < h[m]) m = b;
    if (m == i) break;
    uint64_t t = h[m]; h[m] = h[i]; h[i] = t;
    i = m;
  }
  return top;
}

int32_t oracle_degeneracy(int32_t n, const int32_t* row_ptr, const int32_t* col,
                          int32_t* order) {
  if (n < 0) return -1;
  int64_t m2 = row_ptr[n];
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  char* gone = (char*)calloc((size_t)n + 1, 1);
  uint64_t* heap = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + m2 + 1));
  if (!deg || !gone || !heap) { free(deg); free(gone); free(heap); return -1; }
  int64_t sz = 0;
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = row_ptr[v + 1] - row_ptr[v];
    heap_push(heap, &sz, ((uint64_t)deg[v] << 32) | (uint32_t)v);
  }
  /* repeatedly remove a vertex of minimum current degree, smallest id first */
  int32_t delta = 0, step = 0;
  while (sz > 0) {
    uint64_t key = heap_pop(heap, &sz);
    int32_t v = (int32_t)(key & 0xFFFFFFFFu);
    int32_t dv = (int32_t)(key >> 32);
    if (gone[v] || dv != deg[v]) continue; /* stale entry */
    if (dv > delta) delta = dv;
    gone[v] = 1;
    if (order) order[step] = v;
    ++step;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t x = col[e];
      if (!gone[x]) {
        deg[x] -= 1;
        heap_push(heap, &sz, ((uint64_t)deg[x] << 32) | (uint32_t)x);
      }
    }
  }
  free(deg); free(gone); free(heap);
  return delta;
}

/* ---- secondary reference: pivot-based per-root counting --------------- */

typedef struct {
  int k;
  int32_t d;              /* members of the root's out-neighbourhood */
  unsigned char* adj;     /* d x d adjacency of G[N+(root)] */
  uint64_t* w;            /* g() of each member */
  int32_t* buf;           /* candidate lists, one row of d per depth */
  unsigned char* gone;    /* members excluded by an earlier sibling */
  uint64_t* piv;          /* g() of the pivots on the current path */
  u128 count;
  uint64_t fp;
} pivot_t;

static u128 binom_u128(int q, int r) {
  if (r < 0 || r > q) return 0;
  u128 c = 1;
  for (int i = 0; i < r; ++i) c = c * (u128)(q - i) / (u128)(i + 1);
  return c;
}

/* S: candidate members (all adjacent to every held and pivot vertex so far);
 * h held vertices with weight product fh; q pivots in t->piv[0..q). */
static void pivot_rec(pivot_t* t, const int32_t* S, int32_t ns, int h, int q,
                      uint64_t fh, int depth) {
  if (h > t->k || h + q + ns < t->k) return;
  if (h == t->k) {  /* only the held set itself has exactly k vertices */
    t->count += 1;
    t->fp = add_p(t->fp, fh);
    return;
  }
  if (ns == 0) {
    const int need = t->k - h;  /* pivots to add */
    if (need > q) return;
    t->count += binom_u128(q, need);
    uint64_t e[17] = {1};       /* elementary symmetric sums of pivot weights */
    for (int j = 1; j <= need; ++j) e[j] = 0;
    for (int i = 0; i < q; ++i)
      for (int j = (i + 1 < need ? i + 1 : need); j >= 1; --j)
        e[j] = add_p(e[j], mul_p(e[j - 1], t->piv[i]));
    t->fp = add_p(t->fp, mul_p(fh, e[need]));
    return;
  }
  const int32_t d = t->d;
  /* pivot: the candidate with the most candidate neighbours */
  int32_t p = S[0], best = -1;
  for (int32_t i = 0; i < ns; ++i) {
    int32_t c = 0;
    for (int32_t j = 0; j < ns; ++j) c += t->adj[(size_t)S[i] * d + S[j]];
    if (c > best) { best = c; p = S[i]; }
  }
  int32_t* next = t->buf + (size_t)(depth + 1) * d;
  /* cliques avoiding every non-neighbour of p: p is optional (a pivot) */
  int32_t nn = 0;
  for (int32_t j = 0; j < ns; ++j)
    if (t->adj[(size_t)p * d + S[j]]) next[nn++] = S[j];
  t->piv[q] = t->w[p];
  pivot_rec(t, next, nn, h, q + 1, fh, depth + 1);
  /* cliques containing a non-neighbour v of p, split by the first such v */
  for (int32_t i = 0; i < ns; ++i) {
    const int32_t v = S[i];
    if (v == p || t->adj[(size_t)p * d + v]) continue;
    nn = 0;
    for (int32_t j = 0; j < ns; ++j)
      if (t->adj[(size_t)v * d + S[j]] && !t->gone[S[j]]) next[nn++] = S[j];
    pivot_rec(t, next, nn, h + 1, q, mul_p(fh, t->w[v]), depth + 1);
    t->gone[v] = 1;
  }
  for (int32_t i = 0; i < ns; ++i) t->gone[S[i]] = 0;
}

static int pivot_root(const dag_t* g, int k, int32_t r, u128* count, uint64_t* fp) {
  const int64_t b = g->optr[r];
  const int32_t d = (int32_t)(g->optr[r + 1] - b);
  *count = 0;
  *fp = 0;
  if (k == 1) { *count = 1; *fp = g->gw[r]; return 0; }
  if (d < k - 1) return 0;
  pivot_t t;
  memset(&t, 0, sizeof(t));
  t.k = k;
  t.d = d;
  t.adj = (unsigned char*)calloc((size_t)d * d, 1);
  t.w = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)d);
  t.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)d * (size_t)(d + 2));
  t.gone = (unsigned char*)calloc((size_t)d, 1);
  t.piv = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(d + 1));
  int err = !t.adj || !t.w || !t.buf || !t.gone || !t.piv;
  if (!err) {
    /* local ids: position in the (sorted) out-list of r */
    for (int32_t i = 0; i < d; ++i) {
      const int32_t a = g->ocol[b + i];
      t.w[i] = g->gw[a];
      /* neighbours of a of higher rank that are members too: merge */
      int64_t x = g->optr[a], xe = g->optr[a + 1];
      int32_t j = i + 1;
      while (x < xe && j < d) {
        if (g->ocol[x] < g->ocol[b + j]) ++x;
        else if (g->ocol[x] > g->ocol[b + j]) ++j;
        else {
          t.adj[(size_t)i * d + j] = t.adj[(size_t)j * d + i] = 1;
          ++x; ++j;
        }
      }
    }
    for (int32_t i = 0; i < d; ++i) t.buf[i] = i;
    pivot_rec(&t, t.buf, d, 1, 0, g->gw[r], 0);
    *count = t.count;
    *fp = t.fp;
  }
  free(t.adj); free(t.w); free(t.buf); free(t.gone); free(t.piv);
  return err;
}

int oracle_pivot_count_roots(int32_t n, const int32_t* row_ptr, const int32_t* col,
                             int k, const int32_t* roots, int64_t nroots,
                             int nthreads, uint64_t* out) {
  if (k < 1 || k > 16 || n < 0 || !out || nroots < 0) return 1;
  if (oracle_validate(n, row_ptr, col)) return 1;
  for (int64_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return 1;
  dag_t d;
  if (build_dag(n, row_ptr, col, &d)) { free_dag(&d); return 1; }
  int err = 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(|| : err)
  for (int64_t i = 0; i < nroots; ++i) {
    u128 c;
    uint64_t f;
    if (pivot_root(&d, k, d.rank[roots[i]], &c, &f)) err = 1;
    out[3 * i + 0] = (uint64_t)c;
    out[3 * i + 1] = (uint64_t)(c >> 64);
    out[3 * i + 2] = f;
  }
  free_dag(&d);
  return err;
}
