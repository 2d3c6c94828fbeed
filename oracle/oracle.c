/*
 * ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded CPU reference for the graph computations of
 * GraphBLAST (Yang, Buluc, Owens, ACM TOMS 2021).  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code with the GPU library: it builds its own adjacency lists
 * from the raw edge list and uses nothing from the product package.
 *
 *   oracle_adj_build   graph cleaning (self-loops and duplicates removed,
 *                      optional symmetrisation), as the dataset description
 *                      of the experimental section states for all inputs
 *   oracle_bfs         queue BFS; levels are hop distances (source 0,
 *                      unreached -1); parent = smallest-id neighbour one
 *                      level closer (computed by a separate pass)
 *   oracle_sssp        Dijkstra with a binary heap in double precision
 *   oracle_pagerank    FP64 power iteration with uniform redistribution of
 *                      dangling mass, L1 stopping rule
 *   oracle_pagerank_adaptive  the same iteration with converged vertices
 *                      frozen (PageRankDelta)
 *   oracle_msbfs       k independent oracle_bfs runs (optionally on threads)
 *   oracle_triangles   triangle count (and per-vertex counts) by definition
 *   oracle_mxv         the masked semiring product over dense arrays, by its
 *                      definition, one output index at a time
 *   oracle_cc          connected components of a symmetric graph: each
 *                      vertex labelled with the smallest vertex id of its
 *                      component (the fixed point the linear-algebraic
 *                      connected-components iteration of Section 7.4 reaches)
 *
 * parity pins: see tests/test_oracle_*.py (brute force, closed forms,
 * invariants, library special cases).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *off; /* n + 1 */
  int32_t *nbr; /* nnz, ascending within each row */
  double *w;    /* nnz or NULL */
} oracle_adj;

/* ------------------------------------------------------------------ */
/* adjacency construction                                              */
/* ------------------------------------------------------------------ */

/* LSD radix sort of (key, weight) pairs by 64-bit key, 16-bit digits. */
static int radix_sort_pairs(uint64_t *key, double *val, int64_t m, int key_bits) {
  uint64_t *k2 = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
  double *v2 = val ? (double *)malloc((size_t)m * sizeof(double)) : NULL;
  int64_t *cnt = (int64_t *)malloc(65536 * sizeof(int64_t));
  if (!k2 || (val && !v2) || !cnt) { free(k2); free(v2); free(cnt); return -1; }
  for (int shift = 0; shift < key_bits; shift += 16) {
    memset(cnt, 0, 65536 * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) cnt[(key[i] >> shift) & 0xFFFF]++;
    int64_t s = 0;
    for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = s; s += c; }
    for (int64_t i = 0; i < m; ++i) {
      int64_t p = cnt[(key[i] >> shift) & 0xFFFF]++;
      k2[p] = key[i];
      if (val) v2[p] = val[i];
    }
    memcpy(key, k2, (size_t)m * sizeof(uint64_t));
    if (val) memcpy(val, v2, (size_t)m * sizeof(double));
  }
  free(k2); free(v2); free(cnt);
  return 0;
}

/*
 * Builds adjacency lists from a raw edge list.  Self-loops are dropped;
 * with symmetrise != 0 each edge (u, v) also yields (v, u); duplicate
 * (u, v) pairs collapse to one entry whose weight is the smallest weight
 * among the duplicates.  Returns NULL on allocation failure or bad input.
 */
oracle_adj *oracle_adj_build(int64_t n, int64_t m, const int32_t *src,
                             const int32_t *dst, const float *w, int symmetrise) {
  if (n < 0 || m < 0) return NULL;
  int bits = 1;
  while (bits < 63 && ((int64_t)1 << bits) < n + 1) ++bits;
  int64_t cap = symmetrise ? 2 * m : m;
  uint64_t *key = (uint64_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(uint64_t));
  double *val = w ? (double *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(double)) : NULL;
  if (!key || (w && !val)) { free(key); free(val); return NULL; }
  int64_t k = 0;
  for (int64_t e = 0; e < m; ++e) {
    int64_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) { free(key); free(val); return NULL; }
    if (u == v) continue;
    key[k] = ((uint64_t)u << bits) | (uint64_t)v;
    if (w) val[k] = (double)w[e];
    ++k;
    if (symmetrise) {
      key[k] = ((uint64_t)v << bits) | (uint64_t)u;
      if (w) val[k] = (double)w[e];
      ++k;
    }
  }
  if (radix_sort_pairs(key, val, k, 2 * bits) != 0) { free(key); free(val); return NULL; }

  oracle_adj *a = (oracle_adj *)calloc(1, sizeof(oracle_adj));
  a->n = n;
  a->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  a->nbr = (int32_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int32_t));
  a->w = w ? (double *)malloc((size_t)(k > 0 ? k : 1) * sizeof(double)) : NULL;
  const uint64_t lowmask = ((uint64_t)1 << bits) - 1;
  int64_t out = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i > 0 && key[i] == key[i - 1]) {
      /* duplicate: keep the smaller weight */
      if (w && val[i] < a->w[out - 1]) a->w[out - 1] = val[i];
      continue;
    }
    int64_t u = (int64_t)(key[i] >> bits);
    a->nbr[out] = (int32_t)(key[i] & lowmask);
    if (w) a->w[out] = val[i];
    a->off[u + 1]++;
    ++out;
  }
  for (int64_t v = 0; v < n; ++v) a->off[v + 1] += a->off[v];
  a->nnz = out;
  free(key);
  free(val);
  return a;
}

void oracle_adj_free(oracle_adj *a) {
  if (!a) return;
  free(a->off); free(a->nbr); free(a->w); free(a);
}

int64_t oracle_adj_nnz(const oracle_adj *a) { return a->nnz; }
int64_t oracle_adj_n(const oracle_adj *a) { return a->n; }

/* Copies the adjacency out: off (n+1, int64), nbr (nnz), w (nnz, may be NULL). */
void oracle_adj_copy(const oracle_adj *a, int64_t *off, int32_t *nbr, double *w) {
  if (off) memcpy(off, a->off, (size_t)(a->n + 1) * sizeof(int64_t));
  if (nbr) memcpy(nbr, a->nbr, (size_t)a->nnz * sizeof(int32_t));
  if (w && a->w) memcpy(w, a->w, (size_t)a->nnz * sizeof(double));
}

/* Reverse graph: the adjacency of A^T (in-edges as rows), same weights. */
oracle_adj *oracle_adj_transpose(const oracle_adj *a) {
  oracle_adj *t = (oracle_adj *)calloc(1, sizeof(oracle_adj));
  t->n = a->n;
  t->nnz = a->nnz;
  t->off = (int64_t *)calloc((size_t)a->n + 1, sizeof(int64_t));
  t->nbr = (int32_t *)malloc((size_t)(a->nnz > 0 ? a->nnz : 1) * sizeof(int32_t));
  t->w = a->w ? (double *)malloc((size_t)(a->nnz > 0 ? a->nnz : 1) * sizeof(double)) : NULL;
  for (int64_t e = 0; e < a->nnz; ++e) t->off[a->nbr[e] + 1]++;
  for (int64_t v = 0; v < a->n; ++v) t->off[v + 1] += t->off[v];
  int64_t *pos = (int64_t *)malloc((size_t)(a->n > 0 ? a->n : 1) * sizeof(int64_t));
  memcpy(pos, t->off, (size_t)a->n * sizeof(int64_t));
  /* rows of A visited in ascending order, so each row of A^T ends sorted */
  for (int64_t u = 0; u < a->n; ++u) {
    for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
      int64_t p = pos[a->nbr[e]]++;
      t->nbr[p] = (int32_t)u;
      if (a->w) t->w[p] = a->w[e];
    }
  }
  free(pos);
  return t;
}

/* ------------------------------------------------------------------ */
/* BFS (Algorithm 1 of the paper, in its plain graph form)              */
/* ------------------------------------------------------------------ */

/*
 * level[v] = number of hops from s (s: 0, unreached: -1).
 * parent[v] = min{u : (u, v) is an edge and level[u] = level[v] - 1};
 * parent[s] = s; unreached: -1.  parent may be NULL.
 * Returns the number of BFS levels (max level + 1), or -1 on bad input.
 */
int32_t oracle_bfs(const oracle_adj *a, int32_t s, int32_t *level, int32_t *parent) {
  const int64_t n = a->n;
  if (s < 0 || s >= n) return -1;
  for (int64_t v = 0; v < n; ++v) level[v] = -1;
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return -1;
  int64_t head = 0, tail = 0;
  queue[tail++] = s;
  level[s] = 0;
  int32_t maxlev = 0;
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
      const int32_t v = a->nbr[e];
      if (level[v] < 0) {
        level[v] = level[u] + 1;
        if (level[v] > maxlev) maxlev = level[v];
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  if (parent) {
    for (int64_t v = 0; v < n; ++v) parent[v] = -1;
    parent[s] = s;
    /* every edge u -> v with level[u] = level[v] - 1 is a candidate tree edge */
    for (int64_t u = 0; u < n; ++u) {
      if (level[u] < 0) continue;
      for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
        const int32_t v = a->nbr[e];
        if (v != s && level[v] == level[u] + 1 &&
            (parent[v] < 0 || (int32_t)u < parent[v]))
          parent[v] = (int32_t)u;
      }
    }
  }
  return maxlev + 1;
}

/* ------------------------------------------------------------------ */
/* SSSP: Dijkstra with a binary heap                                   */
/* ------------------------------------------------------------------ */

typedef struct { double d; int32_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *sz, heap_item it) {
  int64_t i = (*sz)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= it.d) break;
    h[i] = h[p];
    i = p;
  }
  h[i] = it;
}

static heap_item heap_pop(heap_item *h, int64_t *sz) {
  heap_item top = h[0];
  heap_item last = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *sz) break;
    if (c + 1 < *sz && h[c + 1].d < h[c].d) ++c;
    if (last.d <= h[c].d) break;
    h[i] = h[c];
    i = c;
  }
  if (*sz > 0) h[i] = last;
  return top;
}

/*
 * Shortest-path distances from s over non-negative weights, computed in
 * double (exact for integer weights with sums below 2^53) and returned as
 * float (+inf for unreached).  dist64 (optional) receives the doubles.
 * Returns the number of reached vertices, or -1 on bad input.
 */
int64_t oracle_sssp(const oracle_adj *a, int32_t s, float *dist, double *dist64) {
  const int64_t n = a->n;
  if (s < 0 || s >= n || !a->w) return -1;
  double *d = (double *)malloc((size_t)n * sizeof(double));
  uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
  /* lazy deletion: at most one push per relaxation plus the source */
  heap_item *h = (heap_item *)malloc((size_t)(a->nnz + 1) * sizeof(heap_item));
  if (!d || !done || !h) { free(d); free(done); free(h); return -1; }
  for (int64_t v = 0; v < n; ++v) d[v] = INFINITY;
  d[s] = 0.0;
  int64_t sz = 0, reached = 0;
  heap_push(h, &sz, (heap_item){0.0, s});
  while (sz > 0) {
    heap_item it = heap_pop(h, &sz);
    if (done[it.v]) continue;
    done[it.v] = 1;
    ++reached;
    for (int64_t e = a->off[it.v]; e < a->off[it.v + 1]; ++e) {
      const int32_t v = a->nbr[e];
      const double nd = it.d + a->w[e];
      if (nd < d[v]) { d[v] = nd; heap_push(h, &sz, (heap_item){nd, v}); }
    }
  }
  for (int64_t v = 0; v < n; ++v) {
    dist[v] = (float)d[v];
    if (dist64) dist64[v] = d[v];
  }
  free(d); free(done); free(h);
  return reached;
}

/* ------------------------------------------------------------------ */
/* PageRank: FP64 power iteration                                      */
/* ------------------------------------------------------------------ */

/*
 * a: out-edge adjacency of a directed graph.  Starting from p = 1/n, each
 * iteration computes
 *   D = sum of p(u) over vertices u with no out-edges,
 *   p'(v) = (1 - alpha)/n + alpha * (sum_{u -> v} p(u)/outdeg(u) + D/n),
 *   delta = ||p' - p||_1,
 * and stops after max_iter iterations or as soon as delta < tol.
 * p (n doubles) receives the result; returns the number of iterations run
 * (the last delta in *delta_out when non-NULL), or -1 on bad input.
 */
int32_t oracle_pagerank(const oracle_adj *a, double alpha, int32_t max_iter,
                        double tol, double *p, double *delta_out) {
  const int64_t n = a->n;
  if (n <= 0 || max_iter < 0) return -1;
  double *q = (double *)malloc((size_t)n * sizeof(double));
  if (!q) return -1;
  for (int64_t v = 0; v < n; ++v) p[v] = 1.0 / (double)n;
  int32_t it = 0;
  double delta = INFINITY;
  while (it < max_iter) {
    double dangling = 0.0;
    for (int64_t u = 0; u < n; ++u)
      if (a->off[u + 1] == a->off[u]) dangling += p[u];
    for (int64_t v = 0; v < n; ++v) q[v] = 0.0;
    for (int64_t u = 0; u < n; ++u) {
      const int64_t deg = a->off[u + 1] - a->off[u];
      if (deg == 0) continue;
      const double share = p[u] / (double)deg;
      for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) q[a->nbr[e]] += share;
    }
    delta = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      const double nv = (1.0 - alpha) / (double)n + alpha * (q[v] + dangling / (double)n);
      delta += fabs(nv - p[v]);
      p[v] = nv;
    }
    ++it;
    if (delta < tol) break;
  }
  free(q);
  if (delta_out) *delta_out = delta;
  return it;
}

/*
 * Adaptive PageRank (PageRankDelta, named in Sections 5.1 and 7.3 as the
 * masked form of PageRank: the mask holds the vertices that have already
 * converged, whose values are no longer updated; Kamvar, Haveliwala and
 * Golub's adaptive method).  Starting from p = 1/n with every vertex
 * active, each iteration
 *   D      = sum of p(u) over all vertices u without out-edges (frozen ones
 *            included),
 *   p'(v)  = (1-alpha)/n + alpha * (sum_{u->v} p(u)/outdeg(u) + D/n)
 *            for active v;  p'(v) = p(v) for frozen v,
 *   delta  = ||p' - p||_1,
 * and then freezes every active v with |p'(v) - p(v)| <= eps * p(v) (its
 * change relative to the previous iterate); a frozen vertex stays frozen.
 * Stops after max_iter iterations, as soon as delta < tol, or when no
 * vertex is left active.  p receives the values, frozen_at (may be NULL)
 * the iteration (1-based) at which each vertex froze or 0 if it never
 * did, *active_out (may be NULL) the count still active.  Returns the
 * iterations run, or -1 on bad input.
 */
int32_t oracle_pagerank_adaptive(const oracle_adj *a, double alpha, int32_t max_iter,
                                 double tol, double eps, double *p, int32_t *frozen_at,
                                 double *delta_out, int64_t *active_out) {
  const int64_t n = a->n;
  if (n <= 0 || max_iter < 0 || !(eps >= 0.0)) return -1;
  double *q = (double *)malloc((size_t)n * sizeof(double));
  int32_t *fz = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!q || !fz) { free(q); free(fz); return -1; }
  for (int64_t v = 0; v < n; ++v) { p[v] = 1.0 / (double)n; fz[v] = 0; }
  int64_t active = n;
  int32_t it = 0;
  double delta = INFINITY;
  while (it < max_iter && active > 0) {
    double dangling = 0.0;
    for (int64_t u = 0; u < n; ++u)
      if (a->off[u + 1] == a->off[u]) dangling += p[u];
    for (int64_t v = 0; v < n; ++v) q[v] = 0.0;
    for (int64_t u = 0; u < n; ++u) {
      const int64_t deg = a->off[u + 1] - a->off[u];
      if (deg == 0) continue;
      const double share = p[u] / (double)deg;
      for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) q[a->nbr[e]] += share;
    }
    ++it;
    delta = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      if (fz[v]) continue;  /* frozen: p'(v) = p(v) */
      const double nv = (1.0 - alpha) / (double)n + alpha * (q[v] + dangling / (double)n);
      const double ch = fabs(nv - p[v]);
      delta += ch;
      if (ch <= eps * p[v]) { fz[v] = it; --active; }
      p[v] = nv;
    }
    if (delta < tol) break;
  }
  if (frozen_at) memcpy(frozen_at, fz, (size_t)n * sizeof(int32_t));
  free(q);
  free(fz);
  if (delta_out) *delta_out = delta;
  if (active_out) *active_out = active;
  return it;
}

/* ------------------------------------------------------------------ */
/* batched BFS: k independent single-source runs                       */
/* ------------------------------------------------------------------ */

typedef struct {
  const oracle_adj *a;
  const int32_t *sources;
  int32_t *levels; /* k x n, row q = levels of query q */
  int64_t k;
  int64_t next;
  pthread_mutex_t mu;
} msbfs_job;

static void *msbfs_worker(void *arg) {
  msbfs_job *job = (msbfs_job *)arg;
  for (;;) {
    pthread_mutex_lock(&job->mu);
    const int64_t q = job->next++;
    pthread_mutex_unlock(&job->mu);
    if (q >= job->k) break;
    oracle_bfs(job->a, job->sources[q], job->levels + q * job->a->n, NULL);
  }
  return NULL;
}

/*
 * levels: k x n int32 (query-major).  Runs the k BFS queries on nthreads
 * threads (each query on one thread).  Returns 0, or -1 on bad input.
 */
int32_t oracle_msbfs(const oracle_adj *a, int64_t k, const int32_t *sources,
                     int32_t *levels, int32_t nthreads) {
  for (int64_t q = 0; q < k; ++q)
    if (sources[q] < 0 || sources[q] >= a->n) return -1;
  if (nthreads < 1) nthreads = 1;
  msbfs_job job = {a, sources, levels, k, 0, PTHREAD_MUTEX_INITIALIZER};
  pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
  for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, msbfs_worker, &job);
  for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  return 0;
}

/* ------------------------------------------------------------------ */
/* triangle counting                                                   */
/* ------------------------------------------------------------------ */

/* first position in nbr[lo, hi) holding a value > x (ascending list) */
static int64_t upper_pos(const int32_t *nbr, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (nbr[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* whether x occurs in nbr[lo, hi) (ascending list) */
static int has_entry(const int32_t *nbr, int64_t lo, int64_t hi, int32_t x) {
  const int64_t p = upper_pos(nbr, lo, hi, x);
  return p > lo && nbr[p - 1] == x;
}

/*
 * Triangle count of an undirected graph (Section 7.5: the number of vertex
 * triples that are pairwise adjacent), by its definition: each triangle
 * u < v < w is found exactly once, from its edge (u, v), as a common
 * neighbour w > v of u and v (the shorter of the two sorted tails above v
 * is walked and each of its entries looked up in the other).  The
 * adjacency must be symmetric.  per_vertex (n entries, may be NULL)
 * receives the number of triangles containing each vertex.  Returns the
 * count, or -1 on bad input.
 */
int64_t oracle_triangles(const oracle_adj *a, int64_t *per_vertex) {
  if (!a || a->n < 0) return -1;
  if (per_vertex)
    for (int64_t v = 0; v < a->n; ++v) per_vertex[v] = 0;
  int64_t total = 0;
  for (int64_t u = 0; u < a->n; ++u) {
    const int64_t ub = a->off[u], ue = a->off[u + 1];
    for (int64_t e = upper_pos(a->nbr, ub, ue, (int32_t)u); e < ue; ++e) {
      const int32_t v = a->nbr[e];  /* v > u */
      const int64_t tu = e + 1;     /* N(u) above v: [tu, ue) */
      const int64_t tv = upper_pos(a->nbr, a->off[v], a->off[v + 1], v);
      const int64_t ve = a->off[v + 1];
      const int walk_u = (ue - tu) <= (ve - tv);
      const int64_t wb = walk_u ? tu : tv, we = walk_u ? ue : ve;
      const int64_t ob = walk_u ? tv : tu, oe = walk_u ? ve : ue;
      for (int64_t k = wb; k < we; ++k) {
        const int32_t w = a->nbr[k];
        if (has_entry(a->nbr, ob, oe, w)) {
          ++total;
          if (per_vertex) { per_vertex[u]++; per_vertex[v]++; per_vertex[w]++; }
        }
      }
    }
  }
  return total;
}

/* ------------------------------------------------------------------ */
/* masked semiring matrix-vector product                               */
/* ------------------------------------------------------------------ */

/* semiring codes, numbered as the library's enum (Table 4 of the paper) */
enum { OR_LOR_LAND = 0, OR_MIN_PLUS_32 = 1, OR_MIN_PLUS_64 = 2, OR_PLUS_TIMES_32 = 3,
       OR_PLUS_TIMES_64 = 4, OR_MIN_FIRST = 5, OR_MIN_SECOND = 6 };
/* accumulators */
enum { OR_NOACCUM = 0, OR_ACC_MIN = 1, OR_ACC_PLUS = 2, OR_ACC_LOR = 3 };
/* descriptor bits */
enum { OR_COMP = 1, OR_STRUCT = 2, OR_REPLACE = 8 };

static double sr_add(int sr, double x, double y) {
  switch (sr) {
    case OR_LOR_LAND: return (x != 0.0 || y != 0.0) ? 1.0 : 0.0;
    case OR_PLUS_TIMES_32:
    case OR_PLUS_TIMES_64: return x + y;
    default: return x < y ? x : y; /* the min semirings */
  }
}

/* the multiply with the operands in the product's order: (a, b) is
 * (A(i,j), u(j)) for mxv and (u(i), A(i,j)) for vxm */
static double sr_mul(int sr, double a, double b) {
  switch (sr) {
    case OR_LOR_LAND: return (a != 0.0 && b != 0.0) ? 1.0 : 0.0;
    case OR_MIN_PLUS_32:
    case OR_MIN_PLUS_64: return a + b;
    case OR_PLUS_TIMES_32:
    case OR_PLUS_TIMES_64: return a * b;
    case OR_MIN_FIRST: return a;
    default: return b; /* OR_MIN_SECOND */
  }
}

/*
 * w<mask> = accum(w, A' u) over a semiring (Section 3.3 and the caption of
 * the mxv figure; masking per Section 3.2.1; accum and REPLACE per the
 * GraphBLAS C API), written out for one output index at a time.  `a` holds
 * the rows of A' (the caller passes the transposed adjacency when the
 * product runs over the transpose); a row with no stored weights counts
 * every entry as 1.  vec_first selects the vxm operand order u(j) (x)
 * A'(i,j); otherwise A'(i,j) (x) u(j).  Dense vectors: value arrays in
 * double plus presence bytes.  mask_has NULL means no mask (mask_val NULL
 * with a mask present means every present entry is non-zero).  Every
 * quantity is computed in double.  Returns 0, or -1 on bad input.
 */
int32_t oracle_mxv(const oracle_adj *a, int32_t sr, int32_t vec_first, const double *u_val,
                   const uint8_t *u_has, const double *w_val, const uint8_t *w_has,
                   const double *mask_val, const uint8_t *mask_has, int32_t flags,
                   int32_t accum, double *out_val, uint8_t *out_has) {
  if (!a || sr < OR_LOR_LAND || sr > OR_MIN_SECOND || !u_val || !u_has || !w_val || !w_has ||
      !out_val || !out_has)
    return -1;
  for (int64_t i = 0; i < a->n; ++i) {
    /* t(i): the semiring sum over the stored j of row i with u(j) present */
    int t_has = 0;
    double t = 0.0;
    for (int64_t e = a->off[i]; e < a->off[i + 1]; ++e) {
      const int32_t j = a->nbr[e];
      if (!u_has[j]) continue;
      const double aij = a->w ? a->w[e] : 1.0;
      const double prod = vec_first ? sr_mul(sr, u_val[j], aij) : sr_mul(sr, aij, u_val[j]);
      t = t_has ? sr_add(sr, t, prod) : prod;
      t_has = 1;
    }
    /* z(i) */
    int z_has = t_has;
    double z = t;
    if (accum != OR_NOACCUM && w_has[i]) {
      if (t_has) {
        if (accum == OR_ACC_MIN) z = w_val[i] < t ? w_val[i] : t;
        else if (accum == OR_ACC_PLUS) z = w_val[i] + t;
        else z = (w_val[i] != 0.0 || t != 0.0) ? 1.0 : 0.0;
      } else {
        z = w_val[i];
      }
      z_has = 1;
    }
    /* mask and REPLACE */
    int allowed = 1;
    if (mask_has) {
      int m = mask_has[i] != 0;
      if (m && !(flags & OR_STRUCT) && mask_val) m = mask_val[i] != 0.0;
      allowed = (flags & OR_COMP) ? !m : m;
    }
    if (allowed) {
      out_has[i] = (uint8_t)z_has;
      out_val[i] = z_has ? z : 0.0;
    } else if (!(flags & OR_REPLACE) && w_has[i]) {
      out_has[i] = 1;
      out_val[i] = w_val[i];
    } else {
      out_has[i] = 0;
      out_val[i] = 0.0;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* connected components                                                */
/* ------------------------------------------------------------------ */

/* label[v] = the smallest id in v's component: vertices are visited in
 * increasing id order, and an unlabelled one starts a queue search that
 * labels its whole component with its own id (no smaller id can be in it,
 * since that vertex would already have labelled the component).  Returns
 * the number of components, or -1 on bad input. */
int64_t oracle_cc(const oracle_adj *a, int32_t *label) {
  if (!a || !label) return -1;
  int32_t *queue = (int32_t *)malloc((size_t)(a->n > 0 ? a->n : 1) * sizeof(int32_t));
  if (!queue) return -1;
  for (int64_t v = 0; v < a->n; ++v) label[v] = -1;
  int64_t comps = 0;
  for (int64_t s = 0; s < a->n; ++s) {
    if (label[s] >= 0) continue;
    ++comps;
    int64_t head = 0, tail = 0;
    label[s] = (int32_t)s;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
      const int32_t u = queue[head++];
      for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
        const int32_t v = a->nbr[e];
        if (label[v] < 0) {
          label[v] = (int32_t)s;
          queue[tail++] = v;
        }
      }
    }
  }
  free(queue);
  return comps;
}
