/*
 * Seeded synthetic inputs for the graph workloads: R-MAT and 2-D grid edge
 * lists, integer edge weights, query sources and Poisson arrival times.
 *
 * This module produces raw inputs only.  It performs none of the method's
 * arithmetic (no cleaning, no CSR, no traversal): both the GPU library and
 * the CPU oracle consume its output and build their own graph structures.
 *
 * Random numbers come from a counter-based generator: the splitmix64 output
 * function (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to a counter, so every draw is a pure
 * function of (seed, counter) and any thread can compute any draw.
 *
 * R-MAT parameters follow the experimental section of the paper
 * (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) with 2^scale vertices and
 * edge_factor * 2^scale generated edges; weights are integers 1..64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z += GG_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double gg_unit(uint64_t counter) {
  return (double)(gg_mix(counter) >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t gg_splitmix64(uint64_t x) { return gg_mix(x); }

/*
 * R-MAT edge list: m = edge_factor << scale edges.  Edge e picks one
 * quadrant per level l = 0..scale-1, most significant bit first, using the
 * draw r(e, l) = unit(seed * golden + e * scale + l).  No noise and no
 * vertex relabelling, so vertex 0 is the highest-degree vertex.
 * src/dst receive m entries each.  Self-loops and duplicates are kept:
 * removing them is the consumer's job.
 */
void gg_rmat_edges(int scale, int64_t edge_factor, uint64_t seed, double a,
                   double b, double c, int32_t *src, int32_t *dst) {
  const int64_t m = edge_factor << scale;
  const uint64_t base = seed * GG_GOLDEN;
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t r = 0, col = 0;
    const uint64_t ctr = base + (uint64_t)e * (uint64_t)scale;
    for (int l = 0; l < scale; ++l) {
      const double x = gg_unit(ctr + (uint64_t)l);
      uint32_t rb, cb;
      if (x < a) { rb = 0; cb = 0; }
      else if (x < ab) { rb = 0; cb = 1; }
      else if (x < abc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      r |= rb << (scale - 1 - l);
      col |= cb << (scale - 1 - l);
    }
    src[e] = (int32_t)r;
    dst[e] = (int32_t)col;
  }
}

/* Number of undirected edges of a rows x cols 4-neighbour grid. */
int64_t gg_grid_num_edges(int64_t rows, int64_t cols) {
  if (rows <= 0 || cols <= 0) return 0;
  return rows * (cols - 1) + (rows - 1) * cols;
}

/*
 * 4-neighbour grid, vertex id = r * cols + c.  Each undirected edge is
 * emitted once (right neighbour, then down neighbour, row-major order).
 */
void gg_grid_edges(int64_t rows, int64_t cols, int32_t *src, int32_t *dst) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    /* edges owned by row r: (cols-1) right edges, then cols down edges */
    int64_t k = r * ((cols - 1) + cols);
    for (int64_t c = 0; c < cols; ++c) {
      const int64_t v = r * cols + c;
      if (c + 1 < cols) { src[k] = (int32_t)v; dst[k] = (int32_t)(v + 1); ++k; }
      if (r + 1 < rows) { src[k] = (int32_t)v; dst[k] = (int32_t)(v + cols); ++k; }
    }
  }
}

/*
 * Edge weight as a symmetric function of the vertex pair:
 * w(u, v) = 1 + (mix(seed ^ (min(u,v) * n + max(u,v))) mod 64), stored as
 * float.  Duplicate edges get equal weights and w(u, v) = w(v, u).
 */
void gg_edge_weights(int64_t m, const int32_t *src, const int32_t *dst,
                     int64_t n, uint64_t seed, float *w) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const uint64_t u = (uint64_t)(uint32_t)src[e], v = (uint64_t)(uint32_t)dst[e];
    const uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
    w[e] = (float)(1 + (gg_mix(seed ^ (lo * (uint64_t)n + hi)) & 63ULL));
  }
}

/*
 * Marks every vertex that is an endpoint of at least one non-self-loop
 * edge (i.e. has degree > 0 once self-loops are dropped).  flags: n bytes.
 */
void gg_touched(int64_t m, const int32_t *src, const int32_t *dst, int64_t n,
                uint8_t *flags) {
  memset(flags, 0, (size_t)n);
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] != dst[e]) { flags[src[e]] = 1; flags[dst[e]] = 1; }
  }
}

/*
 * k distinct sources drawn uniformly from the vertices whose flag is set.
 * Draw i uses mix(seed * golden + i); a repeated vertex is rejected and the
 * next draw is taken.  Returns the number written (< k only if fewer than k
 * candidates exist).
 */
int64_t gg_sources(int64_t n, const uint8_t *flags, int64_t k, uint64_t seed,
                   int32_t *out) {
  int64_t ncand = 0;
  for (int64_t v = 0; v < n; ++v) ncand += flags[v] ? 1 : 0;
  if (ncand == 0 || k <= 0) return 0;
  int32_t *cand = (int32_t *)malloc((size_t)ncand * sizeof(int32_t));
  uint8_t *taken = (uint8_t *)calloc((size_t)ncand, 1);
  if (!cand || !taken) { free(cand); free(taken); return -1; }
  int64_t j = 0;
  for (int64_t v = 0; v < n; ++v) if (flags[v]) cand[j++] = (int32_t)v;
  const int64_t want = k < ncand ? k : ncand;
  int64_t got = 0;
  uint64_t ctr = seed * GG_GOLDEN;
  while (got < want) {
    const uint64_t idx = gg_mix(ctr++) % (uint64_t)ncand;
    if (taken[idx]) continue;
    taken[idx] = 1;
    out[got++] = cand[idx];
  }
  free(cand);
  free(taken);
  return got;
}

/* Uniform integers in [0, bound): out[i] = mix(seed * golden + i) mod bound. */
void gg_uniform_ints(int64_t count, uint64_t seed, uint64_t bound, int64_t *out) {
  const uint64_t base = seed * GG_GOLDEN;
  for (int64_t i = 0; i < count; ++i) out[i] = (int64_t)(gg_mix(base + (uint64_t)i) % bound);
}

/* Uniform doubles in [0, 1): out[i] = unit(seed * golden + i). */
void gg_uniform_doubles(int64_t count, uint64_t seed, double *out) {
  const uint64_t base = seed * GG_GOLDEN;
  for (int64_t i = 0; i < count; ++i) out[i] = gg_unit(base + (uint64_t)i);
}

/*
 * Poisson process arrival times (seconds) at rate lambda: exponential gaps
 * -ln(1 - u) / lambda with u = unit(seed * golden + i).
 */
void gg_poisson_arrivals(int64_t count, uint64_t seed, double lambda, double *out) {
  const uint64_t base = seed * GG_GOLDEN;
  double t = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    const double u = gg_unit(base + (uint64_t)i);
    t += -log1p(-u) / lambda;
    out[i] = t;
  }
}
