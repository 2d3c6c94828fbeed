// Host-side graph materialisation: raw edge list -> cleaned CSR.
//
// Follows the dataset preparation of the experimental section (dataset
// table caption): self-loops removed, duplicate edges removed, undirected
// inputs symmetrised.  Rows are sorted by column so that a pull scan meets
// neighbours in ascending id order (the smallest-id parent is the first
// frontier neighbour found).  Duplicate (u, v) pairs keep their smallest
// weight.  This is setup work, outside every timed path.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/grb.h"

struct grb_csr_builder_s {
  int64_t n = 0;
  int64_t nnz = 0;
  bool weighted = false;
  std::vector<int32_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<float> w;
};

namespace {

// Order-preserving map of a float's bits to an unsigned integer.
inline uint32_t float_key(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
inline float key_float(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

unsigned worker_count() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return std::min(h, 32u);
}

template <class F>
void parallel_rows(int64_t n, F f) {
  const unsigned T = worker_count();
  std::vector<std::thread> th;
  const int64_t chunk = (n + T - 1) / T;
  for (unsigned t = 0; t < T; ++t) {
    const int64_t lo = std::min<int64_t>(n, (int64_t)t * chunk);
    const int64_t hi = std::min<int64_t>(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([=]() { f(lo, hi); });
  }
  for (auto &x : th) x.join();
}

}  // namespace

extern "C" grb_info grb_csr_build(grb_csr_builder *out, int64_t n, int64_t m,
                                  const int32_t *src, const int32_t *dst, const float *w,
                                  int symmetrise) {
  if (!out) return GRB_NULL_POINTER;
  *out = nullptr;
  if (n < 0 || m < 0 || n >= (int64_t)INT32_MAX) return GRB_INVALID_VALUE;
  if (m > 0 && (!src || !dst)) return GRB_NULL_POINTER;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return GRB_INVALID_INDEX;
  grb_csr_builder_s *b = new (std::nothrow) grb_csr_builder_s;
  if (!b) return GRB_OUT_OF_MEMORY;
  try {
    b->n = n;
    b->weighted = (w != nullptr);
    // 1. raw row counts (self-loops dropped)
    std::vector<int64_t> off((size_t)n + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
      if (src[e] == dst[e]) continue;
      off[(size_t)src[e] + 1]++;
      if (symmetrise) off[(size_t)dst[e] + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) off[(size_t)v + 1] += off[(size_t)v];
    const int64_t total = off[(size_t)n];
    // 2. bucket (column, weight key) pairs by row
    std::vector<uint64_t> ent((size_t)total);
    {
      std::vector<int64_t> cur(off.begin(), off.end() - 1);
      for (int64_t e = 0; e < m; ++e) {
        const int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        const uint64_t wk = w ? float_key(w[e]) : 0u;
        ent[(size_t)cur[(size_t)u]++] = ((uint64_t)(uint32_t)v << 32) | wk;
        if (symmetrise) ent[(size_t)cur[(size_t)v]++] = ((uint64_t)(uint32_t)u << 32) | wk;
      }
    }
    // 3. sort each row, drop duplicate columns (the smallest weight sorts first)
    std::vector<int64_t> keep((size_t)n, 0);
    parallel_rows(n, [&](int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        uint64_t *a = ent.data() + off[(size_t)v];
        const int64_t len = off[(size_t)v + 1] - off[(size_t)v];
        std::sort(a, a + len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
          if (k == 0 || (a[i] >> 32) != (a[k - 1] >> 32)) a[k++] = a[i];
        keep[(size_t)v] = k;
      }
    });
    int64_t nnz = 0;
    for (int64_t v = 0; v < n; ++v) nnz += keep[(size_t)v];
    if (nnz > (int64_t)INT32_MAX) { delete b; return GRB_INVALID_VALUE; }
    b->nnz = nnz;
    b->row_ptr.assign((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v)
      b->row_ptr[(size_t)v + 1] = b->row_ptr[(size_t)v] + (int32_t)keep[(size_t)v];
    b->col.resize((size_t)nnz);
    if (w) b->w.resize((size_t)nnz);
    // 4. compact
    parallel_rows(n, [&](int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        const uint64_t *a = ent.data() + off[(size_t)v];
        int32_t p = b->row_ptr[(size_t)v];
        for (int64_t i = 0; i < keep[(size_t)v]; ++i, ++p) {
          b->col[(size_t)p] = (int32_t)(a[i] >> 32);
          if (w) b->w[(size_t)p] = key_float((uint32_t)(a[i] & 0xffffffffu));
        }
      }
    });
  } catch (const std::bad_alloc &) {
    delete b;
    return GRB_OUT_OF_MEMORY;
  }
  *out = b;
  return GRB_SUCCESS;
}

extern "C" grb_info grb_csr_nnz(grb_csr_builder b, int64_t *nnz) {
  if (!b) return GRB_UNINITIALIZED_OBJECT;
  if (!nnz) return GRB_NULL_POINTER;
  *nnz = b->nnz;
  return GRB_SUCCESS;
}

extern "C" grb_info grb_csr_copy(grb_csr_builder b, int32_t *row_ptr, int32_t *col_idx,
                                 float *values) {
  if (!b) return GRB_UNINITIALIZED_OBJECT;
  if (!row_ptr || (!col_idx && b->nnz > 0)) return GRB_NULL_POINTER;
  if (values && !b->weighted) return GRB_INVALID_VALUE;
  std::memcpy(row_ptr, b->row_ptr.data(), ((size_t)b->n + 1) * sizeof(int32_t));
  if (b->nnz > 0) std::memcpy(col_idx, b->col.data(), (size_t)b->nnz * sizeof(int32_t));
  if (values && b->nnz > 0) std::memcpy(values, b->w.data(), (size_t)b->nnz * sizeof(float));
  return GRB_SUCCESS;
}

extern "C" grb_info grb_csr_free(grb_csr_builder *b) {
  if (!b) return GRB_NULL_POINTER;
  delete *b;
  *b = nullptr;
  return GRB_SUCCESS;
}

// Degree-ordered strict lower triangle for triangle counting (Section 7.5:
// the count is the reduction of L L^T .* L).  Vertices are renumbered by
// decreasing degree (ties by increasing id), so row i of L holds the
// neighbours of i that come earlier in that order, i.e. have at least its
// degree: at most sqrt(2 * nnz) of them.  The result is a new builder
// (structure only, rows sorted); rank[v] (may be NULL) receives the new id
// of vertex v.
extern "C" grb_info grb_csr_lower_by_degree(grb_csr_builder src, grb_csr_builder *out,
                                           int32_t *rank) {
  if (!src || !out) return GRB_NULL_POINTER;
  *out = nullptr;
  const int64_t n = src->n;
  grb_csr_builder_s *b = new (std::nothrow) grb_csr_builder_s;
  if (!b) return GRB_OUT_OF_MEMORY;
  try {
    std::vector<int32_t> order((size_t)n), rk((size_t)n);
    for (int64_t v = 0; v < n; ++v) order[(size_t)v] = (int32_t)v;
    const std::vector<int32_t> &rp = src->row_ptr;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
      return rp[(size_t)a + 1] - rp[(size_t)a] > rp[(size_t)c + 1] - rp[(size_t)c];
    });
    for (int64_t i = 0; i < n; ++i) rk[(size_t)order[(size_t)i]] = (int32_t)i;
    b->n = n;
    b->weighted = false;
    b->row_ptr.assign((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v)
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e)
        if (rk[(size_t)src->col[(size_t)e]] < rk[(size_t)v]) b->row_ptr[(size_t)rk[(size_t)v] + 1]++;
    for (int64_t i = 0; i < n; ++i) b->row_ptr[(size_t)i + 1] += b->row_ptr[(size_t)i];
    b->nnz = b->row_ptr[(size_t)n];
    b->col.resize((size_t)b->nnz);
    std::vector<int32_t> pos(b->row_ptr.begin(), b->row_ptr.end() - 1);
    for (int64_t v = 0; v < n; ++v)
      for (int32_t e = rp[(size_t)v]; e < rp[(size_t)v + 1]; ++e) {
        const int32_t c = rk[(size_t)src->col[(size_t)e]];
        if (c < rk[(size_t)v]) b->col[(size_t)pos[(size_t)rk[(size_t)v]]++] = c;
      }
    for (int64_t i = 0; i < n; ++i)
      std::sort(b->col.begin() + b->row_ptr[(size_t)i], b->col.begin() + b->row_ptr[(size_t)i + 1]);
    if (rank) std::memcpy(rank, rk.data(), (size_t)n * sizeof(int32_t));
  } catch (const std::bad_alloc &) {
    delete b;
    return GRB_OUT_OF_MEMORY;
  }
  *out = b;
  return GRB_SUCCESS;
}
