// Host side of the C ABI: argument validation, handles, workspace layout
// and the driver loops of BFS, SSSP and PageRank.  Every computation step
// runs in the HIP kernels; this file only validates, carves the caller's
// workspace and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <new>
#include <vector>

#include "grb_internal.h"

using namespace grb;

namespace {

thread_local grb_stats g_stats;

int elem_size(grb_type t) {
  switch (t) {
    case GRB_BOOL: return 1;
    case GRB_INT32: return 4;
    case GRB_FP32: return 4;
    case GRB_FP64: return 8;
  }
  return 0;
}

bool valid_type(int t) { return t >= GRB_BOOL && t <= GRB_FP64; }

grb_info check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GRB_SUCCESS : GRB_PANIC;
}

grb_info resolve_desc(const grb_descriptor *d, grb_descriptor *out) {
  grb_descriptor_init(out);
  if (!d) return GRB_SUCCESS;
  *out = *d;
  const uint32_t known =
      GRB_MASK_COMP | GRB_MASK_STRUCT | GRB_TRAN_A | GRB_REPLACE | GRB_PROFILE | GRB_LOOP_NO_WAIT;
  if (out->flags & ~known) return GRB_INVALID_VALUE;
  if (out->direction < GRB_DIR_AUTO || out->direction > GRB_DIR_PULL) return GRB_INVALID_VALUE;
  if (out->switch_rule != GRB_SWITCH_PAPER && out->switch_rule != GRB_SWITCH_EXACT)
    return GRB_INVALID_VALUE;
  if (out->switch_denominator < 0 || out->max_iter < 0) return GRB_INVALID_VALUE;
  for (int i = 0; i < 3; ++i)
    if (out->reserved[i] != 0) return GRB_INVALID_VALUE;
  if (out->switch_denominator == 0) out->switch_denominator = 10;
  return GRB_SUCCESS;
}

// ---- workspace carving ----------------------------------------------------
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  template <class T>
  T *take(size_t count) {
    T *p = base ? (T *)(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

struct BfsWs {
  Ctrl *ctrl;
  int64_t *stats;
  uint64_t *visited, *F[3];
  CoopCtl *coop;  // multi-workgroup loop: shared state, two queues of kCoopSegsMax segments
  int32_t *qv;
  uint64_t *qe;
  int32_t qseg;
  size_t bytes;
};

BfsWs bfs_layout(void *ws, int64_t n) {
  Carver c(ws);
  BfsWs t{};
  const int64_t nw = words_of(n);
  t.ctrl = c.take<Ctrl>(1);
  t.stats = c.take<int64_t>((size_t)kStatsCap * kStatFields);
  t.visited = c.take<uint64_t>((size_t)nw);
  for (int i = 0; i < 3; ++i) t.F[i] = c.take<uint64_t>((size_t)nw);
  t.qseg = (int32_t)std::max<int64_t>(std::min<int64_t>(kCoopSeg, n), 1);
  t.coop = c.take<CoopCtl>(1);
  const size_t qn = 2 * (size_t)kCoopSegsMax * (size_t)t.qseg;
  t.qv = c.take<int32_t>(qn);
  t.qe = c.take<uint64_t>(qn);
  t.bytes = c.off;
  return t;
}

// SSSP: the BFS state plus three rotating "frontier distance" vectors
// (dist of the frontier's vertices, +inf elsewhere)
struct SsspWs {
  BfsWs b;
  float *fd[3];
  size_t bytes;
};

SsspWs sssp_layout(void *ws, int64_t n) {
  SsspWs t{};
  t.b = bfs_layout(ws, n);
  Carver c(ws);
  c.off = t.b.bytes;
  for (int i = 0; i < 3; ++i) t.fd[i] = c.take<float>((size_t)std::max<int64_t>(n, 1));
  t.bytes = c.off;
  return t;
}

struct MsWs {
  Ctrl *ctrl;
  int64_t *stats;
  unsigned long long *cnt;
  uint64_t *V, *F[3], *act[3];
  // sessions: start level per query, three "has a frontier bit" arrays of W
  // words, the joining queries' bits per word, lane / source staging
  int32_t *start, *lanes, *sources;
  unsigned long long *alive;
  uint64_t *clr;
  size_t bytes;
};

MsWs ms_layout(void *ws, int64_t n, int64_t k) {
  Carver c(ws);
  MsWs t{};
  const int64_t W = (k + 63) / 64, nb = std::max<int64_t>(n * W, 1), nw = words_of(n);
  t.ctrl = c.take<Ctrl>(1);
  t.stats = c.take<int64_t>((size_t)kStatsCap * kStatFields);
  t.cnt = c.take<unsigned long long>((size_t)6 * kCntStripes);
  t.V = c.take<uint64_t>((size_t)nb);
  for (int i = 0; i < 3; ++i) t.F[i] = c.take<uint64_t>((size_t)nb);
  for (int i = 0; i < 3; ++i) t.act[i] = c.take<uint64_t>((size_t)std::max<int64_t>(nw, 1));
  t.start = c.take<int32_t>((size_t)std::max<int64_t>(k, 1));
  t.lanes = c.take<int32_t>((size_t)std::max<int64_t>(k, 1));
  t.sources = c.take<int32_t>((size_t)std::max<int64_t>(k, 1));
  t.alive = c.take<unsigned long long>((size_t)3 * std::max<int64_t>(W, 1));
  t.clr = c.take<uint64_t>((size_t)std::max<int64_t>(W, 1));
  t.bytes = c.off;
  return t;
}

struct PrWs {
  Ctrl *ctrl;
  int64_t *stats;
  void *x0, *x1, *heavy_part;
  double *blk_part;
  uint64_t *act[3];  // adaptive PageRank: rotating activity bitmaps
  int nblk, nblk_long;
  size_t bytes;
};

PrWs pr_layout(void *ws, int64_t n, const Csr &pull, int esize) {
  Carver c(ws);
  PrWs t{};
  t.nblk = kSweepGrid;
  t.nblk_long = pr_long_grid(pull.nsplit_rows);
  t.ctrl = c.take<Ctrl>(1);
  t.stats = c.take<int64_t>((size_t)kStatsCap * kStatFields);
  t.x0 = c.take<char>((size_t)std::max<int64_t>(n, 1) * esize);
  t.x1 = c.take<char>((size_t)std::max<int64_t>(n, 1) * esize);
  t.heavy_part = c.take<char>((size_t)std::max<int64_t>(pull.nsplit, 1) * esize);
  t.blk_part = c.take<double>((size_t)kPrFields * (t.nblk + t.nblk_long));
  for (int i = 0; i < 3; ++i) t.act[i] = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n), 1));
  t.bytes = c.off;
  return t;
}

struct MxvWs {
  Ctrl *ctrl;
  int64_t *part, *blk_part;
  uint64_t *status, *status_out, *status_list, *t_bm, *t_vb;
  int32_t *list, *degpre, *rowstart, *tiles;
  int64_t tiles_cap;
  void *t_val, *hp_val;
  uint8_t *hp_has, *settled;
  uint64_t *ubm, *mbm, *wbm;  // bitmaps of operands given only as lists
  int nblk, nblk_out, nblk_list;
  size_t bytes;
};

MxvWs mxv_layout(void *ws, int64_t n_in, int64_t n_out, int64_t nnz, int64_t npieces) {
  Carver c(ws);
  MxvWs t{};
  t.nblk = compact_blocks(words_of(n_in));
  t.nblk_out = compact_blocks(words_of(n_out));
  t.nblk_list = (int)std::max<int64_t>(1, (n_in + kMxvListChunk - 1) / kMxvListChunk);
  t.ctrl = c.take<Ctrl>(1);
  t.part = c.take<int64_t>((size_t)2 * kMxvParts);
  t.blk_part = c.take<int64_t>((size_t)2 * t.nblk);
  t.status = c.take<uint64_t>((size_t)2 * t.nblk);
  t.status_out = c.take<uint64_t>((size_t)2 * t.nblk_out);
  t.status_list = c.take<uint64_t>((size_t)t.nblk_list);
  t.list = c.take<int32_t>((size_t)std::max<int64_t>(n_in, 1));
  t.degpre = c.take<int32_t>((size_t)std::max<int64_t>(n_in, 1));
  t.rowstart = c.take<int32_t>((size_t)std::max<int64_t>(n_in, 1));
  t.tiles_cap = (n_in + nnz) / kPushTile + 3;
  t.tiles = c.take<int32_t>((size_t)t.tiles_cap);
  t.t_bm = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n_out), 1));
  t.t_vb = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n_out), 1));
  t.t_val = c.take<char>((size_t)std::max<int64_t>(n_out, 1) * 8);
  t.hp_val = c.take<char>((size_t)std::max<int64_t>(npieces, 1) * 8);
  t.hp_has = c.take<uint8_t>((size_t)std::max<int64_t>(npieces, 1));
  t.settled = c.take<uint8_t>((size_t)std::max<int64_t>(n_out, 1));
  t.ubm = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n_in), 1));
  t.mbm = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n_out), 1));
  t.wbm = c.take<uint64_t>((size_t)std::max<int64_t>(words_of(n_out), 1));
  t.bytes = c.off;
  return t;
}

int64_t split_bound(int64_t nnz) { return nnz / kPushSplit + nnz / (kPushSplit + 1) + 2; }

struct ExtractWs {
  Ctrl *ctrl;
  uint64_t *status;
  int32_t *list, *cnt;
  void *vals;
  int nblk;
  size_t bytes;
};

ExtractWs extract_layout(void *ws, int64_t n) {
  Carver c(ws);
  ExtractWs t{};
  t.nblk = compact_blocks(words_of(n));
  t.ctrl = c.take<Ctrl>(1);
  t.status = c.take<uint64_t>((size_t)2 * t.nblk);
  t.cnt = c.take<int32_t>(1);
  t.list = c.take<int32_t>((size_t)std::max<int64_t>(n, 1));
  t.vals = c.take<char>((size_t)std::max<int64_t>(n, 1) * 8);
  t.bytes = c.off;
  return t;
}

struct CcWs {
  int64_t *changed;
  int32_t *f, *f_old, *gf, *mngf;
  uint64_t *gf_bm, *mngf_bm;
  void *mxv;
  size_t mxv_bytes;
  size_t bytes;
};

CcWs cc_layout(void *ws, int64_t n, size_t mxv_bytes) {
  Carver c(ws);
  CcWs t{};
  const size_t m = (size_t)std::max<int64_t>(n, 1), mw = (size_t)std::max<int64_t>(words_of(n), 1);
  t.changed = c.take<int64_t>((size_t)kStatsCap);
  t.f = c.take<int32_t>(m);
  t.f_old = c.take<int32_t>(m);
  t.gf = c.take<int32_t>(m);
  t.mngf = c.take<int32_t>(m);
  t.gf_bm = c.take<uint64_t>(mw);
  t.mngf_bm = c.take<uint64_t>(mw);
  t.mxv = c.take<char>(mxv_bytes);
  t.mxv_bytes = mxv_bytes;
  t.bytes = c.off;
  return t;
}

grb_info check_ws(void *ws, size_t have, size_t need) {
  if (need > have) return GRB_INSUFFICIENT_SPACE;
  if (!ws) return GRB_NULL_POINTER;
  if (((uintptr_t)ws) % 256 != 0) return GRB_INVALID_VALUE;
  return GRB_SUCCESS;
}

// ---- matrix metadata ---------------------------------------------------------
struct MetaLayout {
  size_t heavy_off, heavy_rows_off, split_off, split_rows_off, wpart_off, iso_off, first2_off,
      bytes;
  int64_t max_pieces, max_rows, max_split, max_split_rows;
};

MetaLayout meta_layout_one(int64_t nnz, int64_t nrows, size_t base) {
  MetaLayout m{};
  m.max_rows = nnz / (kHeavyDeg + 1) + 1;
  m.max_pieces = nnz / kHeavyChunk + m.max_rows + 1;
  m.max_split = nnz / kPushSplit + nnz / (kPushSplit + 1) + 1;
  m.heavy_off = base;
  m.heavy_rows_off = align_up(base + (size_t)m.max_pieces * 2 * sizeof(int32_t));
  m.split_off = align_up(m.heavy_rows_off + (size_t)m.max_rows * 3 * sizeof(int32_t));
  m.max_split_rows = nnz / (kPushSplit + 1) + 1;
  m.split_rows_off = align_up(m.split_off + (size_t)m.max_split * 2 * sizeof(int32_t));
  m.wpart_off = align_up(m.split_rows_off + (size_t)m.max_split_rows * 3 * sizeof(int32_t));
  m.iso_off = align_up(m.wpart_off + (size_t)(kWaveParts + 1) * sizeof(int32_t));
  m.first2_off = align_up(m.iso_off + (size_t)words_of(nrows) * sizeof(uint64_t));
  m.bytes = align_up(m.first2_off + (size_t)nrows * 2 * sizeof(int32_t));
  return m;
}

grb_info build_meta(Csr &c, char *meta, const MetaLayout &L, hipStream_t s) {
  std::vector<int32_t> rp;
  try {
    rp.resize((size_t)c.nrows + 1);
  } catch (const std::bad_alloc &) {
    return GRB_OUT_OF_MEMORY;
  }
  if (hipMemcpyAsync(rp.data(), c.rp, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GRB_PANIC;
  if (rp[0] != 0 || rp[(size_t)c.nrows] != c.nnz) return GRB_INVALID_VALUE;
  std::vector<int32_t> pieces, rows, split, split_rows;
  for (int64_t r = 0; r < c.nrows; ++r) {
    const int32_t b = rp[(size_t)r], e = rp[(size_t)r + 1];
    if (e < b) return GRB_INVALID_VALUE;
    if (e - b > kPushSplit) {
      split_rows.push_back((int32_t)r);
      split_rows.push_back((int32_t)(split.size() / 2));
      int32_t np = 0;
      for (int32_t p = b; p < e; p += kPushSplit, ++np) {
        split.push_back((int32_t)r);
        split.push_back(p);
      }
      split_rows.push_back(np);
    }
    if (e - b > kHeavyDeg) {
      rows.push_back((int32_t)r);
      rows.push_back((int32_t)(pieces.size() / 2));
      int32_t np = 0;
      for (int32_t p = b; p < e; p += kHeavyChunk, ++np) {
        pieces.push_back((int32_t)r);
        pieces.push_back(p);
      }
      rows.push_back(np);
    }
  }
  int64_t max_deg = 0;
  for (int64_t r = 0; r < c.nrows; ++r)
    max_deg = std::max<int64_t>(max_deg, rp[(size_t)r + 1] - rp[(size_t)r]);
  c.max_deg = max_deg;
  if ((int64_t)pieces.size() / 2 > L.max_pieces || (int64_t)rows.size() / 3 > L.max_rows ||
      (int64_t)split.size() / 2 > L.max_split ||
      (int64_t)split_rows.size() / 3 > L.max_split_rows)
    return GRB_PANIC;
  int32_t *hp = (int32_t *)(meta + L.heavy_off);
  int32_t *hr = (int32_t *)(meta + L.heavy_rows_off);
  // word runs of about equal work for the full sweeps
  const int64_t nw = words_of(c.nrows);
  std::vector<int64_t> wcost((size_t)nw + 1, 0);
  for (int64_t w = 0; w < nw; ++w) {
    int64_t e = 256;  // fixed cost of a word: about one step of the stream
    const int64_t r1 = std::min<int64_t>(c.nrows, (w + 1) * 64);
    for (int64_t r = w * 64; r < r1; ++r) {
      const int64_t d = rp[(size_t)r + 1] - rp[(size_t)r];
      if (d <= kPushSplit) e += d;
    }
    wcost[(size_t)w + 1] = wcost[(size_t)w] + e;
  }
  std::vector<int32_t> wpart((size_t)kWaveParts + 1);
  {
    const int64_t tot = wcost[(size_t)nw];
    int64_t w = 0;
    for (int64_t p = 0; p <= kWaveParts; ++p) {
      const int64_t goal = (int64_t)((__int128)tot * p / kWaveParts);
      while (w < nw && wcost[(size_t)w] < goal) ++w;
      wpart[(size_t)p] = (int32_t)w;
    }
    wpart[(size_t)kWaveParts] = (int32_t)nw;
  }
  // rows without entries; padding bits past nrows count as such
  std::vector<uint64_t> iso((size_t)nw, 0ull);
  for (int64_t w = 0; w < nw; ++w) {
    uint64_t bits = 0ull;
    for (int b = 0; b < 64; ++b) {
      const int64_t r = w * 64 + b;
      if (r >= c.nrows || rp[(size_t)r + 1] == rp[(size_t)r]) bits |= 1ull << b;
    }
    iso[(size_t)w] = bits;
  }
  uint64_t *isop = (uint64_t *)(meta + L.iso_off);
  if (nw > 0 &&
      hipMemcpyAsync(isop, iso.data(), iso.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  int32_t *wp = (int32_t *)(meta + L.wpart_off);
  if (hipMemcpyAsync(wp, wpart.data(), wpart.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  int32_t *sp = (int32_t *)(meta + L.split_off);
  int32_t *sr = (int32_t *)(meta + L.split_rows_off);
  if (!split_rows.empty() && hipMemcpyAsync(sr, split_rows.data(), split_rows.size() * 4,
                                            hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  if (!split.empty() &&
      hipMemcpyAsync(sp, split.data(), split.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  if (!pieces.empty() &&
      hipMemcpyAsync(hp, pieces.data(), pieces.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  if (!rows.empty() &&
      hipMemcpyAsync(hr, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  int2 *f2 = (int2 *)(meta + L.first2_off);
  // negative (or NaN) values: shortest paths refuse the matrix; the flag
  // word borrows the first-two array's first slot, written right after
  int32_t neg = 0;
  if (c.val && (c.vtype == GRB_FP32 || c.vtype == GRB_FP64) && c.nrows > 0) {
    int32_t *flag = (int32_t *)f2;
    launch_any_negative(c.val, c.vtype, c.nnz, flag, s);
    if (hipGetLastError() != hipSuccess) return GRB_PANIC;
    if (hipMemcpyAsync(&neg, flag, sizeof(neg), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return GRB_PANIC;
  }
  c.negative = neg != 0;
  launch_first_two(c.rp, c.ci, c.nrows, f2, s);
  if (hipGetLastError() != hipSuccess) return GRB_PANIC;
  if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;
  c.first2 = f2;
  c.heavy = hp;
  c.nheavy = (int64_t)pieces.size() / 2;
  c.heavy_rows = hr;
  c.nheavy_rows = (int64_t)rows.size() / 3;
  c.split = sp;
  c.nsplit = (int64_t)split.size() / 2;
  c.split_rows = sr;
  c.nsplit_rows = (int64_t)split_rows.size() / 3;
  c.wpart = wp;
  c.iso = isop;
  return GRB_SUCCESS;
}

// ---- profiling events --------------------------------------------------------
struct EventPool {
  std::vector<hipEvent_t> ev;
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipEvent_t get(size_t i) {
    while (ev.size() <= i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[i];
  }
};
thread_local EventPool g_events;

// ---- control-block readback ----------------------------------------------------
// The drivers read their control block back once per batch of launches.  A
// device-to-host copy into pageable memory goes through the runtime's bounce
// buffer and takes about twice the round trip of one into pinned memory, so
// the copies land in a pinned staging buffer (one per host thread, grown on
// demand, kept for the thread's lifetime) and are then copied on the host.
thread_local bool g_no_alloc = false;  // a caller that must not allocate is running

struct Staging {
  char *buf = nullptr;
  size_t cap = 0;
  char *get(size_t bytes) {
    if (bytes <= cap) return buf;
    if (g_no_alloc) return nullptr;  // direct copies instead of a new pinned buffer
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipHostMalloc((void **)&buf, bytes, hipHostMallocDefault) != hipSuccess) {
      buf = nullptr;
      return nullptr;
    }
    cap = bytes;
    return buf;
  }
};
thread_local Staging g_staging;

}  // namespace

grb::NoAllocScope::NoAllocScope() : prev_(g_no_alloc) { g_no_alloc = true; }
grb::NoAllocScope::~NoAllocScope() { g_no_alloc = prev_; }

namespace {

struct Region {
  void *dst;        // host destination
  const void *src;  // device source
  size_t bytes;
};

// Copies every region device-to-host on stream s and waits for the stream.
// Falls back to direct copies if no pinned memory can be had.  False on any
// HIP error.
bool read_back(std::initializer_list<Region> regs, hipStream_t s) {
  auto slot = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t total = 0;
  for (const Region &r : regs) total += slot(r.bytes);
  char *st = g_staging.get(total);
  size_t off = 0;
  for (const Region &r : regs) {
    if (r.bytes == 0) continue;
    void *to = st ? (void *)(st + off) : r.dst;
    if (hipMemcpyAsync(to, r.src, r.bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    off += slot(r.bytes);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  if (st) {
    off = 0;
    for (const Region &r : regs) {
      if (r.bytes == 0) continue;
      std::memcpy(r.dst, st + off, r.bytes);
      off += slot(r.bytes);
    }
  }
  return true;
}

void finish_stats(int op, int iterations, const std::vector<int64_t> &rec,
                  const std::vector<float> &kms, int launches, double ms_all) {
  grb_stats &s = g_stats;
  std::memset(&s, 0, sizeof(s));
  s.op = op;
  s.iterations = iterations;
  s.launches = launches;
  s.expand_ms_all = ms_all;
  s.recorded = std::min(iterations, (int)kStatsCap);
  for (int i = 0; i < s.recorded; ++i) {
    s.frontier[i] = rec[(size_t)i * kStatFields + 0];
    s.edges[i] = rec[(size_t)i * kStatFields + 1];
    s.direction[i] = (int32_t)rec[(size_t)i * kStatFields + 2];
    if (s.direction[i] == GRB_DIR_PUSH) {
      s.pushes++;
      s.edges_push += s.edges[i];
    } else if (s.direction[i] == GRB_DIR_PULL) {
      s.pulls++;
    }
    if (i < (int)kms.size()) {
      s.kernel_ms[i] = kms[(size_t)i];
      if (s.direction[i] == GRB_DIR_PUSH) s.expand_ms_push += kms[(size_t)i];
      else s.expand_ms_pull += kms[(size_t)i];
    }
  }
}

// BFS: one kernel per level (all state on the device); the host reads the
// frontier size back once per batch of levels to detect the end.
grb_info run_bfs(grb_matrix A, int32_t source, int32_t *levels, int32_t *parents,
                 const grb_descriptor &desc, void *ws, size_t ws_bytes, void *stream) {
  const int64_t n = A->nrows;
  const bool can_pull = A->at.valid();
  if (!can_pull && (desc.direction == GRB_DIR_PULL || parents)) return GRB_NOT_IMPLEMENTED;
  BfsWs w = bfs_layout(ws, n);
  grb_info info = check_ws(ws, ws_bytes, w.bytes);
  if (info != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  BfsArgs ba;
  ba.n = n;
  ba.nw = words_of(n);
  ba.nnz = A->nnz;
  ba.push = A->a;
  ba.pull = A->at;
  ba.can_pull = can_pull;
  ba.same_csr = A->symmetric;
  ba.visited = w.visited;
  ba.levels = levels;
  ba.parents = parents;
  ba.ctrl = w.ctrl;
  ba.stats = w.stats;
  ba.rule = desc.switch_rule;
  ba.denom = desc.switch_denominator;
  ba.forced = desc.direction;
  int32_t *cnt = w.ctrl->lists;
  auto at_level = [&](int64_t d) {
    const int i = (int)(d % 3), j = (int)((d + 1) % 3), k = (int)((d + 2) % 3);
    ba.fcur = w.F[i];
    ba.fnxt = w.F[j];
    ba.fclr = w.F[k];
    ba.cnt_cur = cnt + i * kCntSlots;
    ba.cnt_nxt = cnt + j * kCntSlots;
    ba.cnt_clr = cnt + k * kCntSlots;
    ba.d = (int32_t)std::min<int64_t>(d, INT32_MAX);
  };
  at_level(0);
  const int64_t cap = desc.max_iter > 0 ? desc.max_iter : INT64_MAX;
  int64_t d = 0;
  const size_t rec_bytes = (size_t)kStatsCap * kStatFields * sizeof(int64_t);
  const size_t head = (size_t)((char *)w.stats - (char *)w.ctrl);
  std::vector<char> host(head + rec_bytes);
  Ctrl hc{};
  bool empty_seen = false;
  int64_t launches = 0;  // kernel launches timed by the profile events
  std::vector<int64_t> launch_level;  // first level of each launch
  // High-diameter, low-degree graphs: levels run back to back in the
  // multi-workgroup loop while the frontier is small (no launch per level);
  // a frontier that outgrows it, or a barrier it gave up, continues with the
  // level kernel below.
  const bool small = A->a.max_deg <= kCoopMaxDeg && desc.direction != GRB_DIR_PULL;
  if (small) {
    ba.coop = w.coop;
    ba.qv = w.qv;
    ba.qe = w.qe;
    ba.qseg = w.qseg;
  }
  launch_bfs_start(ba, source, w.F[1], w.F[2], stream);
  if (small) {
    if (profile) (void)hipEventRecord(g_events.get(0), s);
    uint64_t *F[3] = {w.F[0], w.F[1], w.F[2]};
    launch_bfs_coop(ba, source, cap, F, (desc.flags & GRB_LOOP_NO_WAIT) ? 0 : kCoopWaitTicks,
                    stream);
    if (profile) (void)hipEventRecord(g_events.get(1), s);
    launch_level.push_back(0);
    launches = 1;
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (!read_back({{host.data(), w.ctrl, head + rec_bytes}}, s)) return GRB_PANIC;
    std::memcpy(&hc, host.data(), sizeof(Ctrl));
    d = hc.small_levels;
    empty_seen = !hc.spilled;  // done, or stopped by the level cap
  }
  // The first batch covers the depth expected of a random graph of this
  // size and mean degree, ln n / ln(nnz / n), plus one spare, or the depth
  // of the last search on this matrix where that is larger (up to twice the
  // estimate: skewed degrees make searches deeper than the estimate); later
  // batches start at two levels and double, so a deeper search pays few
  // empty launches.  A batch whose last level found no next frontier ends
  // the search without launching the empty level.  Control block and level
  // records come back in one copy.
  int chunk = 6;
  {
    const double dbar = n > 0 ? (double)A->nnz / (double)n : 0.0;
    if (n > 1 && dbar > 1.5)
      chunk = (int)std::min(64.0, std::ceil(std::log((double)n) / std::log(dbar)) + 1.0);
    const int last = A->bfs_depth.load(std::memory_order_relaxed);
    chunk = std::max(chunk, std::min(last, 2 * chunk));
  }
  bool first_batch = true;
  bool capped = false;  // stopped by the level cap with a frontier left
  while (!empty_seen && d < cap) {
    for (int i = 0; i < chunk && d < cap; ++i, ++d) {
      at_level(d);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)launches), s);
      launch_bfs_level(ba, stream);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)launches + 1), s);
      launch_level.push_back(d);
      ++launches;
    }
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    const size_t recs = (size_t)std::min<int64_t>(d, kStatsCap) * kStatFields * sizeof(int64_t);
    if (!read_back({{host.data(), w.ctrl, head + recs}}, s)) return GRB_PANIC;
    std::memcpy(&hc, host.data(), sizeof(Ctrl));
    if (hc.nlev < d) {  // a launched level found the frontier empty
      empty_seen = true;
      break;
    }
    int32_t next = 0;  // frontier the last launched level found
    for (int t = 0; t < kCntStripes; ++t) next += hc.lists[(d % 3) * kCntSlots + kCntFields * t];
    if (next == 0) {
      empty_seen = true;
      break;
    }
    chunk = first_batch ? 2 : std::min(chunk * 2, 256);
    first_batch = false;
  }
  // parents the level kernel did not resolve: a search stopped by the level
  // cap, or levels run by the multi-workgroup loop
  capped = !empty_seen && hc.nlev >= d;
  if (parents && (small || capped)) {
    launch_bfs_parents(ba, stream);
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;
  }
  const int iters = hc.nlev;
  A->bfs_depth.store(iters, std::memory_order_relaxed);
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  const int nrec = std::min(iters, (int)kStatsCap);
  std::memcpy(rec.data(), host.data() + head, rec_bytes);
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    // per level: a level launch's time; the multi-workgroup loop's time is
    // spread evenly over the levels it ran
    kms.assign((size_t)std::max(nrec, 0), 0.0f);
    for (int64_t i = 0; i < launches; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, g_events.get(2 * (size_t)i), g_events.get(2 * (size_t)i + 1));
      ms_all += ms;
      const int64_t l0 = launch_level[(size_t)i];
      const int64_t l1 = (small && i == 0) ? std::max<int64_t>(hc.small_levels, 1) : l0 + 1;
      for (int64_t l = l0; l < l1 && l < nrec; ++l) kms[(size_t)l] = ms / (float)(l1 - l0);
    }
  }
  finish_stats(GRB_OP_BFS, iters, rec, kms, (int)std::min<int64_t>(launches, INT32_MAX), ms_all);
  return GRB_SUCCESS;
}

// SSSP: one kernel per round, same batching of rounds as BFS.
grb_info run_sssp(grb_matrix A, int32_t source, float *dist, const grb_descriptor &desc,
                  void *ws, size_t ws_bytes, void *stream) {
  const int64_t n = A->nrows;
  const bool can_pull = A->at.valid();
  if (!can_pull && desc.direction == GRB_DIR_PULL) return GRB_NOT_IMPLEMENTED;
  SsspWs sw = sssp_layout(ws, n);
  grb_info info = check_ws(ws, ws_bytes, sw.bytes);
  if (info != GRB_SUCCESS) return info;
  const BfsWs &w = sw.b;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  SsspArgs sa;
  sa.n = n;
  sa.nw = words_of(n);
  sa.nnz = A->nnz;
  sa.push = A->a;
  sa.pull = A->at;
  sa.can_pull = can_pull;
  sa.same_csr = A->symmetric;
  sa.wpush = (const float *)A->a.val;
  sa.wpull = can_pull ? (const float *)A->at.val : nullptr;
  sa.dist = dist;
  sa.iso = w.visited;
  sa.ctrl = w.ctrl;
  sa.stats = w.stats;
  sa.rule = desc.switch_rule;
  sa.denom = desc.switch_denominator;
  sa.forced = desc.direction;
  int32_t *cnt = w.ctrl->lists;
  auto at_round = [&](int64_t d) {
    const int i = (int)(d % 3), j = (int)((d + 1) % 3), k = (int)((d + 2) % 3);
    sa.fcur = w.F[i];
    sa.fnxt = w.F[j];
    sa.fclr = w.F[k];
    sa.fd_cur = sw.fd[i];
    sa.fd_nxt = sw.fd[j];
    sa.fd_clr = sw.fd[k];
    sa.cnt_cur = cnt + i * kCntSlots;
    sa.cnt_nxt = cnt + j * kCntSlots;
    sa.cnt_clr = cnt + k * kCntSlots;
    sa.d = (int32_t)std::min<int64_t>(d, INT32_MAX);
  };
  at_round(0);
  launch_sssp_start(sa, source, w.F[1], w.F[2], sw.fd[1], sw.fd[2], stream);
  const int64_t cap = desc.max_iter > 0 ? desc.max_iter : INT64_MAX;
  int64_t d = 0;
  int chunk = 8;
  Ctrl hc{};
  for (;;) {
    for (int i = 0; i < chunk && d < cap; ++i, ++d) {
      at_round(d);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)d), s);
      launch_sssp_round(sa, stream);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)d + 1), s);
    }
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (!read_back({{&hc, w.ctrl, sizeof(Ctrl)}}, s)) return GRB_PANIC;
    int64_t next = 0;
    for (int t = 0; t < kCntStripes; ++t) next += hc.lists[(d % 3) * kCntSlots + kCntFields * t];
    if (next == 0 || d >= cap) break;
    chunk = std::min(chunk * 2, 512);
  }
  const int iters = hc.nlev;
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  const int nrec = std::min(iters, (int)kStatsCap);
  if (!read_back({{rec.data(), w.stats, (size_t)std::max(nrec, 0) * kStatFields * sizeof(int64_t)}}, s))
    return GRB_PANIC;
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    for (int64_t i = 0; i < d; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, g_events.get(2 * (size_t)i), g_events.get(2 * (size_t)i + 1));
      if (i < nrec) kms.push_back(ms);
      ms_all += ms;
    }
  }
  finish_stats(GRB_OP_SSSP, iters, rec, kms, (int)std::min<int64_t>(d, INT32_MAX), ms_all);
  return GRB_SUCCESS;
}

// Bucketed SSSP: one push kernel per round over the pending set, the host
// reads the counters back once per batch of rounds.
grb_info run_sssp_delta(grb_matrix A, int32_t source, float *dist, float delta,
                        const grb_descriptor &desc, void *ws, size_t ws_bytes, void *stream) {
  const int64_t n = A->nrows;
  SsspWs sw = sssp_layout(ws, n);
  grb_info info = check_ws(ws, ws_bytes, sw.bytes);
  if (info != GRB_SUCCESS) return info;
  const BfsWs &w = sw.b;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  SsspArgs sa;
  sa.n = n;
  sa.nw = words_of(n);
  sa.nnz = A->nnz;
  sa.push = A->a;
  sa.pull = A->at;
  sa.can_pull = false;
  sa.same_csr = A->symmetric;
  sa.wpush = (const float *)A->a.val;
  sa.dist = dist;
  sa.ctrl = w.ctrl;
  sa.stats = w.stats;
  sa.delta = delta;
  int32_t *cnt = w.ctrl->lists;
  auto at_round = [&](int64_t d) {
    const int i = (int)(d % 3), j = (int)((d + 1) % 3), k = (int)((d + 2) % 3);
    sa.fcur = w.F[i];
    sa.fnxt = w.F[j];
    sa.fclr = w.F[k];
    sa.cnt_cur = cnt + i * kDeltaSlots;
    sa.cnt_nxt = cnt + j * kDeltaSlots;
    sa.cnt_clr = cnt + k * kDeltaSlots;
    sa.d = (int32_t)std::min<int64_t>(d, INT32_MAX);
  };
  at_round(0);
  // low-degree graphs: rounds back to back in the multi-workgroup loop while
  // the pending set is small (no launch per round); a larger set, or a
  // barrier the loop gave up, continues with the round kernel
  const bool small = A->a.max_deg <= kCoopMaxDeg;
  if (small) {
    sa.coop = w.coop;
    sa.qv = w.qv;
    sa.qe = w.qe;
    sa.qseg = w.qseg;
  }
  launch_sssp_delta_start(sa, source, w.F[1], w.F[2], stream);
  const int64_t cap = desc.max_iter > 0 ? desc.max_iter : INT64_MAX;
  int64_t d = 0;
  const size_t rec_bytes = (size_t)kStatsCap * kStatFields * sizeof(int64_t);
  const size_t head = (size_t)((char *)w.stats - (char *)w.ctrl);
  std::vector<char> host(head + rec_bytes);
  Ctrl hc{};
  bool done = false;
  int64_t launches = 0;
  std::vector<int64_t> launch_round;
  if (small) {
    if (profile) (void)hipEventRecord(g_events.get(0), s);
    uint64_t *F[3] = {w.F[0], w.F[1], w.F[2]};
    launch_sssp_delta_coop(sa, cap, F, (desc.flags & GRB_LOOP_NO_WAIT) ? 0 : kCoopWaitTicks,
                           stream);
    if (profile) (void)hipEventRecord(g_events.get(1), s);
    launch_round.push_back(0);
    launches = 1;
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (!read_back({{host.data(), w.ctrl, head + rec_bytes}}, s)) return GRB_PANIC;
    std::memcpy(&hc, host.data(), sizeof(Ctrl));
    d = hc.small_levels;
    done = !hc.spilled;
  }
  int chunk = 16;
  while (!done && d < cap) {
    for (int i = 0; i < chunk && d < cap; ++i, ++d) {
      at_round(d);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)launches), s);
      launch_sssp_delta_round(sa, stream);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)launches + 1), s);
      launch_round.push_back(d);
      ++launches;
    }
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    const size_t recs = (size_t)std::min<int64_t>(d, kStatsCap) * kStatFields * sizeof(int64_t);
    if (!read_back({{host.data(), w.ctrl, head + recs}}, s)) return GRB_PANIC;
    std::memcpy(&hc, host.data(), sizeof(Ctrl));
    if (hc.nlev < d) break;  // a launched round found nothing pending
    chunk = std::min(chunk * 2, 512);
  }
  const int iters = hc.nlev;
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  std::memcpy(rec.data(), host.data() + head, rec_bytes);
  const int nrec = std::min(iters, (int)kStatsCap);
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    // per round: a round launch's time; the multi-workgroup loop's time is
    // spread evenly over the rounds it ran
    kms.assign((size_t)std::max(nrec, 0), 0.0f);
    for (int64_t i = 0; i < launches; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, g_events.get(2 * (size_t)i), g_events.get(2 * (size_t)i + 1));
      ms_all += ms;
      const int64_t l0 = launch_round[(size_t)i];
      const int64_t l1 = (small && i == 0) ? std::max<int64_t>(hc.small_levels, 1) : l0 + 1;
      for (int64_t l = l0; l < l1 && l < nrec; ++l) kms[(size_t)l] = ms / (float)(l1 - l0);
    }
  }
  finish_stats(GRB_OP_SSSP, iters, rec, kms, (int)std::min<int64_t>(launches, INT32_MAX), ms_all);
  return GRB_SUCCESS;
}

// PageRank and adaptive PageRank: batches of 8 iterations, the host reads
// the control block back after each batch (the device decides convergence).
grb_info run_pagerank(void *p, grb_type type, grb_matrix A, double damping, int32_t max_iter,
                      double tol, bool adaptive, double eps, int32_t *iters, double *delta_out,
                      int64_t *active_out, const grb_descriptor *d, void *ws, size_t ws_bytes,
                      void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!p || !iters) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (type != GRB_FP32 && type != GRB_FP64) return GRB_DOMAIN_MISMATCH;
  if (A->nrows == 0 || max_iter < 0 || !(damping >= 0.0 && damping <= 1.0) || !(tol >= 0.0))
    return GRB_INVALID_VALUE;
  if (!A->at.valid()) return GRB_NOT_IMPLEMENTED;
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  const int is64 = type == GRB_FP64;
  const int64_t n = A->nrows;
  PrWs w = pr_layout(ws, n, A->at, is64 ? 8 : 4);
  if ((info = check_ws(ws, ws_bytes, w.bytes)) != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  PrArgs pa;
  pa.n = n;
  pa.nw = words_of(n);
  pa.pull = A->at;
  pa.out_rp = A->a.rp;
  pa.p = p;
  pa.x = w.x0;
  pa.xn = w.x0;
  pa.heavy_part = w.heavy_part;
  pa.blk_part = w.blk_part;
  pa.nblk = w.nblk;
  pa.nblk_long = w.nblk_long;
  pa.ctrl = w.ctrl;
  pa.stats = w.stats;
  pa.alpha = damping;
  pa.tol = tol;
  pa.eps = eps;
  auto at_iter = [&](int k) {
    if (!adaptive) return;
    pa.act_cur = w.act[k % 3];
    pa.act_nxt = w.act[(k + 1) % 3];
    pa.act_prev = w.act[(k + 2) % 3];
  };
  at_iter(0);
  launch_pr_init(is64, pa, stream);
  Ctrl hc{};
  int k = 0;
  while (k < max_iter) {
    const int stop = std::min(max_iter, k + 8);
    for (; k < stop; ++k) {
      pa.x = (k % 2 == 0) ? w.x0 : w.x1;
      pa.xn = (k % 2 == 0) ? w.x1 : w.x0;
      at_iter(k);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)k), s);
      launch_pr_iter(is64, pa, stream);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)k + 1), s);
    }
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (!read_back({{&hc, w.ctrl, sizeof(Ctrl)}}, s)) return GRB_PANIC;
    if (hc.converged) break;
  }
  if (max_iter == 0) {
    if (!read_back({{&hc, w.ctrl, sizeof(Ctrl)}}, s)) return GRB_PANIC;
  }
  *iters = hc.iters;
  if (delta_out) *delta_out = hc.delta;
  if (active_out) *active_out = adaptive ? hc.active : 0;
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  const int nrec = std::min(hc.iters, (int)kStatsCap);
  if (adaptive) {
    if (!read_back({{rec.data(), w.stats, (size_t)std::max(nrec, 0) * kStatFields * sizeof(int64_t)}},
                   s))
      return GRB_PANIC;
  } else {
    for (int i = 0; i < nrec; ++i) {
      rec[(size_t)i * kStatFields + 0] = n;
      rec[(size_t)i * kStatFields + 1] = A->nnz;
      rec[(size_t)i * kStatFields + 2] = GRB_DIR_PULL;
    }
  }
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    for (int i = 0; i < k; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, g_events.get(2 * (size_t)i), g_events.get(2 * (size_t)i + 1));
      if (i < nrec) kms.push_back(ms);
      ms_all += ms;
    }
  }
  finish_stats(GRB_OP_PAGERANK, hc.iters, rec, kms, k, ms_all);
  return GRB_SUCCESS;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

int32_t grb_version(void) { return 100; }

const char *grb_error_string(grb_info info) {
  switch (info) {
    case GRB_SUCCESS: return "success";
    case GRB_NO_VALUE: return "no value";
    case GRB_UNINITIALIZED_OBJECT: return "uninitialized object (NULL handle or matrix not prepared)";
    case GRB_NULL_POINTER: return "required pointer is NULL";
    case GRB_INVALID_VALUE: return "invalid value";
    case GRB_INVALID_INDEX: return "index out of range";
    case GRB_DOMAIN_MISMATCH: return "type does not match the semiring";
    case GRB_DIMENSION_MISMATCH: return "dimension mismatch";
    case GRB_NOT_IMPLEMENTED: return "not implemented";
    case GRB_INSUFFICIENT_SPACE: return "workspace or metadata buffer too small";
    case GRB_OUT_OF_MEMORY: return "host allocation failed";
    case GRB_PANIC: return "HIP runtime or device error";
  }
  return "unknown error code";
}

grb_info grb_descriptor_init(grb_descriptor *d) {
  if (!d) return GRB_NULL_POINTER;
  std::memset(d, 0, sizeof(*d));
  d->direction = GRB_DIR_AUTO;
  d->switch_rule = GRB_SWITCH_PAPER;
  d->switch_denominator = 10;
  return GRB_SUCCESS;
}

grb_info grb_last_stats(grb_stats *s) {
  if (!s) return GRB_NULL_POINTER;
  *s = g_stats;
  return GRB_SUCCESS;
}

grb_info grb_stream_check(void *stream) {
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GRB_PANIC;
  return check_launch();
}

// ---- matrix ------------------------------------------------------------------

grb_info grb_matrix_create(grb_matrix *A, int64_t nrows, int64_t ncols, int64_t nnz,
                           const int32_t *row_ptr, const int32_t *col_idx, const void *values,
                           grb_type vtype, const int32_t *t_row_ptr, const int32_t *t_col_idx,
                           const void *t_values, uint32_t flags) {
  if (!A) return GRB_NULL_POINTER;
  *A = nullptr;
  if (nrows < 0 || ncols < 0 || nnz < 0 || nrows >= INT32_MAX || ncols >= INT32_MAX ||
      nnz > INT32_MAX)
    return GRB_INVALID_VALUE;
  if (flags & ~GRB_MATRIX_SYMMETRIC) return GRB_INVALID_VALUE;
  if (!row_ptr || (nnz > 0 && !col_idx)) return GRB_NULL_POINTER;
  if (values && vtype != GRB_INT32 && vtype != GRB_FP32 && vtype != GRB_FP64)
    return GRB_INVALID_VALUE;
  const bool sym = (flags & GRB_MATRIX_SYMMETRIC) != 0;
  if (sym && (nrows != ncols || t_row_ptr || t_col_idx || t_values)) return GRB_INVALID_VALUE;
  if (!t_row_ptr && (t_col_idx || t_values)) return GRB_INVALID_VALUE;
  if (t_row_ptr && nnz > 0 && !t_col_idx) return GRB_NULL_POINTER;
  if (t_values && !values) return GRB_INVALID_VALUE;
  if (values && t_row_ptr && !t_values) return GRB_NULL_POINTER;
  grb_matrix_s *m = new (std::nothrow) grb_matrix_s;
  if (!m) return GRB_OUT_OF_MEMORY;
  m->nrows = nrows;
  m->ncols = ncols;
  m->nnz = nnz;
  m->symmetric = sym;
  m->a.rp = row_ptr;
  m->a.ci = col_idx;
  m->a.val = values;
  m->a.vtype = values ? (int)vtype : -1;
  m->a.nrows = nrows;
  m->a.ncols = ncols;
  m->a.nnz = nnz;
  if (sym) {
    m->at = m->a;
  } else if (t_row_ptr) {
    m->at.rp = t_row_ptr;
    m->at.ci = t_col_idx;
    m->at.val = t_values;
    m->at.vtype = t_values ? (int)vtype : -1;
    m->at.nrows = ncols;
    m->at.ncols = nrows;
    m->at.nnz = nnz;
  }
  *A = m;
  return GRB_SUCCESS;
}

grb_info grb_matrix_free(grb_matrix *A) {
  if (!A) return GRB_NULL_POINTER;
  delete *A;
  *A = nullptr;
  return GRB_SUCCESS;
}

grb_info grb_matrix_nrows(grb_matrix A, int64_t *n) {
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  if (!n) return GRB_NULL_POINTER;
  *n = A->nrows;
  return GRB_SUCCESS;
}

grb_info grb_matrix_ncols(grb_matrix A, int64_t *n) {
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  if (!n) return GRB_NULL_POINTER;
  *n = A->ncols;
  return GRB_SUCCESS;
}

grb_info grb_matrix_nvals(grb_matrix A, int64_t *nnz) {
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  if (!nnz) return GRB_NULL_POINTER;
  *nnz = A->nnz;
  return GRB_SUCCESS;
}

grb_info grb_matrix_meta_size(grb_matrix A, size_t *bytes) {
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  if (!bytes) return GRB_NULL_POINTER;
  MetaLayout la = meta_layout_one(A->nnz, A->nrows, 0);
  size_t total = la.bytes;
  if (!A->symmetric && A->at.valid()) total = meta_layout_one(A->nnz, A->ncols, total).bytes;
  *bytes = total;
  return GRB_SUCCESS;
}

grb_info grb_matrix_prepare(grb_matrix A, void *meta, size_t meta_bytes, void *stream) {
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  size_t need = 0;
  grb_matrix_meta_size(A, &need);
  if (meta_bytes < need) return GRB_INSUFFICIENT_SPACE;
  if (!meta) return GRB_NULL_POINTER;
  if (((uintptr_t)meta) % 256 != 0) return GRB_INVALID_VALUE;
  hipStream_t s = (hipStream_t)stream;
  MetaLayout la = meta_layout_one(A->nnz, A->nrows, 0);
  grb_info info = build_meta(A->a, (char *)meta, la, s);
  if (info != GRB_SUCCESS) return info;
  if (A->symmetric) {
    A->at = A->a;
  } else if (A->at.valid()) {
    MetaLayout lt = meta_layout_one(A->nnz, A->ncols, la.bytes);
    info = build_meta(A->at, (char *)meta, lt, s);
    if (info != GRB_SUCCESS) return info;
  }
  A->prepared = true;
  return GRB_SUCCESS;
}

// ---- vector ------------------------------------------------------------------

grb_info grb_vector_create(grb_vector *v, int64_t n, grb_type type, void *values,
                           uint64_t *bitmap, int32_t *indices, int32_t *count) {
  if (!v) return GRB_NULL_POINTER;
  *v = nullptr;
  if (n < 0 || n >= INT32_MAX || !valid_type(type)) return GRB_INVALID_VALUE;
  if ((indices == nullptr) != (count == nullptr)) return GRB_NULL_POINTER;
  if (n > 0 && !bitmap && !indices) return GRB_NULL_POINTER;  // no presence storage
  grb_vector_s *x = new (std::nothrow) grb_vector_s;
  if (!x) return GRB_OUT_OF_MEMORY;
  x->n = n;
  x->type = type;
  x->values = values;
  x->bitmap = bitmap;
  x->indices = indices;
  x->count = count;
  *v = x;
  return GRB_SUCCESS;
}

grb_info grb_vector_free(grb_vector *v) {
  if (!v) return GRB_NULL_POINTER;
  delete *v;
  *v = nullptr;
  return GRB_SUCCESS;
}

grb_info grb_vector_size(grb_vector v, int64_t *n) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (!n) return GRB_NULL_POINTER;
  *n = v->n;
  return GRB_SUCCESS;
}

grb_info grb_vector_clear(grb_vector v, void *stream) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (v->bitmap) launch_fill_u64(v->bitmap, words_of(v->n), 0ull, stream);
  if (v->count) {
    const int32_t zero = 0;
    launch_fill_bytes_pattern(v->count, 1, 4, &zero, stream);
  }
  return check_launch();
}

grb_info grb_vector_fill(grb_vector v, const void *scalar, void *stream) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (!scalar && v->values) return GRB_NULL_POINTER;
  if (v->n == 0) return grb_vector_clear(v, stream);
  if (v->values) launch_fill_bytes_pattern(v->values, v->n, elem_size(v->type), scalar, stream);
  if (v->bitmap) {
    const int64_t nw = words_of(v->n);
    launch_fill_u64(v->bitmap, nw, ~0ull, stream);
    if (v->n % 64) launch_fill_u64(v->bitmap + nw - 1, 1, (1ull << (v->n % 64)) - 1, stream);
  }
  if (v->indices) launch_iota(v->indices, v->n, v->count, stream);
  return check_launch();
}

grb_info grb_vector_build(grb_vector v, const int32_t *idx, const void *vals, int64_t count,
                          void *stream) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (count < 0) return GRB_INVALID_VALUE;
  if (count > 0 && !idx) return GRB_NULL_POINTER;
  if (vals && !v->values) return GRB_INVALID_VALUE;  // the vector stores no values
  if (!v->bitmap) return GRB_NOT_IMPLEMENTED;       // a list-only vector is written by its owner
  uint64_t one = 0;
  switch (v->type) {
    case GRB_BOOL: one = 1; break;
    case GRB_INT32: one = 1; break;
    case GRB_FP32: { float f = 1.0f; std::memcpy(&one, &f, 4); break; }
    case GRB_FP64: { double f = 1.0; std::memcpy(&one, &f, 8); break; }
  }
  launch_vector_build(v->bitmap, v->values, elem_size(v->type), v->n, idx, vals, count, one, stream);
  // the list (if the vector keeps one) follows the bitmap
  if (v->indices) launch_bitmap_to_list_small(v->bitmap, v->n, v->indices, v->count, stream);
  return check_launch();
}

grb_info grb_vector_nvals(grb_vector v, int64_t *nvals, void *ws, size_t ws_bytes, void *stream) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (!nvals) return GRB_NULL_POINTER;
  grb_info info = check_ws(ws, ws_bytes, 64);
  if (info != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  if (!v->bitmap) {
    int32_t c = 0;
    if (!read_back({{&c, v->count, sizeof(c)}}, s)) return GRB_PANIC;
    *nvals = std::min<int64_t>(std::max<int32_t>(c, 0), v->n);
    return GRB_SUCCESS;
  }
  launch_popcount(v->bitmap, words_of(v->n), (int64_t *)ws, stream);
  if ((info = check_launch()) != GRB_SUCCESS) return info;
  int64_t h = 0;
  if (!read_back({{&h, ws, sizeof(h)}}, s)) return GRB_PANIC;
  *nvals = h;
  return GRB_SUCCESS;
}

grb_info grb_vector_extract(grb_vector v, int32_t *indices, void *values, int64_t capacity,
                            int64_t *nvals, void *ws, size_t ws_bytes, void *stream) {
  if (!v) return GRB_UNINITIALIZED_OBJECT;
  if (!nvals) return GRB_NULL_POINTER;
  if (capacity < 0) return GRB_INVALID_VALUE;
  ExtractWs t = extract_layout(ws, v->n);
  grb_info info = check_ws(ws, ws_bytes, t.bytes);
  if (info != GRB_SUCCESS) return info;
  if (v->n == 0) {
    *nvals = 0;
    return GRB_SUCCESS;
  }
  hipStream_t s = (hipStream_t)stream;
  const int32_t *list = v->indices;
  const int32_t *cnt = v->count;
  if (!list) {
    // bitmap -> sorted list in the workspace (the compaction's look-back
    // needs its status words and ticket cleared first)
    launch_fill_u64((uint64_t *)t.ctrl, sizeof(Ctrl) / 8, 0ull, stream);
    launch_fill_u64(t.status, 2 * (int64_t)t.nblk, 0ull, stream);
    CompactArgs ca;
    ca.nb = v->bitmap;
    ca.nw = words_of(v->n);
    ca.nbits = v->n;
    ca.list = t.list;
    ca.status_cur = t.status;
    ca.status_next = t.status + t.nblk;
    ca.ctrl = t.ctrl;
    ca.count_out = t.cnt;
    launch_compact(ca, stream);
    list = t.list;
    cnt = t.cnt;
  }
  const int esz = elem_size(v->type);
  if (v->values && values)
    launch_gather_values(v->values, esz, list, cnt, v->n, t.vals, stream);
  if ((info = check_launch()) != GRB_SUCCESS) return info;
  int32_t c = 0;
  if (!read_back({{&c, cnt, sizeof(c)}}, s)) return GRB_PANIC;
  const int64_t m = std::min<int64_t>(std::max<int32_t>(c, 0), v->n);
  *nvals = m;
  if (m > capacity) return GRB_INSUFFICIENT_SPACE;
  if (m > 0) {
    if (indices && hipMemcpyAsync(indices, list, (size_t)m * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return GRB_PANIC;
    if (values) {
      if (v->values) {
        if (hipMemcpyAsync(values, t.vals, (size_t)m * esz, hipMemcpyDeviceToHost, s) != hipSuccess)
          return GRB_PANIC;
      } else {
        // a vector without values holds 1 at every entry
        for (int64_t k = 0; k < m; ++k) {
          char *dst = (char *)values + k * esz;
          switch (v->type) {
            case GRB_BOOL: *(uint8_t *)dst = 1; break;
            case GRB_INT32: *(int32_t *)dst = 1; break;
            case GRB_FP32: *(float *)dst = 1.0f; break;
            default: *(double *)dst = 1.0; break;
          }
        }
      }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;
  }
  return GRB_SUCCESS;
}

// ---- workspace -----------------------------------------------------------------

grb_info grb_workspace_size(grb_op op, grb_matrix A, int64_t k, size_t *bytes) {
  if (!bytes) return GRB_NULL_POINTER;
  if (op == GRB_OP_NVALS) {
    *bytes = 256;
    return GRB_SUCCESS;
  }
  if (op == GRB_OP_MXM) {
    *bytes = kMxmWs;
    return GRB_SUCCESS;
  }
  if (op == GRB_OP_CC) {
    if (!A) return GRB_UNINITIALIZED_OBJECT;
    size_t mb = 0;
    grb_info info = grb_workspace_size(GRB_OP_MXV, A, 0, &mb);
    if (info != GRB_SUCCESS) return info;
    *bytes = cc_layout(nullptr, A->nrows, mb).bytes;
    return GRB_SUCCESS;
  }
  if (op == GRB_OP_EXTRACT) {
    if (k < 0 || k >= INT32_MAX) return GRB_INVALID_VALUE;
    *bytes = extract_layout(nullptr, k).bytes;
    return GRB_SUCCESS;
  }
  if (!A) return GRB_UNINITIALIZED_OBJECT;
  switch (op) {
    case GRB_OP_BFS: *bytes = bfs_layout(nullptr, A->nrows).bytes; break;
    case GRB_OP_SSSP: *bytes = sssp_layout(nullptr, A->nrows).bytes; break;
    case GRB_OP_PAGERANK: {
      if (k != 1 && k != 2) return GRB_INVALID_VALUE;
      Csr pull = A->at;
      pull.nsplit = split_bound(A->nnz);
      pull.nsplit_rows = A->nnz / (kPushSplit + 1) + 1;
      *bytes = pr_layout(nullptr, A->nrows, pull, k == 2 ? 8 : 4).bytes;
      break;
    }
    case GRB_OP_MSBFS:
      if (k < 1 || k > INT32_MAX) return GRB_INVALID_VALUE;
      *bytes = ms_layout(nullptr, A->nrows, k).bytes;
      break;
    case GRB_OP_MXV: {
      const int64_t m = std::max(A->nrows, A->ncols);
      *bytes = mxv_layout(nullptr, m, m, A->nnz, split_bound(A->nnz)).bytes;
      break;
    }
    default: return GRB_INVALID_VALUE;
  }
  return GRB_SUCCESS;
}

// ---- drivers -------------------------------------------------------------------

grb_info grb_bfs(int32_t *levels, int32_t *parents, grb_matrix A, int32_t source,
                 const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!levels) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (source < 0 || source >= A->nrows) return GRB_INVALID_INDEX;
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  return run_bfs(A, source, levels, parents, desc, ws, ws_bytes, stream);
}

grb_info grb_sssp(float *dist, grb_matrix A, int32_t source, const grb_descriptor *d, void *ws,
                  size_t ws_bytes, void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!dist) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (source < 0 || source >= A->nrows) return GRB_INVALID_INDEX;
  if (A->a.vtype != GRB_FP32) return GRB_DOMAIN_MISMATCH;
  if (A->a.negative || A->at.negative) return GRB_INVALID_VALUE;  // min-plus needs weights >= 0
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  return run_sssp(A, source, dist, desc, ws, ws_bytes, stream);
}

grb_info grb_sssp_delta(float *dist, grb_matrix A, int32_t source, float delta,
                        const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!dist) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (source < 0 || source >= A->nrows) return GRB_INVALID_INDEX;
  if (A->a.vtype != GRB_FP32) return GRB_DOMAIN_MISMATCH;
  if (A->a.negative || A->at.negative) return GRB_INVALID_VALUE;  // min-plus needs weights >= 0
  if (!(delta > 0.0f) || !(delta < 3.0e38f)) return GRB_INVALID_VALUE;
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  if (desc.direction == GRB_DIR_PULL) return GRB_NOT_IMPLEMENTED;
  return run_sssp_delta(A, source, dist, delta, desc, ws, ws_bytes, stream);
}

grb_info grb_msbfs(int32_t *levels, grb_matrix A, const int32_t *sources, int32_t k,
                   const grb_msbfs_tile *tile, const grb_descriptor *d, void *ws, size_t ws_bytes,
                   void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!levels || !sources) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (k < 1) return GRB_INVALID_VALUE;
  const int W = (int)((k + 63) / 64);
  int kt = W, grid = kExpandGrid;
  if (tile) {
    if (tile->reserved[0] || tile->reserved[1] || tile->words_per_pass < 0 ||
        tile->words_per_pass > W || tile->grid < 0 || tile->grid > 65535)
      return GRB_INVALID_VALUE;
    if (tile->words_per_pass) kt = tile->words_per_pass;
    if (tile->grid) grid = tile->grid;
  }
  kt = std::min(kt, kMsMaxWordsPerPass);
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  const bool can_pull = A->at.valid();
  if (desc.direction == GRB_DIR_PULL && !can_pull) return GRB_NOT_IMPLEMENTED;
  const int64_t n = A->nrows;
  MsWs w = ms_layout(ws, n, k);
  if ((info = check_ws(ws, ws_bytes, w.bytes)) != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  MsbfsArgs ma;
  ma.n = n;
  ma.nw = words_of(n);
  ma.nnz = A->nnz;
  ma.k = k;
  ma.W = W;
  ma.kt = kt;
  ma.push = A->a;
  ma.pull = A->at;
  ma.can_pull = can_pull;
  ma.levels = levels;
  ma.V = w.V;
  ma.cnt_base = w.cnt;
  ma.ctrl = w.ctrl;
  ma.stats = w.stats;
  ma.rule = desc.switch_rule;
  ma.denom = desc.switch_denominator;
  ma.forced = desc.direction;
  auto at_level = [&](int64_t dd) {
    const int i = (int)(dd % 3), j = (int)((dd + 1) % 3), q = (int)((dd + 2) % 3);
    ma.F = w.F[i];
    ma.Fn = w.F[j];
    ma.Fc = w.F[q];
    ma.act = w.act[i];
    ma.actn = w.act[j];
    ma.actc = w.act[q];
    ma.cnt_cur = w.cnt + (size_t)i * 2 * kCntStripes;
    ma.cnt_nxt = w.cnt + (size_t)j * 2 * kCntStripes;
    ma.cnt_clr = w.cnt + (size_t)q * 2 * kCntStripes;
    ma.d = (int32_t)std::min<int64_t>(dd, INT32_MAX);
  };
  at_level(0);
  launch_msbfs_start(ma, sources, w.F[1], w.F[2], w.act[1], w.act[2], stream);
  const int64_t cap = desc.max_iter > 0 ? desc.max_iter : INT64_MAX;
  int64_t dlev = 0;
  int chunk = 6;
  std::vector<unsigned long long> hcnt((size_t)6 * kCntStripes);
  Ctrl hc{};
  for (;;) {
    for (int i = 0; i < chunk && dlev < cap; ++i, ++dlev) {
      at_level(dlev);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)dlev), s);
      launch_msbfs_level(ma, grid, stream);
      if (profile) (void)hipEventRecord(g_events.get(2 * (size_t)dlev + 1), s);
    }
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (!read_back({{hcnt.data(), w.cnt, hcnt.size() * sizeof(unsigned long long)},
                    {&hc, w.ctrl, sizeof(Ctrl)}},
                   s))
      return GRB_PANIC;
    unsigned long long next = 0;
    for (int t = 0; t < kCntStripes; ++t) next += hcnt[(size_t)(dlev % 3) * 2 * kCntStripes + 2 * t];
    if (next == 0 || dlev >= cap) break;
    chunk = std::min(chunk * 2, 256);
  }
  const int iters = hc.nlev;
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  const int nrec = std::min(iters, (int)kStatsCap);
  if (!read_back({{rec.data(), w.stats, (size_t)std::max(nrec, 0) * kStatFields * sizeof(int64_t)}}, s))
    return GRB_PANIC;
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    for (int64_t i = 0; i < dlev; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, g_events.get(2 * (size_t)i), g_events.get(2 * (size_t)i + 1));
      if (i < nrec) kms.push_back(ms);
      ms_all += ms;
    }
  }
  finish_stats(GRB_OP_MSBFS, iters, rec, kms, (int)std::min<int64_t>(dlev, INT32_MAX), ms_all);
  // a source outside [0, n) was skipped on the device; the others ran to the end
  return hc.error ? GRB_INVALID_INDEX : GRB_SUCCESS;
}

}  // extern "C"

// ---- batched BFS sessions (continuous batching) ---------------------------------

struct grb_msbfs_session_s {
  grb_matrix A = nullptr;
  MsWs w{};
  MsbfsArgs ma;
  int64_t d = 0;  // levels run so far
  int grid = 0;
  std::vector<uint64_t> busy;  // queries joined and not yet retired
};

namespace {

void session_level(grb_msbfs_session_s &ss, int64_t dd) {
  const int i = (int)(dd % 3), j = (int)((dd + 1) % 3), q = (int)((dd + 2) % 3);
  MsbfsArgs &ma = ss.ma;
  ma.F = ss.w.F[i];
  ma.Fn = ss.w.F[j];
  ma.Fc = ss.w.F[q];
  ma.act = ss.w.act[i];
  ma.actn = ss.w.act[j];
  ma.actc = ss.w.act[q];
  ma.cnt_cur = ss.w.cnt + (size_t)i * 2 * kCntStripes;
  ma.cnt_nxt = ss.w.cnt + (size_t)j * 2 * kCntStripes;
  ma.cnt_clr = ss.w.cnt + (size_t)q * 2 * kCntStripes;
  ma.alive_nxt = ss.w.alive + (size_t)j * ma.W;
  ma.alive_clr = ss.w.alive + (size_t)q * ma.W;
  ma.d = (int32_t)std::min<int64_t>(dd, INT32_MAX);
}

}  // namespace

extern "C" {

grb_info grb_msbfs_session_create(grb_msbfs_session *ss, grb_matrix A, int32_t k, int32_t *levels,
                                  const grb_msbfs_tile *tile, const grb_descriptor *d, void *ws,
                                  size_t ws_bytes, void *stream) {
  if (!ss) return GRB_NULL_POINTER;
  *ss = nullptr;
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!levels) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (k < 1) return GRB_INVALID_VALUE;
  const int W = (int)((k + 63) / 64);
  int kt = W, grid = kExpandGrid;
  if (tile) {
    if (tile->reserved[0] || tile->reserved[1] || tile->words_per_pass < 0 ||
        tile->words_per_pass > W || tile->grid < 0 || tile->grid > 65535)
      return GRB_INVALID_VALUE;
    if (tile->words_per_pass) kt = tile->words_per_pass;
    if (tile->grid) grid = tile->grid;
  }
  kt = std::min(kt, kMsMaxWordsPerPass);
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  const bool can_pull = A->at.valid();
  if (desc.direction == GRB_DIR_PULL && !can_pull) return GRB_NOT_IMPLEMENTED;
  const int64_t n = A->nrows;
  MsWs w = ms_layout(ws, n, k);
  if ((info = check_ws(ws, ws_bytes, w.bytes)) != GRB_SUCCESS) return info;
  grb_msbfs_session_s *x = new (std::nothrow) grb_msbfs_session_s;
  if (!x) return GRB_OUT_OF_MEMORY;
  try {
    x->busy.assign((size_t)W, 0ull);
  } catch (const std::bad_alloc &) {
    delete x;
    return GRB_OUT_OF_MEMORY;
  }
  x->A = A;
  x->w = w;
  x->grid = grid;
  MsbfsArgs &ma = x->ma;
  ma.n = n;
  ma.nw = words_of(n);
  ma.nnz = A->nnz;
  ma.k = k;
  ma.W = W;
  ma.kt = kt;
  ma.push = A->a;
  ma.pull = A->at;
  ma.can_pull = can_pull;
  ma.levels = levels;
  ma.V = w.V;
  ma.cnt_base = w.cnt;
  ma.ctrl = w.ctrl;
  ma.stats = nullptr;
  ma.rule = desc.switch_rule;
  ma.denom = desc.switch_denominator;
  ma.forced = desc.direction;
  ma.start = w.start;
  session_level(*x, 0);
  launch_msbfs_session_init(ma, w.F[1], w.F[2], w.act[1], w.act[2], w.alive, stream);
  if ((info = check_launch()) != GRB_SUCCESS) {
    delete x;
    return info;
  }
  *ss = x;
  return GRB_SUCCESS;
}

grb_info grb_msbfs_session_join(grb_msbfs_session ss, const int32_t *lanes,
                                const int32_t *sources, int32_t count, void *stream) {
  if (!ss) return GRB_UNINITIALIZED_OBJECT;
  if (count < 0 || count > ss->ma.k) return GRB_INVALID_VALUE;
  if (count == 0) return GRB_SUCCESS;
  if (!lanes || !sources) return GRB_NULL_POINTER;
  const int W = ss->ma.W;
  std::vector<uint64_t> clr((size_t)W, 0ull);
  for (int32_t i = 0; i < count; ++i) {
    const int32_t q = lanes[i], v = sources[i];
    if (q < 0 || q >= ss->ma.k || v < 0 || v >= ss->ma.n) return GRB_INVALID_INDEX;
    const uint64_t bit = 1ull << (q & 63);
    // a query still running, or named twice, cannot join
    if ((ss->busy[(size_t)(q >> 6)] | clr[(size_t)(q >> 6)]) & bit) return GRB_INVALID_VALUE;
    clr[(size_t)(q >> 6)] |= bit;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(ss->w.clr, clr.data(), (size_t)W * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ss->w.lanes, lanes, (size_t)count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ss->w.sources, sources, (size_t)count * 4, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return GRB_PANIC;
  session_level(*ss, ss->d);
  launch_msbfs_session_join(ss->ma, ss->w.lanes, ss->w.sources, count, ss->w.clr, ss->w.start,
                            ss->w.alive + (size_t)(ss->d % 3) * W, stream);
  grb_info info = check_launch();
  if (info != GRB_SUCCESS) return info;
  if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;  // host arrays are released
  for (int j = 0; j < W; ++j) ss->busy[(size_t)j] |= clr[(size_t)j];
  return GRB_SUCCESS;
}

grb_info grb_msbfs_session_step(grb_msbfs_session ss, int32_t max_levels, uint64_t *done,
                                int32_t *levels_run, void *stream) {
  if (!ss) return GRB_UNINITIALIZED_OBJECT;
  if (max_levels < 0) return GRB_INVALID_VALUE;
  if (!done) return GRB_NULL_POINTER;
  const int W = ss->ma.W;
  bool any = false;
  for (int j = 0; j < W; ++j) any |= ss->busy[(size_t)j] != 0ull;
  int32_t ran = 0;
  hipStream_t s = (hipStream_t)stream;
  if (any) {
    for (; ran < max_levels; ++ran, ++ss->d) {
      session_level(*ss, ss->d);
      launch_msbfs_level(ss->ma, ss->grid, stream);
    }
  }
  grb_info info = check_launch();
  if (info != GRB_SUCCESS) return info;
  std::vector<uint64_t> alive((size_t)W, 0ull);
  if (!read_back({{alive.data(), ss->w.alive + (size_t)(ss->d % 3) * W, (size_t)W * 8}}, s))
    return GRB_PANIC;
  for (int j = 0; j < W; ++j) {
    done[j] = ss->busy[(size_t)j] & ~alive[(size_t)j];
    ss->busy[(size_t)j] &= alive[(size_t)j];
  }
  if (levels_run) *levels_run = ran;
  return GRB_SUCCESS;
}

grb_info grb_msbfs_session_extract(grb_msbfs_session ss, const int32_t *lanes, int32_t count,
                                   int32_t *out, void *stream) {
  if (!ss) return GRB_UNINITIALIZED_OBJECT;
  if (count < 0 || count > ss->ma.k) return GRB_INVALID_VALUE;
  if (count == 0) return GRB_SUCCESS;
  if (!lanes || !out) return GRB_NULL_POINTER;
  for (int32_t i = 0; i < count; ++i)
    if (lanes[i] < 0 || lanes[i] >= ss->ma.k) return GRB_INVALID_INDEX;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(ss->w.lanes, lanes, (size_t)count * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return GRB_PANIC;
  launch_msbfs_session_extract(ss->ma, ss->w.lanes, count, out, stream);
  grb_info info = check_launch();
  if (info != GRB_SUCCESS) return info;
  if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;
  return GRB_SUCCESS;
}

grb_info grb_msbfs_session_free(grb_msbfs_session *ss) {
  if (!ss) return GRB_NULL_POINTER;
  delete *ss;
  *ss = nullptr;
  return GRB_SUCCESS;
}

grb_info grb_cc(int32_t *labels, grb_matrix A, int32_t *iters, const grb_descriptor *d,
                void *ws, size_t ws_bytes, void *stream) {
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (!labels) return GRB_NULL_POINTER;
  if (A->nrows != A->ncols) return GRB_DIMENSION_MISMATCH;
  if (!A->symmetric && !A->at.valid()) return GRB_NOT_IMPLEMENTED;  // needs both directions
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  if (desc.flags & ~(uint32_t)GRB_PROFILE) return GRB_INVALID_VALUE;
  size_t mb = 0;
  if ((info = grb_workspace_size(GRB_OP_MXV, A, 0, &mb)) != GRB_SUCCESS) return info;
  const int64_t n = A->nrows;
  CcWs t = cc_layout(ws, n, mb);
  if ((info = check_ws(ws, ws_bytes, t.bytes)) != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  CcArgs a;
  a.n = n;
  a.nw = words_of(n);
  a.f = t.f;
  a.f_old = t.f_old;
  a.gf = t.gf;
  a.mngf = t.mngf;
  a.labels = labels;
  a.gf_bm = t.gf_bm;
  a.mngf_bm = t.mngf_bm;
  a.changed = t.changed;
  int32_t it = 0;
  if (n > 0) {
    launch_cc_init(a, stream);
    grb_vector_s gfv, mnv;
    gfv.n = mnv.n = n;
    gfv.type = mnv.type = GRB_INT32;
    gfv.values = t.gf;
    gfv.bitmap = t.gf_bm;
    mnv.values = t.mngf;
    mnv.bitmap = t.mngf_bm;
    // the product: mngf = min(mngf, A (min, second) gf); a directed matrix
    // also takes A^T (weak components)
    grb_descriptor pd = desc;
    pd.flags = 0;
    grb_descriptor pt = pd;
    pt.flags = GRB_TRAN_A;
    const int64_t cap = desc.max_iter > 0 ? desc.max_iter : (int64_t)INT32_MAX;
    int chunk = 4;
    bool done = false;
    // per-iteration change counts, a ring of kStatsCap slots (cleared before
    // each batch reuses them); the first kStatsCap go to the stats
    std::vector<int64_t> ch((size_t)kStatsCap, 0), rec_ch((size_t)kStatsCap, 0);
    while (!done && it < cap) {
      const int32_t it0 = it;
      const int nb = (int)std::min<int64_t>(chunk, cap - it);
      const int s0 = it0 % kStatsCap, s1 = std::min(kStatsCap, s0 + nb);
      launch_fill_u64((uint64_t *)t.changed + s0, s1 - s0, 0ull, stream);
      if (s0 + nb > kStatsCap) launch_fill_u64((uint64_t *)t.changed, s0 + nb - kStatsCap, 0ull, stream);
      for (int i = 0; i < nb; ++i, ++it) {
        info = grb_mxv(&mnv, nullptr, GRB_ACCUM_MIN, GRB_MIN_SECOND_INT32, A, &gfv, &pd, t.mxv,
                       t.mxv_bytes, stream);
        if (info == GRB_SUCCESS && !A->symmetric)
          info = grb_mxv(&mnv, nullptr, GRB_ACCUM_MIN, GRB_MIN_SECOND_INT32, A, &gfv, &pt, t.mxv,
                         t.mxv_bytes, stream);
        if (info != GRB_SUCCESS) return info;
        launch_cc_step(a, it % kStatsCap, stream);
      }
      if ((info = check_launch()) != GRB_SUCCESS) return info;
      if (!read_back({{ch.data(), t.changed, (size_t)kStatsCap * sizeof(int64_t)}}, s))
        return GRB_PANIC;
      for (int32_t i = it0; i < it; ++i) {
        const int64_t c = ch[(size_t)(i % kStatsCap)];
        if (i < kStatsCap) rec_ch[(size_t)i] = c;
        if (c == 0) {  // no grandparent changed: converged
          it = i + 1;
          done = true;
          break;
        }
      }
      chunk = std::min(chunk * 2, 64);
    }
    launch_cc_out(a, stream);
    if ((info = check_launch()) != GRB_SUCCESS) return info;
    if (hipStreamSynchronize(s) != hipSuccess) return GRB_PANIC;
    std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
    for (int32_t i = 0; i < std::min<int32_t>(it, kStatsCap); ++i) {
      rec[(size_t)i * kStatFields + 0] = rec_ch[(size_t)i];
      rec[(size_t)i * kStatFields + 2] = GRB_DIR_PULL;
    }
    finish_stats(GRB_OP_CC, it, rec, {}, it * (A->symmetric ? 4 : 5), 0.0);
  }
  if (iters) *iters = it;
  return GRB_SUCCESS;
}

grb_info grb_pagerank(void *p, grb_type type, grb_matrix A, double damping, int32_t max_iter,
                      double tol, int32_t *iters, double *delta_out, const grb_descriptor *d,
                      void *ws, size_t ws_bytes, void *stream) {
  return run_pagerank(p, type, A, damping, max_iter, tol, false, 0.0, iters, delta_out, nullptr,
                      d, ws, ws_bytes, stream);
}

grb_info grb_pagerank_adaptive(void *p, grb_type type, grb_matrix A, double damping,
                               int32_t max_iter, double tol, double eps, int32_t *iters,
                               double *delta_out, int64_t *active_out, const grb_descriptor *d,
                               void *ws, size_t ws_bytes, void *stream) {
  if (!(eps >= 0.0) || !std::isfinite(eps)) return GRB_INVALID_VALUE;
  return run_pagerank(p, type, A, damping, max_iter, tol, true, eps, iters, delta_out,
                      active_out, d, ws, ws_bytes, stream);
}

grb_info grb_mxm_masked(void *c, grb_matrix M, grb_matrix A, grb_matrix B, grb_semiring s,
                        const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream) {
  if (!M || !A || !B) return GRB_UNINITIALIZED_OBJECT;
  if (M->nrows != A->nrows || M->ncols != B->nrows || A->ncols != B->ncols)
    return GRB_DIMENSION_MISMATCH;
  int vt = GRB_INT32;
  if (s == GRB_PLUS_TIMES_FP32 || s == GRB_PLUS_TIMES_FP64) {
    vt = s == GRB_PLUS_TIMES_FP32 ? GRB_FP32 : GRB_FP64;
    if (A->a.vtype != vt || B->a.vtype != vt) return GRB_DOMAIN_MISMATCH;
  } else if (s != GRB_PLUS_PAIR_INT32) {
    return (s >= GRB_LOR_LAND_BOOL && s <= GRB_MIN_SECOND_INT32) ? GRB_NOT_IMPLEMENTED
                                                                 : GRB_INVALID_VALUE;
  }
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  if (desc.flags & ~GRB_PROFILE) return GRB_NOT_IMPLEMENTED;
  if (!c && M->nnz > 0) return GRB_NULL_POINTER;
  if ((info = check_ws(ws, ws_bytes, kMxmWs)) != GRB_SUCCESS) return info;
  if (M->nnz == 0 || M->nrows == 0) return GRB_SUCCESS;
  MxmArgs ma;
  ma.nrows = M->nrows;
  ma.M = M->a;
  ma.A = A->a;
  ma.B = B->a;
  ma.c = c;
  ma.vt = vt;
  launch_mxm_dot(ma, false, stream);
  return check_launch();
}

grb_info grb_tricount(int64_t *count, grb_matrix L, const grb_descriptor *d, void *ws,
                      size_t ws_bytes, void *stream) {
  if (!L) return GRB_UNINITIALIZED_OBJECT;
  if (!count) return GRB_NULL_POINTER;
  if (L->nrows != L->ncols) return GRB_DIMENSION_MISMATCH;
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  if (desc.flags & ~GRB_PROFILE) return GRB_NOT_IMPLEMENTED;
  if ((info = check_ws(ws, ws_bytes, kMxmWs)) != GRB_SUCCESS) return info;
  hipStream_t s = (hipStream_t)stream;
  const bool profile = (desc.flags & GRB_PROFILE) != 0;
  unsigned long long *cnt = (unsigned long long *)ws;
  launch_fill_u64((uint64_t *)cnt, 1, 0ull, stream);
  MxmArgs ma;
  ma.nrows = L->nrows;
  ma.M = L->a;
  ma.A = L->a;
  ma.B = L->a;
  ma.count = cnt;
  if (profile) (void)hipEventRecord(g_events.get(0), s);
  if (L->nnz > 0) launch_mxm_dot(ma, true, stream);
  if (profile) (void)hipEventRecord(g_events.get(1), s);
  if ((info = check_launch()) != GRB_SUCCESS) return info;
  unsigned long long h = 0;
  if (!read_back({{&h, cnt, sizeof(h)}}, s)) return GRB_PANIC;
  *count = (int64_t)h;
  std::vector<int64_t> rec((size_t)kStatsCap * kStatFields, 0);
  rec[0] = L->nnz;
  rec[2] = GRB_DIR_PULL;
  std::vector<float> kms;
  double ms_all = 0.0;
  if (profile) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g_events.get(0), g_events.get(1));
    kms.push_back(ms);
    ms_all = ms;
  }
  finish_stats(GRB_OP_MXM, 1, rec, kms, 1, ms_all);
  return GRB_SUCCESS;
}

}  // extern "C"

namespace {

grb_type domain_of(grb_semiring s) {
  switch (s) {
    case GRB_LOR_LAND_BOOL: return GRB_BOOL;
    case GRB_MIN_PLUS_FP32:
    case GRB_PLUS_TIMES_FP32: return GRB_FP32;
    case GRB_MIN_PLUS_FP64:
    case GRB_PLUS_TIMES_FP64: return GRB_FP64;
    default: return GRB_INT32;
  }
}

bool accum_fits(grb_semiring s, grb_binop acc) {
  if (acc == GRB_NOACCUM) return true;
  switch (s) {
    case GRB_LOR_LAND_BOOL: return acc == GRB_ACCUM_LOR;
    case GRB_PLUS_TIMES_FP32:
    case GRB_PLUS_TIMES_FP64: return acc == GRB_ACCUM_PLUS;
    default: return acc == GRB_ACCUM_MIN;
  }
}

// Shared by grb_mxv (is_vxm = false) and grb_vxm (is_vxm = true).
grb_info run_product(bool is_vxm, grb_vector w, grb_vector mask, grb_binop accum, grb_semiring s,
                     grb_matrix A, grb_vector u, const grb_descriptor *d, void *ws,
                     size_t ws_bytes, void *stream) {
  if (!w || !u || !A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  if (s == GRB_PLUS_PAIR_INT32) return GRB_NOT_IMPLEMENTED;  // masked SpGEMM only
  if (s < GRB_LOR_LAND_BOOL || s > GRB_MIN_SECOND_INT32) return GRB_INVALID_VALUE;
  if (accum < GRB_NOACCUM || accum > GRB_ACCUM_LOR) return GRB_INVALID_VALUE;
  grb_descriptor desc;
  grb_info info = resolve_desc(d, &desc);
  if (info != GRB_SUCCESS) return info;
  if (w == u || (mask && w == mask)) return GRB_INVALID_VALUE;  // output must not alias an input
  {
    const void *wp[] = {w->values, w->bitmap, w->indices, w->count};
    const void *ip[] = {u->values, u->bitmap, u->indices, u->count,
                        mask ? mask->values : nullptr, mask ? mask->bitmap : nullptr,
                        mask ? mask->indices : nullptr, mask ? mask->count : nullptr};
    for (const void *x : wp)
      for (const void *y : ip)
        if (x && x == y) return GRB_INVALID_VALUE;
  }
  if (!w->values && w->n > 0) return GRB_INVALID_VALUE;  // the output stores values
  const grb_type dom = domain_of(s);
  if (w->type != dom || u->type != dom) return GRB_DOMAIN_MISMATCH;
  if (!accum_fits(s, accum)) return GRB_DOMAIN_MISMATCH;
  // A' = A or A^T; mxv: w = A' u; vxm: w = u A' = A'^T u
  const bool tran = (desc.flags & GRB_TRAN_A) != 0;
  const bool out_rows_of_a = is_vxm ? tran : !tran;  // output index = row of A?
  const grb::Csr &pull = out_rows_of_a ? A->a : A->at;
  const grb::Csr &push = out_rows_of_a ? A->at : A->a;
  const int64_t n_out = out_rows_of_a ? A->nrows : A->ncols;
  const int64_t n_in = out_rows_of_a ? A->ncols : A->nrows;
  if (w->n != n_out || u->n != n_in || (mask && mask->n != n_out)) return GRB_DIMENSION_MISMATCH;
  const bool can_pull = pull.valid(), can_push = push.valid();
  if ((desc.direction == GRB_DIR_PULL && !can_pull) ||
      (desc.direction == GRB_DIR_PUSH && !can_push) || (!can_pull && !can_push))
    return GRB_NOT_IMPLEMENTED;
  MxvWs t = mxv_layout(ws, n_in, n_out, A->nnz, can_pull ? pull.nsplit : 0);
  if ((info = check_ws(ws, ws_bytes, t.bytes)) != GRB_SUCCESS) return info;
  MxvArgs a;
  a.n_out = n_out;
  a.n_in = n_in;
  a.nw_out = words_of(n_out);
  a.nw_in = words_of(n_in);
  a.nnz = A->nnz;
  a.push = push;
  a.pull = pull;
  a.can_push = can_push;
  a.can_pull = can_pull;
  a.semiring = s;
  a.accum = accum;
  // multiply operand order: mxv A(i,j) (x) u(j), vxm u(i) (x) A(i,j)
  a.pick_vec = (s == GRB_MIN_FIRST_INT32) ? is_vxm : !is_vxm;
  a.has_mask = mask != nullptr;
  a.mask_comp = (desc.flags & GRB_MASK_COMP) != 0;
  a.mask_struct = (desc.flags & GRB_MASK_STRUCT) != 0;
  a.replace = (desc.flags & GRB_REPLACE) != 0;
  // input: a list feeds push directly; pull reads the bitmap, built from the
  // list in the workspace when the vector has none
  a.u_val = u->values;
  if (u->indices) {
    a.u_list = u->indices;
    a.u_cnt = u->count;
  }
  a.u_bm = u->bitmap ? u->bitmap : t.ubm;
  a.u_from_list = u->bitmap == nullptr;
  a.w_val = w->values;
  a.w_bm = w->bitmap ? w->bitmap : t.wbm;
  if (w->indices) {
    a.w_list = w->indices;
    a.w_cnt = w->count;
  }
  if (mask) {
    a.m_val = mask->values;
    a.m_bm = mask->bitmap ? mask->bitmap : t.mbm;
    a.m_type = mask->type;
  }
  a.t_val = t.t_val;
  a.t_bm = t.t_bm;
  a.t_vb = t.t_vb;
  a.hp_val = t.hp_val;
  a.hp_has = t.hp_has;
  a.settled = t.settled;
  a.list = u->indices ? u->indices : t.list;
  a.degpre = t.degpre;
  a.rowstart = t.rowstart;
  a.tiles = t.tiles;
  a.tiles_cap = t.tiles_cap;
  a.status = t.status;
  a.status_out = t.status_out;
  a.status_list = t.status_list;
  a.nblk = t.nblk;
  a.nblk_out = t.nblk_out;
  a.nblk_list = t.nblk_list;
  a.part = t.part;
  a.blk_part = t.blk_part;
  a.ctrl = t.ctrl;
  a.gate.part = t.part;
  a.gate.decided = &t.ctrl->dir;  // the control block is cleared by the first kernel
  a.gate.forced = desc.direction;
  a.gate.can_push = can_push;
  a.gate.can_pull = can_pull;
  a.gate.rule = desc.switch_rule;
  a.gate.denom = desc.switch_denominator;
  a.gate.nnz = A->nnz;
  a.gate.n_in = n_in;
  if (n_out == 0) return GRB_SUCCESS;
  // operands given only as lists: their bitmaps in the workspace
  if (mask && !mask->bitmap) launch_list_to_bitmap(mask->indices, mask->count, n_out, t.mbm, stream);
  if (!w->bitmap) launch_list_to_bitmap(w->indices, w->count, n_out, t.wbm, stream);
  launch_mxv(a, stream);
  if (w->indices) {
    // the output's list follows its new bitmap (bitmap -> sorted list)
    CompactArgs ca;
    ca.nb = a.w_bm;
    ca.nw = a.nw_out;
    ca.nbits = n_out;
    ca.list = w->indices;
    ca.status_cur = t.status_out;
    ca.status_next = t.status_out + t.nblk_out;
    ca.ctrl = t.ctrl;
    ca.count_out = w->count;
    launch_compact(ca, stream);
  }
  return check_launch();
}

}  // namespace

extern "C" {

grb_info grb_mxv(grb_vector w, grb_vector mask, grb_binop accum, grb_semiring s, grb_matrix A,
                 grb_vector u, const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream) {
  return run_product(false, w, mask, accum, s, A, u, d, ws, ws_bytes, stream);
}

grb_info grb_vxm(grb_vector w, grb_vector mask, grb_binop accum, grb_semiring s, grb_vector u,
                 grb_matrix A, const grb_descriptor *d, void *ws, size_t ws_bytes, void *stream) {
  return run_product(true, w, mask, accum, s, A, u, d, ws, ws_bytes, stream);
}

}  // extern "C"
