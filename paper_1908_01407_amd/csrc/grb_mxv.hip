// Generic masked semiring products w<mask> = accum(w, A' u) (Section 3.3 of
// the paper; operand decomposition per its mxv figure), over the closed set
// of semirings of grb.h, in either direction:
// * the first kernel clears the control block and, for the automatic
//   choice, leaves per-workgroup partials of the input's entry count and
//   degree sum; every later kernel evaluates the switch rule (Section 4.3.1,
//   Table 5) from them and returns at once when its direction is not taken,
//   so the input is compacted only when the product really pushes;
// * push (SpMSpV): the input as a sorted list with degree prefix (the
//   compaction kernel for a bitmap input; a list input is used as it is, its
//   prefix built by a look-back scan over the list); merge-path tiles over
//   (entries + edges) scatter products into a temporary t with atomic
//   semiring adds, testing the mask at the scatter; a merge pass applies
//   accum / mask / REPLACE to w;
// * pull (masked SpMV, mask first): each wave sweeps a run of output bitmap
//   words of about equal work (prepared with the matrix); a word without an
//   allowed non-empty row is finished with word operations; otherwise its
//   rows up to kPushSplit long are streamed as one concatenated list, 64
//   positions per step: LOR_LAND pre-checks each row's first two neighbours
//   and stops a row at its first true product, the other semirings find each
//   position's row by bisection so that several steps' loads are in flight,
//   and reduce each row's segments in a fixed order (floating-point results
//   repeat bit for bit).  Rows longer than kPushSplit are cut into pieces
//   that any wave takes; a fix-up kernel (a wave per long row) combines a
//   row's pieces in a fixed order and applies the epilogue.
#include <hip/hip_runtime.h>

#include <climits>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

// ---- semiring traits ---------------------------------------------------------
template <int SR> struct Sr;
template <> struct Sr<GRB_LOR_LAND_BOOL> {
  using T = uint8_t;
  static constexpr bool lor = true;
  __device__ static T identity() { return 0; }
  __device__ static T add(T a, T b) { return (T)(a || b); }
};
template <class V, bool MIN_ADD, bool MUL_PLUS> struct SrArith {
  using T = V;
  static constexpr bool lor = false;
  __device__ static T identity() {
    if (MIN_ADD) return (T)__builtin_huge_val();
    return (T)0;
  }
  __device__ static T add(T a, T b) { return MIN_ADD ? (a < b ? a : b) : a + b; }
  __device__ static T mul(T m, T u, bool) { return MUL_PLUS ? m + u : m * u; }
};
template <> struct Sr<GRB_MIN_PLUS_FP32> : SrArith<float, true, true> {};
template <> struct Sr<GRB_MIN_PLUS_FP64> : SrArith<double, true, true> {};
template <> struct Sr<GRB_PLUS_TIMES_FP32> : SrArith<float, false, false> {};
template <> struct Sr<GRB_PLUS_TIMES_FP64> : SrArith<double, false, false> {};
struct SrMinSel {
  using T = int32_t;
  static constexpr bool lor = false;
  __device__ static T identity() { return INT_MAX; }
  __device__ static T add(T a, T b) { return a < b ? a : b; }
  __device__ static T mul(T m, T u, bool pick_vec) { return pick_vec ? u : m; }
};
template <> struct Sr<GRB_MIN_FIRST_INT32> : SrMinSel {};
template <> struct Sr<GRB_MIN_SECOND_INT32> : SrMinSel {};

template <int SR> struct SrAdd {
  __device__ __forceinline__ typename Sr<SR>::T operator()(typename Sr<SR>::T a,
                                                           typename Sr<SR>::T b) const {
    return Sr<SR>::add(a, b);
  }
};

template <int SR>
__device__ __forceinline__ typename Sr<SR>::T atomic_add_sr(typename Sr<SR>::T *p,
                                                            typename Sr<SR>::T v) {
  if constexpr (SR == GRB_MIN_PLUS_FP32) return atomic_min_f32(p, v);
  else if constexpr (SR == GRB_MIN_PLUS_FP64) return atomic_min_f64(p, v);
  else if constexpr (SR == GRB_PLUS_TIMES_FP32 || SR == GRB_PLUS_TIMES_FP64) return atomicAdd(p, v);
  else return atomicMin(p, v);
}

// matrix entry as the semiring's domain (no values: 1)
template <class T>
__device__ __forceinline__ T mat_value(const Csr &c, int64_t pos) {
  if (!c.val) return (T)1;
  if (c.vtype == GRB_INT32) return (T)((const int32_t *)c.val)[pos];
  if (c.vtype == GRB_FP32) return (T)((const float *)c.val)[pos];
  return (T)((const double *)c.val)[pos];
}
__device__ __forceinline__ bool mat_true(const Csr &c, int64_t pos) {
  if (!c.val) return true;
  if (c.vtype == GRB_INT32) return ((const int32_t *)c.val)[pos] != 0;
  if (c.vtype == GRB_FP32) return ((const float *)c.val)[pos] != 0.0f;
  return ((const double *)c.val)[pos] != 0.0;
}

// input value of index j (a vector without values holds 1 at every entry)
template <class T>
__device__ __forceinline__ T u_at(const MxvArgs &a, int64_t j) {
  return a.u_val ? ((const T *)a.u_val)[j] : (T)1;
}

__device__ __forceinline__ bool mask_allowed(const MxvArgs &a, int64_t i) {
  if (!a.has_mask) return true;
  bool m = bit_of(a.m_bm, i);
  if (m && !a.mask_struct && a.m_val) {
    switch (a.m_type) {
      case GRB_BOOL: m = ((const uint8_t *)a.m_val)[i] != 0; break;
      case GRB_INT32: m = ((const int32_t *)a.m_val)[i] != 0; break;
      case GRB_FP32: m = ((const float *)a.m_val)[i] != 0.0f; break;
      default: m = ((const double *)a.m_val)[i] != 0.0; break;
    }
  }
  return m != a.mask_comp;
}

// the mask as one word operation (no mask, structural mask, or a mask
// without values); `word_mask` says whether that form applies
__device__ __forceinline__ uint64_t allowed_word(const MxvArgs &a, int64_t wd) {
  if (!a.has_mask) return ~0ull;
  const uint64_t m = a.m_bm[wd];
  return a.mask_comp ? ~m : m;
}

__device__ __forceinline__ int mxv_dir(const MxvArgs &a) { return gate_dir(a.gate); }

// z / mask / REPLACE for one output index; returns whether w(i) is present
// afterwards and its value in *out.
template <int SR>
__device__ __forceinline__ bool epilogue(const MxvArgs &a, int64_t i, bool allowed, bool t_has,
                                         typename Sr<SR>::T t, typename Sr<SR>::T *out) {
  using T = typename Sr<SR>::T;
  const T *w = (const T *)a.w_val;
  const bool w_has = bit_of(a.w_bm, i);
  if (!allowed) {
    if (w_has && !a.replace) {
      *out = w[i];
      return true;
    }
    return false;
  }
  if (a.accum == GRB_NOACCUM || !w_has) {
    *out = t;
    return t_has;
  }
  const T old = w[i];
  if (!t_has) {
    *out = old;
    return true;
  }
  if constexpr (Sr<SR>::lor) *out = (T)((old != 0) || (t != 0));
  else if (a.accum == GRB_ACCUM_MIN) *out = old < t ? old : t;
  else *out = old + t;
  return true;
}

// ---- first kernel: control block, direction partials ------------------------
template <int SR>
__global__ __launch_bounds__(kMxvPartThreads) void k_mxv_init(MxvArgs a) {
  __shared__ int64_t s_c[kMxvPartThreads / 64], s_d[kMxvPartThreads / 64];
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + tid;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  if (blockIdx.x == 0) {
    // the control block (a few KB, every field zero when cleared) and the
    // look-back status words of the compactions and the list preparation
    static_assert(sizeof(Ctrl) % 8 == 0, "Ctrl is cleared in 8-byte words");
    for (int k = tid; k < (int)(sizeof(Ctrl) / 8); k += blockDim.x)
      reinterpret_cast<uint64_t *>(a.ctrl)[k] = 0ull;
  }
  for (int64_t i = gt; i < 2 * (int64_t)a.nblk; i += nthr) a.status[i] = 0ull;
  for (int64_t i = gt; i < 2 * (int64_t)a.nblk_out; i += nthr) a.status_out[i] = 0ull;
  for (int64_t i = gt; i < (int64_t)a.nblk_list; i += nthr) a.status_list[i] = 0ull;
  // the OR push's temporary bitmaps (other semirings clear theirs only
  // when they push: their value array is n elements)
  if (Sr<SR>::lor && a.gate.can_push && a.gate.forced != GRB_DIR_PULL)
    for (int64_t i = gt; i < a.nw_out; i += nthr) {
      a.t_bm[i] = 0ull;
      a.t_vb[i] = 0ull;
    }
  // OR pull: long rows' "settled by the probes" flags
  if (Sr<SR>::lor && a.gate.can_pull && a.gate.forced != GRB_DIR_PUSH)
    for (int64_t k = gt; k < a.pull.nsplit_rows; k += nthr) a.settled[a.pull.split_rows[3 * k]] = 0;
  const bool auto_dir = !a.gate.forced && a.gate.can_push && a.gate.can_pull;
  const int32_t *rp = a.push.rp;
  if (a.blk_part && !a.u_list && a.n_in > 0 && a.gate.can_push &&
      a.gate.forced != GRB_DIR_PULL) {
    // every compaction block of the bitmap input (kCompactWords words, the
    // compaction's layout: 16 words per wave): entries and their degree
    // sum, so that the compaction takes its offsets from their prefix; the
    // same sums are the direction partials
    static_assert(kMxvPartThreads == kCompactThreads, "one block per workgroup pass");
    constexpr int WPW = kCompactWords / (kCompactThreads / 64);
    const int64_t wlast = (a.n_in - 1) >> 6;
    const uint64_t mlast = mask_below((int)(a.n_in - wlast * 64));
    int64_t tc = 0, td = 0;  // this workgroup's totals (thread 0)
    for (int64_t b = blockIdx.x; b < a.nblk; b += gridDim.x) {
      int wc = 0, wdg = 0;
#pragma unroll 4
      for (int k = 0; k < WPW; ++k) {
        const int64_t w = b * kCompactWords + wv * WPW + k;
        const uint64_t word = w < a.nw_in ? (a.u_bm[w] & (w == wlast ? mlast : ~0ull)) : 0ull;
        if ((word >> ln) & 1ull) {
          const int64_t v = w * 64 + ln;
          wc += 1;
          wdg += rp[v + 1] - rp[v];
        }
      }
      if (__ballot(wc != 0)) {
        wc = wave_sum(wc);
        wdg = wave_sum(wdg);
      }
      if (ln == 0) {
        s_c[wv] = wc;
        s_d[wv] = wdg;
      }
      __syncthreads();
      if (tid == 0) {
        int64_t bc = 0, bd = 0;
        for (int k = 0; k < kMxvPartThreads / 64; ++k) {
          bc += s_c[k];
          bd += s_d[k];
        }
        a.blk_part[2 * b] = bc;
        a.blk_part[2 * b + 1] = bd;
        tc += bc;
        td += bd;
      }
      __syncthreads();
    }
    if (auto_dir && tid == 0) {
      a.part[2 * blockIdx.x] = tc;
      a.part[2 * blockIdx.x + 1] = td;
    }
    return;
  }
  if (!auto_dir) return;
  // partials of the input's entry count and degree sum (rows of the push CSR)
  const bool exact = a.gate.rule == GRB_SWITCH_EXACT;
  int64_t c = 0, d = 0;
  if (a.u_list) {
    int64_t cnt = *a.u_cnt;
    cnt = cnt < 0 ? 0 : (cnt > a.n_in ? a.n_in : cnt);
    if (gt == 0) c = cnt;
    if (exact)
      for (int64_t k = gt; k < cnt; k += nthr) {
        const int64_t v = a.u_list[k];
        if (v >= 0 && v < a.n_in) d += rp[v + 1] - rp[v];
      }
  } else if (!exact) {
    for (int64_t w = gt; w < a.nw_in; w += nthr) c += __popcll(a.u_bm[w]);
  } else {
    // a wave per word (lane = row), four words in flight
    const int64_t gwv = gt >> 6, nwv = nthr >> 6;
    for (int64_t w0 = gwv; w0 < a.nw_in; w0 += 4 * nwv) {
      uint64_t word[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t w = w0 + q * nwv;
        word[q] = w < a.nw_in ? a.u_bm[w] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t v = (w0 + q * nwv) * 64 + ln;
        if (((word[q] >> ln) & 1ull) && v < a.n_in) {
          c += 1;
          d += rp[v + 1] - rp[v];
        }
      }
    }
  }
  c = wave_sum64(c);
  d = wave_sum64(d);
  if (ln == 0) {
    s_c[wv] = c;
    s_d[wv] = d;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t tc = 0, td = 0;
    for (int k = 0; k < kMxvPartThreads / 64; ++k) {
      tc += s_c[k];
      td += s_d[k];
    }
    a.part[2 * blockIdx.x] = tc;
    a.part[2 * blockIdx.x + 1] = td;
  }
}

// ---- push -------------------------------------------------------------------

// A list input's degree prefix, row starts and merge-path tile starts (what
// the compaction produces for a bitmap input), by a decoupled look-back over
// chunks of kListChunk entries; workgroups are ordered by ticket.
constexpr int kListPer = kMxvListChunk / kCompactThreads;
constexpr int kListChunk = kMxvListChunk;
constexpr uint64_t kStAgg = 1, kStPre = 2;

__global__ __launch_bounds__(kCompactThreads) void k_mxv_list_prep(MxvArgs a) {
  constexpr int NWV = kCompactThreads / 64;
  __shared__ int s_blk;
  __shared__ int64_t s_wsum[NWV];
  __shared__ int64_t s_base;
  if (mxv_dir(a) != GRB_DIR_PUSH) return;
  const int tid = threadIdx.x, wid = tid >> 6, ln = tid & 63;
  int64_t cnt = *a.u_cnt;
  cnt = cnt < 0 ? 0 : (cnt > a.n_in ? a.n_in : cnt);
  // exactly the first ceil(cnt / kListChunk) workgroups take tickets, so the
  // chunks are covered and every workgroup a look-back waits on is running
  if ((int64_t)blockIdx.x * kListChunk >= cnt) return;
  if (tid == 0) s_blk = atomicAdd(&a.ctrl->ticket_list, 1);
  __syncthreads();
  const int blk = s_blk;
  const int64_t k0 = (int64_t)blk * kListChunk;
  const int32_t *rp = a.push.rp;
  int deg[kListPer], rs[kListPer];
  int64_t tsum = 0;
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    const int64_t k = k0 + (int64_t)tid * kListPer + j;
    deg[j] = 0;
    rs[j] = 0;
    if (k < cnt) {
      const int64_t v = a.u_list[k];
      if (v >= 0 && v < a.n_in) {
        rs[j] = rp[v];
        deg[j] = rp[v + 1] - rs[j];
      }
    }
    tsum += deg[j];
  }
  // block scan of the threads' degree sums
  int64_t incl = tsum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(incl, off);
    if (ln >= off) incl += y;
  }
  if (ln == 63) s_wsum[wid] = incl;
  __syncthreads();
  int64_t before = 0, btot = 0;
  for (int k = 0; k < NWV; ++k) {
    if (k < wid) before += s_wsum[k];
    btot += s_wsum[k];
  }
  if (wid == 0) {
    // status word: flag (2 bits) | degree sum (62 bits)
    int64_t ed = 0;
    if (blk > 0) {
      if (ln == 0)
        store_relaxed_u64(&a.status_list[blk], (kStAgg << 62) | (uint64_t)btot);
      for (int jhi = blk - 1;; jhi -= 64) {
        const int j = jhi - ln;
        uint64_t st = kStPre << 62;
        if (j >= 0) {
          do { st = load_relaxed_u64(&a.status_list[j]); } while ((st >> 62) == 0);
        }
        const uint64_t pre = __ballot((st >> 62) == kStPre);
        const int f = pre ? (__ffsll((unsigned long long)pre) - 1) : 64;
        ed += wave_sum64(ln <= f ? (int64_t)(st & ((1ull << 62) - 1)) : 0);
        if (pre) break;
      }
    }
    if (ln == 0) {
      store_relaxed_u64(&a.status_list[blk], (kStPre << 62) | (uint64_t)(ed + btot));
      s_base = ed;
      if (k0 + kListChunk >= cnt) {  // the workgroup holding the list's end
        const int64_t sd = ed + btot;
        const int64_t nt = (cnt + sd + kPushTile - 1) / kPushTile;
        // a list with repeated indices can exceed the tile capacity: then it
        // contributes nothing (its result is undefined, memory stays safe)
        const bool fits = nt < a.tiles_cap && sd <= a.nnz;
        a.ctrl->count = fits ? (int)cnt : 0;
        a.ctrl->sumdeg = fits ? (int)sd : 0;
        a.ctrl->ntiles = fits ? (int)nt : 0;
        if (fits) a.tiles[nt] = (int)(cnt - 1);
      }
    }
  }
  __syncthreads();
  int64_t dex = s_base + before + incl - tsum;
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    const int64_t k = k0 + (int64_t)tid * kListPer + j;
    if (k < cnt) {
      a.degpre[k] = (int)dex;
      a.rowstart[k] = rs[j];
      const int64_t s0 = dex + k, s1 = s0 + deg[j];
      for (int64_t t = (s0 + kPushTile - 1) / kPushTile; t * kPushTile <= s1 && t < a.tiles_cap;
           ++t)
        a.tiles[t] = (int)k;
    }
    dex += deg[j];
  }
}

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_prep(MxvArgs a) {
  using T = typename Sr<SR>::T;
  if (mxv_dir(a) != GRB_DIR_PUSH) return;
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = gw; w < a.nw_out; w += nwaves) {
    if (ln == 0) {
      a.t_bm[w] = 0ull;
      a.t_vb[w] = 0ull;
    }
    const int64_t i = w * 64 + ln;
    if (i < a.n_out) ((T *)a.t_val)[i] = Sr<SR>::identity();
  }
}

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_push(MxvArgs a) {
  using T = typename Sr<SR>::T;
  __shared__ int s_deg[kPushTile + 1], s_rs[kPushTile + 1];
  __shared__ T s_val[kPushTile + 1];
  if (mxv_dir(a) != GRB_DIR_PUSH) return;
  const int ntiles = a.ctrl->ntiles, sumdeg = a.ctrl->sumdeg;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int i0 = a.tiles[t], i1 = a.tiles[t + 1];
    const int ne = i1 - i0 + 1;
    for (int k = threadIdx.x; k < ne; k += kBlock) {
      const int j = a.list[i0 + k];
      s_deg[k] = a.degpre[i0 + k];
      s_rs[k] = a.rowstart[i0 + k];
      s_val[k] = (j >= 0 && j < a.n_in) ? u_at<T>(a, j) : (T)0;
    }
    __syncthreads();
    const int64_t e0 = (int64_t)t * kPushTile - i0;
    int64_t e1 = (int64_t)(t + 1) * kPushTile - i1;
    if (e1 > sumdeg) e1 = sumdeg;
    if constexpr (Sr<SR>::lor) {
      // One OR per run of lanes whose edges hit the same word of the same
      // bitmap (t_vb: a true product, t_bm: a false one; the merge reads
      // presence as either): a long row's sorted targets share words.  The
      // loop is wave-uniform so that the whole wave combines its runs.
      const int ln = threadIdx.x & 63;
      for (int64_t eb = e0 + (threadIdx.x & ~63); eb < e1; eb += kBlock) {
        const int64_t e = eb + ln;
        int lo = 0, hi = ne - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_deg[mid] <= e) lo = mid; else hi = mid - 1;
        }
        int i = -1;
        int64_t pos = 0;
        if (e < e1) {
          pos = s_rs[lo] + (e - s_deg[lo]);
          i = a.push.ci[pos];
          if (!mask_allowed(a, i)) i = -1;
        }
        const bool tru = i >= 0 && s_val[lo] != 0 && mat_true(a.push, pos);
        const int64_t key = i >= 0 ? (((int64_t)(i >> 6) << 1) | (tru ? 1 : 0)) : -1;
        int tail;
        const uint64_t run = run_tail_or(key, i >= 0 ? 1ull << (i & 63) : 0ull, tail);
        if (key >= 0 && run) {
          const int64_t wd = key >> 1;
          if (key & 1) {
            if (~a.t_vb[wd] & run) atomicOr((unsigned long long *)&a.t_vb[wd], run);
          } else {
            if (~a.t_bm[wd] & run) atomicOr((unsigned long long *)&a.t_bm[wd], run);
          }
        }
      }
    } else {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
        int lo = 0, hi = ne - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_deg[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int64_t pos = s_rs[lo] + (e - s_deg[lo]);
        const int i = a.push.ci[pos];
        if (!mask_allowed(a, i)) continue;
        const uint64_t b = 1ull << (i & 63);
        const T prod = Sr<SR>::mul(mat_value<T>(a.push, pos), s_val[lo], a.pick_vec);
        atomic_add_sr<SR>(&((T *)a.t_val)[i], prod);
        if (!(a.t_bm[i >> 6] & b)) atomicOr((unsigned long long *)&a.t_bm[i >> 6], b);
      }
    }
    __syncthreads();
  }
}

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_merge(MxvArgs a) {
  using T = typename Sr<SR>::T;
  if (mxv_dir(a) != GRB_DIR_PUSH) return;
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  T *w = (T *)a.w_val;
  if constexpr (Sr<SR>::lor) {
    if (!a.has_mask || a.mask_struct || !a.m_val) {
      // one output word per lane, 64 words per wave: presence by word
      // operations; a value is written only where the product sets it
      // (kept entries outside the mask and accumulated entries with no
      // product keep their value)
      const bool acc = a.accum != GRB_NOACCUM;
      const int64_t wlast = a.nw_out - 1;
      const uint64_t mlast = mask_below((int)(a.n_out - wlast * 64));
      for (int64_t w0 = gw * 64; w0 < a.nw_out; w0 += nwaves * 64) {
        const int64_t wd = w0 + ln;
        uint64_t wr = 0ull, tvb = 0ull, plain = 0ull;
        if (wd < a.nw_out) {
          const uint64_t valid = wd == wlast ? mlast : ~0ull;
          const uint64_t A = allowed_word(a, wd), W = a.w_bm[wd];
          tvb = a.t_vb[wd];
          const uint64_t th = a.t_bm[wd] | tvb;
          const uint64_t keep = a.replace ? 0ull : (~A & W);
          plain = A & (acc ? ~W : ~0ull);          // w = t where t is present
          const uint64_t accw = acc ? (A & W) : 0ull;  // w = w (+) t, present either way
          a.w_bm[wd] = (keep | (plain & th) | accw) & valid;
          wr = (plain | accw) & th & valid;
        }
        for (uint64_t any = __ballot(wr != 0ull); any; any &= any - 1) {
          const int j = __builtin_ctzll(any);
          const uint64_t wrj = __shfl(wr, j), tvj = __shfl(tvb, j), pj = __shfl(plain, j);
          if ((wrj >> ln) & 1ull) {
            const int64_t i = (w0 + j) * 64 + ln;
            const bool tv = (tvj >> ln) & 1ull;
            w[i] = ((pj >> ln) & 1ull) ? (T)tv : (T)((w[i] != 0) || tv);
          }
        }
      }
      return;
    }
  }
  for (int64_t wd = gw; wd < a.nw_out; wd += nwaves) {
    const int64_t i = wd * 64 + ln;
    bool has = false;
    if (i < a.n_out) {
      bool t_has = bit_of(a.t_bm, i);
      T tv;
      if constexpr (Sr<SR>::lor) {
        tv = (T)bit_of(a.t_vb, i);
        t_has = t_has || tv;
      } else {
        tv = ((const T *)a.t_val)[i];
      }
      T out = tv;
      has = epilogue<SR>(a, i, mask_allowed(a, i), t_has, tv, &out);
      if (has) w[i] = out;
    }
    const uint64_t bits = __ballot(has);
    if (ln == 0) a.w_bm[wd] = bits;
  }
}

// ---- pull -------------------------------------------------------------------

// The 64 rows of output word wd: rows up to kPushSplit long are computed
// here; allowed longer rows are left to the fix-up kernel (their bits of
// the output word are kept).
template <int SR>
__device__ void pull_word(const MxvArgs &a, int64_t wd, int *mark, int *s_end, int *s_base) {
  using T = typename Sr<SR>::T;
  const int ln = threadIdx.x & 63;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  T *w = (T *)a.w_val;
  const int64_t i = wd * 64 + ln;
  const bool inb = i < a.n_out;
  const bool allowed = inb && mask_allowed(a, i);
  int cur = 0, end = 0;
  bool lng = false;
  if (allowed) {
    cur = rp[i];
    end = rp[i + 1];
    lng = end - cur > kPushSplit;
  }
  const bool act = allowed && !lng && end > cur;
  T acc = Sr<SR>::identity();
  bool has = false;
  if constexpr (Sr<SR>::lor) {
    // first two neighbours of every allowed row first (prepared first-two
    // array), so that rows settled by them never stream
    bool q0 = false, q1 = false, p0 = false, p1 = false;
    if (act) {
      const int2 f = a.pull.first2[i];
      q0 = f.x >= 0;
      q1 = f.y >= 0;
      p0 = q0 && bit_of(a.u_bm, f.x);
      p1 = q1 && bit_of(a.u_bm, f.y);
      if (p0 || p1) has = true;
      if ((p0 && u_at<T>(a, f.x) != 0 && mat_true(a.pull, cur)) ||
          (p1 && u_at<T>(a, f.y) != 0 && mat_true(a.pull, cur + 1)))
        acc = 1;
      cur = min(cur + 2, end);
    }
    // the probes' hit rate estimates the frontier's density d; a row then
    // streams about 2/d positions per step (its first frontier entry is
    // expected 1/d in), so a dense frontier does not gather past the first
    const int np = __popcll(__ballot(q0)) + __popcll(__ballot(q1));
    const int nh = __popcll(__ballot(p0)) + __popcll(__ballot(p1));
    const int cmin = nh == 0 ? 64 : min(64, max(4, 2 * np / nh));
    for (;;) {
      int len = (act && acc == 0) ? end - cur : 0;  // OR saturates at true
      if (cmin < 64) {
        const int nl = __popcll(__ballot(len > 0));
        len = min(len, max(cmin, nl ? (64 + nl - 1) / nl : 64));
      }
      const int incl = wave_incl_scan(len);
      const int total = lane_last(incl);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
      const int64_t pos = ln < total ? rcur + (ln - rexcl) : -1;
      const int sev = min(incl, 64);
      if (starts) cur += sev - excl;
      const int j = pos >= 0 ? ci[pos] : -1;
      const bool pres = j >= 0 && bit_of(a.u_bm, j);
      const bool prod = pres && u_at<T>(a, j) != 0 && mat_true(a.pull, pos);
      const uint64_t seg = starts ? (mask_below(sev) & ~mask_below(excl)) : 0ull;
      if (__ballot(pres) & seg) has = true;
      if (__ballot(prod) & seg) acc = 1;
    }
  } else {
    // the word's rows as one list of `total` positions; each position finds
    // its row by bisection of the rows' prefix ends (LDS), so the loads of
    // kUnroll steps are in flight together; each row adds its segment of a
    // step in step order (fixed order)
    const int len = act ? end - cur : 0;
    const int incl = wave_incl_scan(len);
    const int total = lane_last(incl);
    const int excl = incl - len;
    s_end[ln] = incl;
    s_base[ln] = cur - excl;
    wave_lds_sync();
    for (int q0 = 0; q0 < total; q0 += 64 * kUnroll) {
      int row[kUnroll];
      int64_t pos[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int q = q0 + s * 64 + ln;
        row[s] = -1;
        pos[s] = -1;
        if (q < total) {
          int r = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (s_end[r + step - 1] <= q) r += step;
          row[s] = r;
          pos[s] = (int64_t)s_base[r] + q;
        }
      }
      int jv[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) jv[s] = pos[s] >= 0 ? ci[pos[s]] : -1;
      bool pres[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) pres[s] = jv[s] >= 0 && bit_of(a.u_bm, jv[s]);
      T prod[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s)
        prod[s] = pres[s] ? Sr<SR>::mul(mat_value<T>(a.pull, pos[s]), u_at<T>(a, jv[s]), a.pick_vec)
                          : Sr<SR>::identity();
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int sb = q0 + s * 64;
        const T y = wave_seg_scan(prod[s], row[s], Sr<SR>::identity(), SrAdd<SR>());
        const uint64_t pm = __ballot(pres[s]);
        // this lane's row: its part of step s and the lane holding its end
        const int lo = max(excl, sb) - sb, hi = min(incl, sb + 64) - sb;
        const bool mine = len > 0 && lo < hi;
        const T segv = __shfl(y, mine ? hi - 1 : 0);
        if (mine && (pm & mask_below(hi) & ~mask_below(lo))) {
          has = true;
          acc = Sr<SR>::add(acc, segv);
        }
      }
    }
    wave_lds_sync();
  }
  bool out_has = false;
  if (inb && !(allowed && lng)) {
    T out = acc;
    out_has = epilogue<SR>(a, i, allowed, has, acc, &out);
    if (out_has) w[i] = out;
  }
  const uint64_t lmask = __ballot(allowed && lng);
  const uint64_t bits = __ballot(out_has);
  if (ln == 0) a.w_bm[wd] = (bits & ~lmask) | (a.w_bm[wd] & lmask);
}

// OR pull (LOR_LAND) over up to four output words at once: lane l holds row
// l of each word, and the rows' extents, first two entries and their probes
// are loaded together for all the words; a probe settles a row at a true
// product.  The rows left open (more entries, no true product yet) are
// compacted across the words and stream their remaining entries, 64 rows at
// a time, with early exit; a row takes at most about 2/d positions per step
// while enough rows are live (d = the input's density estimated from the
// probes), so a dense input does not gather past a row's first hit.  Then
// each word's epilogue; allowed rows longer than kPushSplit keep their
// output bits for the fix-up kernel.  res: per-wave LDS, [4][64] results.
// The OR stream of the open rows (one per lane: `own`; positions [rc, re)),
// K steps of 64 positions laid out and loaded at once (K > 1 when the
// probes found the input sparse: a row then rarely stops early).
template <int K>
__device__ __forceinline__ void or_stream(const MxvArgs &a, int *mark, int cmin, bool own,
                                          int &rc, int re, bool &has, bool &tru) {
  using T = uint8_t;
  const int ln = threadIdx.x & 63;
  const int32_t *ci = a.pull.ci;
  for (bool more = true; more;) {
    int64_t pos[K];
    int sev[K], exv[K];
    bool st[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      pos[s] = -1;
      sev[s] = exv[s] = 0;
      st[s] = false;
      if (!more) continue;
      int len = (own && !tru) ? re - rc : 0;
      if (cmin < 64) {
        const int nl = __popcll(__ballot(len > 0));
        len = min(len, max(cmin, nl ? (64 + nl - 1) / nl : 64));
      }
      const int incl = wave_incl_scan(len);
      const int total = lane_last(incl);
      if (total == 0) {
        more = false;
        continue;
      }
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(rc, r), rexcl = __shfl(excl, r);
      if (ln < total) pos[s] = rcur + (ln - rexcl);
      sev[s] = min(incl, 64);
      exv[s] = excl;
      st[s] = starts;
      if (starts) rc += sev[s] - excl;
    }
    int jj[K];
#pragma unroll
    for (int s = 0; s < K; ++s) jj[s] = pos[s] >= 0 ? ci[pos[s]] : -1;
    uint64_t bw[K];
#pragma unroll
    for (int s = 0; s < K; ++s) bw[s] = jj[s] >= 0 ? a.u_bm[jj[s] >> 6] : 0ull;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const bool pres = jj[s] >= 0 && ((bw[s] >> (jj[s] & 63)) & 1ull);
      const bool prod = pres && u_at<T>(a, jj[s]) != 0 && mat_true(a.pull, pos[s]);
      const uint64_t seg = st[s] ? (mask_below(sev[s]) & ~mask_below(exv[s])) : 0ull;
      if (__ballot(pres) & seg) has = true;
      if (__ballot(prod) & seg) tru = true;
    }
  }
}

__device__ void pull_or_words(const MxvArgs &a, const int64_t (&wd)[4], int nq, int *mark,
                              uint8_t (*res)[64]) {
  using T = uint8_t;
  const int ln = threadIdx.x & 63;
  const int32_t *rp = a.pull.rp;
  T *w = (T *)a.w_val;
  int64_t ri[4];
  bool inb[4], allowed[4], lng[4], act[4];
  int cur[4], end[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ri[q] = wd[q] * 64 + ln;
    inb[q] = q < nq && ri[q] < a.n_out;
    allowed[q] = inb[q] && mask_allowed(a, ri[q]);
    cur[q] = allowed[q] ? rp[ri[q]] : 0;
    end[q] = allowed[q] ? rp[ri[q] + 1] : 0;
  }
  int2 f[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    lng[q] = end[q] - cur[q] > kPushSplit;
    // long rows take the probes too: a true one settles the row here, and
    // its pieces and fix-up are skipped
    act[q] = allowed[q] && end[q] > cur[q];
    f[q] = act[q] ? a.pull.first2[ri[q]] : make_int2(-1, -1);
  }
  bool settled[4];
  uint64_t b0[4], b1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b0[q] = f[q].x >= 0 ? a.u_bm[f[q].x >> 6] : 0ull;
    b1[q] = f[q].y >= 0 ? a.u_bm[f[q].y >> 6] : 0ull;
  }
  int np = 0, nh = 0;
  uint64_t rest[4];
  int nrest = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool p0 = f[q].x >= 0 && ((b0[q] >> (f[q].x & 63)) & 1ull);
    const bool p1 = f[q].y >= 0 && ((b1[q] >> (f[q].y & 63)) & 1ull);
    const bool tru = (p0 && u_at<T>(a, f[q].x) != 0 && mat_true(a.pull, cur[q])) ||
                     (p1 && u_at<T>(a, f[q].y) != 0 && mat_true(a.pull, cur[q] + 1));
    np += __popcll(__ballot(f[q].x >= 0)) + __popcll(__ballot(f[q].y >= 0));
    nh += __popcll(__ballot(p0)) + __popcll(__ballot(p1));
    res[q][ln] = (uint8_t)((p0 || p1 ? 1 : 0) | (tru ? 2 : 0));
    settled[q] = lng[q] && tru;
    if (allowed[q] && lng[q]) a.settled[ri[q]] = tru ? 1 : 0;
    cur[q] = min(cur[q] + 2, end[q]);
    rest[q] = __ballot(act[q] && !lng[q] && !tru && end[q] > cur[q]);
    nrest += __popcll(rest[q]);
  }
  const int cmin = nh == 0 ? 64 : min(64, max(4, 2 * np / nh));
  for (int sb = 0; sb < nrest; sb += 64) {
    // this lane's row among the open rows: word oq, lane li
    const int j = sb + ln;
    int oq = -1, li = 0, rc = 0, re = 0;
    int before = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cq = __popcll(rest[q]);
      const bool mine = j >= before && j < before + cq;
      const int lq = mine ? nth_set_bit(rest[q], j - before) : 0;
      const int sc = __shfl(cur[q], lq), se = __shfl(end[q], lq);
      if (mine) {
        oq = q;
        li = lq;
        rc = sc;
        re = se;
      }
      before += cq;
    }
    bool has = false, tru = false;
    if (cmin == 64) or_stream<kUnroll>(a, mark, cmin, oq >= 0, rc, re, has, tru);
    else or_stream<1>(a, mark, cmin, oq >= 0, rc, re, has, tru);
    if (oq >= 0) res[oq][li] |= (uint8_t)((has ? 1 : 0) | (tru ? 2 : 0));
  }
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q >= nq) break;
    const uint8_t rv = res[q][ln];
    const bool t_has = (rv & 3) != 0;
    const T acc = (T)((rv >> 1) & 1);
    bool out_has = false;
    const bool deferred = allowed[q] && lng[q] && !settled[q];
    if (inb[q] && !deferred) {
      T out = acc;
      out_has = epilogue<GRB_LOR_LAND_BOOL>(a, ri[q], allowed[q], t_has, acc, &out);
      if (out_has) w[ri[q]] = out;
    }
    const uint64_t lmask = __ballot(deferred);
    const uint64_t bits = __ballot(out_has);
    if (ln == 0) a.w_bm[wd[q]] = (bits & ~lmask) | (a.w_bm[wd[q]] & lmask);
  }
  wave_lds_sync();
}

// OR pieces of long rows, four at a time: the first step of each, then the
// rest of those without a true product in it, all loads of a phase issued
// together.  Writes each piece's result (presence bit 0, true bit 1 as in
// hp_has / the partial value).
__device__ void pull_or_pieces4(const MxvArgs &a, const int64_t (&rk)[4], const int64_t (&bk)[4],
                                const int64_t (&hk)[4], int np) {
  using T = uint8_t;
  const int ln = threadIdx.x & 63;
  const int32_t *ci = a.pull.ci;
  int64_t ek[4];
  bool has[4], tru[4];
  int j0[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ek[k] = k < np ? min(bk[k] + (int64_t)kPushSplit, (int64_t)a.pull.rp[rk[k] + 1]) : 0;
    const int64_t pos = bk[k] + ln;
    j0[k] = (k < np && pos < ek[k]) ? ci[pos] : -1;
  }
  uint64_t bw0[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) bw0[k] = j0[k] >= 0 ? a.u_bm[j0[k] >> 6] : 0ull;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool pres = j0[k] >= 0 && ((bw0[k] >> (j0[k] & 63)) & 1ull);
    has[k] = __ballot(pres) != 0ull;
    tru[k] = __ballot(pres && u_at<T>(a, j0[k]) != 0 && mat_true(a.pull, bk[k] + ln)) != 0ull;
  }
  int jr[4][kUnroll - 1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int s = 1; s < kUnroll; ++s) {
      const int64_t pos = bk[k] + s * 64 + ln;
      jr[k][s - 1] = (k < np && !tru[k] && pos < ek[k]) ? ci[pos] : -1;
    }
  uint64_t bw[4][kUnroll - 1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int s = 0; s < kUnroll - 1; ++s) bw[k][s] = jr[k][s] >= 0 ? a.u_bm[jr[k][s] >> 6] : 0ull;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int s = 0; s < kUnroll - 1; ++s) {
      const int jj = jr[k][s];
      const bool pres = jj >= 0 && ((bw[k][s] >> (jj & 63)) & 1ull);
      if (__ballot(pres)) has[k] = true;
      if (__ballot(pres && u_at<T>(a, jj) != 0 && mat_true(a.pull, bk[k] + (s + 1) * 64 + ln)))
        tru[k] = true;
    }
    if (ln == 0 && k < np) {
      ((T *)a.hp_val)[hk[k]] = tru[k] ? 1 : 0;
      a.hp_has[hk[k]] = has[k] ? 1 : 0;
    }
  }
}

// One piece (positions [b, e), at most kPushSplit = 64 * kUnroll) of a long
// row, reduced by the wave in a fixed order; every lane gets the result.
template <int SR>
__device__ __forceinline__ void pull_piece(const MxvArgs &a, int64_t b, int64_t e,
                                           typename Sr<SR>::T &acc, bool &has) {
  using T = typename Sr<SR>::T;
  const int ln = threadIdx.x & 63;
  const int32_t *ci = a.pull.ci;
  acc = Sr<SR>::identity();
  has = false;
  if constexpr (Sr<SR>::lor) {
    // the first step alone (a dense frontier ends the piece there), then
    // the rest at once
    {
      const int64_t pos = b + ln;
      const int j = pos < e ? ci[pos] : -1;
      const bool pres = j >= 0 && bit_of(a.u_bm, j);
      has = __ballot(pres) != 0ull;
      if (__ballot(pres && u_at<T>(a, j) != 0 && mat_true(a.pull, pos))) {
        acc = 1;
        return;
      }
    }
    int jv[kUnroll - 1];
#pragma unroll
    for (int s = 1; s < kUnroll; ++s) {
      const int64_t pos = b + s * 64 + ln;
      jv[s - 1] = pos < e ? ci[pos] : -1;
    }
    bool pres[kUnroll - 1], tru[kUnroll - 1];
#pragma unroll
    for (int s = 1; s < kUnroll; ++s) {
      const int64_t pos = b + s * 64 + ln;
      pres[s - 1] = jv[s - 1] >= 0 && bit_of(a.u_bm, jv[s - 1]);
      tru[s - 1] = pres[s - 1] && u_at<T>(a, jv[s - 1]) != 0 && mat_true(a.pull, pos);
    }
#pragma unroll
    for (int s = 0; s < kUnroll - 1; ++s) {
      if (__ballot(pres[s])) has = true;
      if (__ballot(tru[s])) acc = 1;
    }
  } else {
    int jv[kUnroll];
#pragma unroll
    for (int s = 0; s < kUnroll; ++s) {
      const int64_t pos = b + s * 64 + ln;
      jv[s] = pos < e ? ci[pos] : -1;
    }
    bool pres[kUnroll];
#pragma unroll
    for (int s = 0; s < kUnroll; ++s) pres[s] = jv[s] >= 0 && bit_of(a.u_bm, jv[s]);
#pragma unroll
    for (int s = 0; s < kUnroll; ++s) {
      const int64_t pos = b + s * 64 + ln;
      const T prod = pres[s] ? Sr<SR>::mul(mat_value<T>(a.pull, pos), u_at<T>(a, jv[s]),
                                           a.pick_vec)
                             : Sr<SR>::identity();
      if (__ballot(pres[s])) has = true;
      acc = Sr<SR>::add(acc, lane_last(wave_scan(prod, Sr<SR>::identity(), SrAdd<SR>())));
    }
  }
}

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_sweep(MxvArgs a) {
  using T = typename Sr<SR>::T;
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int s_end[kWavesPerBlock][64];
  __shared__ int s_base[kWavesPerBlock][64];
  __shared__ uint8_t s_res[kWavesPerBlock][4][64];
  if (mxv_dir(a) != GRB_DIR_PULL) return;
  const int wid = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  // the mask as a word operation: none, structural, or without values
  const bool word_mask = !a.has_mask || a.mask_struct || !a.m_val;
  for (int64_t part = gw; part < kWaveParts; part += nwaves) {
    const int64_t wlo = a.pull.wpart[part], whi = a.pull.wpart[part + 1];
    for (int64_t w0 = wlo; w0 < whi; w0 += 64) {
      // 64 words at once: a word without an allowed row that has entries
      // gets no product, so its output word is a word operation
      const int64_t mw = w0 + ln;
      bool rows = false;
      if (mw < whi) {
        if (word_mask) {
          const uint64_t allow = allowed_word(a, mw);
          if ((allow & ~a.pull.iso[mw]) == 0ull) {
            const uint64_t old = a.w_bm[mw];
            const uint64_t nb = (allow & (a.accum != GRB_NOACCUM ? old : 0ull)) |
                                (~allow & (a.replace ? 0ull : old));
            if (nb != old) a.w_bm[mw] = nb;
          } else {
            rows = true;
          }
        } else {
          rows = true;
        }
      }
      uint64_t todo = __ballot(rows);
      if constexpr (Sr<SR>::lor) {
        while (todo) {
          int64_t wds[4] = {0, 0, 0, 0};
          int nq = 0;
          while (todo && nq < 4) {
            wds[nq++] = w0 + __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
          }
          pull_or_words(a, wds, nq, s_mark[wid], s_res[wid]);
        }
      } else {
        for (; todo; todo &= todo - 1) {
          const int k = __ffsll((unsigned long long)todo) - 1;
          pull_word<SR>(a, w0 + k, s_mark[wid], s_end[wid], s_base[wid]);
        }
      }
    }
  }
  // pieces of the allowed long rows: partial results, combined in piece
  // order by the fix-up kernel; lane l of a wave holds piece hb + l * nwaves
  T *hv = (T *)a.hp_val;
  for (int64_t hb = gw; hb < a.pull.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int64_t r = -1, b = 0;
    if (h < a.pull.nsplit) {
      r = a.pull.split[2 * h];
      b = a.pull.split[2 * h + 1];
      if (!mask_allowed(a, r)) r = -1;
      // an OR row its probes settled needs no pieces (the flag may not be
      // set yet when the piece comes first: the work is then only redundant)
      else if (Sr<SR>::lor && a.settled[r]) r = -1;
    }
    uint64_t todo = __ballot(r >= 0);
    if constexpr (Sr<SR>::lor) {
      while (todo) {
        int64_t rk[4] = {0, 0, 0, 0}, bk[4] = {0, 0, 0, 0}, hk[4] = {0, 0, 0, 0};
        int np = 0;
        while (todo && np < 4) {
          const int k = __ffsll((unsigned long long)todo) - 1;
          todo &= todo - 1;
          rk[np] = __shfl(r, k);
          bk[np] = __shfl(b, k);
          hk[np] = hb + (int64_t)k * nwaves;
          ++np;
        }
        pull_or_pieces4(a, rk, bk, hk, np);
      }
    } else {
      for (; todo; todo &= todo - 1) {
        const int k = __ffsll((unsigned long long)todo) - 1;
        const int64_t rk = __shfl(r, k), bk = __shfl(b, k);
        const int64_t ek = min(bk + (int64_t)kPushSplit, (int64_t)a.pull.rp[rk + 1]);
        T acc;
        bool has;
        pull_piece<SR>(a, bk, ek, acc, has);
        if (ln == 0) {
          const int64_t hk = hb + (int64_t)k * nwaves;
          hv[hk] = acc;
          a.hp_has[hk] = has ? 1 : 0;
        }
      }
    }
  }
}

// Epilogue of long row r from its combined pieces, output bit by atomic
// (other rows of the word are written by other lanes and waves).
template <int SR>
__device__ __forceinline__ void long_row_out(const MxvArgs &a, int64_t r, bool has,
                                             typename Sr<SR>::T acc) {
  using T = typename Sr<SR>::T;
  T out = acc;
  const bool out_has = epilogue<SR>(a, r, true, has, acc, &out);
  const unsigned long long bit = 1ull << (r & 63);
  if (out_has) {
    ((T *)a.w_val)[r] = out;
    atomicOr((unsigned long long *)&a.w_bm[r >> 6], bit);
  } else {
    atomicAnd((unsigned long long *)&a.w_bm[r >> 6], ~bit);
  }
}

// The allowed long rows not settled by their probes, in two phases.
// First each wave takes 64 consecutive rows (ascending), a lane per row,
// and combines the pieces of rows with at most kFixLanePieces in order, the
// loads of eight pieces issued together; the rows of one bitmap word then
// sit in consecutive lanes, and a segmented OR over the lanes gathers each
// word's set and cleared bits in its last lane, which writes the word with
// one read-modify-write (atomics for the first and last word of the step,
// which neighbouring steps may share, and for words holding a row of the
// second phase).  Then the rows with more pieces, which cluster at the hub
// ids, are dealt to the waves with a stride (lane l of wave w: row
// w + l * waves), each combined by the whole wave (lane l: pieces l,
// l + 64, ..., then the lanes in a fixed order).  One fixed order per row.
constexpr int kFixLanePieces = 32;

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_fixup(MxvArgs a) {
  using T = typename Sr<SR>::T;
  if (mxv_dir(a) != GRB_DIR_PULL) return;
  const T *hv = (const T *)a.hp_val;
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t nrows = a.pull.nsplit_rows;
  for (int64_t k0 = gw * 64; k0 < nrows; k0 += nwaves * 64) {
    const int64_t k = k0 + ln;
    int r = -1, first = 0, cnt = 0;
    bool todo = false;
    if (k < nrows) {
      r = a.pull.split_rows[3 * k];
      first = a.pull.split_rows[3 * k + 1];
      cnt = a.pull.split_rows[3 * k + 2];
      // rows outside the mask were written by the sweep, and so were the OR
      // rows their probes settled
      todo = mask_allowed(a, r) && !(Sr<SR>::lor && a.settled[r]);
    }
    const bool big = todo && cnt > kFixLanePieces;
    unsigned long long set = 0, clr = 0;
    int wide = big ? 1 : 0;
    if (todo && !big) {
      T acc = Sr<SR>::identity();
      bool has = false;
      for (int p0 = 0; p0 < cnt; p0 += 8) {
        uint8_t hh[8];
        T vv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool ok = p0 + q < cnt;
          hh[q] = ok ? a.hp_has[first + p0 + q] : (uint8_t)0;
          vv[q] = ok ? hv[first + p0 + q] : Sr<SR>::identity();
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (hh[q]) {
            has = true;
            acc = Sr<SR>::add(acc, vv[q]);
          }
      }
      T out = acc;
      const bool out_has = epilogue<SR>(a, r, true, has, acc, &out);
      const unsigned long long bit = 1ull << (r & 63);
      if (out_has) {
        ((T *)a.w_val)[r] = out;
        set = bit;
      } else {
        clr = bit;
      }
    }
    // segmented inclusive OR over lanes of the same word (rows ascend)
    const int word = r >= 0 ? (r >> 6) : -1;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int wu = __shfl_up(word, d);
      const unsigned long long su = __shfl_up(set, d), cu = __shfl_up(clr, d);
      const int bu = __shfl_up(wide, d);
      if (ln >= d && wu == word) {
        set |= su;
        clr |= cu;
        wide |= bu;
      }
    }
    const int wd = __shfl_down(word, 1);
    const int w_first = __shfl(word, 0), w_last = __shfl(word, 63);
    const bool seg_end = ln == 63 || wd != word;
    if (word >= 0 && seg_end && (set | clr)) {
      unsigned long long *wp = (unsigned long long *)&a.w_bm[word];
      const bool shared = word == w_first || word == w_last || k0 + 64 >= nrows || wide;
      if (shared) {
        if (set) atomicOr(wp, set);
        if (clr) atomicAnd(wp, ~clr);
      } else {
        *wp = (*wp | set) & ~clr;
      }
    }
  }
  for (int64_t hb = gw; hb < nrows; hb += 64 * nwaves) {
    const int64_t k = hb + (int64_t)ln * nwaves;
    int r = -1, first = 0, cnt = 0;
    if (k < nrows) {
      r = a.pull.split_rows[3 * k];
      first = a.pull.split_rows[3 * k + 1];
      cnt = a.pull.split_rows[3 * k + 2];
    }
    const bool big = r >= 0 && cnt > kFixLanePieces && mask_allowed(a, r) &&
                     !(Sr<SR>::lor && a.settled[r]);
    for (uint64_t bm = __ballot(big); bm; bm &= bm - 1) {
      const int kk = __ffsll((unsigned long long)bm) - 1;
      const int rr = __shfl(r, kk), ff = __shfl(first, kk), cc = __shfl(cnt, kk);
      T acc = Sr<SR>::identity();
      bool has = false;
      for (int p = ln; p < cc; p += 64) {
        if (!a.hp_has[ff + p]) continue;
        has = true;
        acc = Sr<SR>::add(acc, hv[ff + p]);
      }
      has = __ballot(has) != 0ull;
      acc = lane_last(wave_scan(acc, Sr<SR>::identity(), SrAdd<SR>()));
      if (ln == 0) long_row_out<SR>(a, rr, has, acc);
    }
  }
}

template <int SR>
void run_mxv(const MxvArgs &a, hipStream_t s) {
  const int gw_out = (int)std::max<int64_t>(
      1, std::min<int64_t>((a.nw_out + kWavesPerBlock - 1) / kWavesPerBlock, 1 << 16));
  hipLaunchKernelGGL(k_mxv_init<SR>, dim3(kMxvParts), dim3(kMxvPartThreads), 0, s, a);
  const bool want_push = a.gate.can_push && a.gate.forced != GRB_DIR_PULL;
  const bool want_pull = a.gate.can_pull && a.gate.forced != GRB_DIR_PUSH;
  if (want_push) {
    if (a.u_list) {
      const int g = (int)std::max<int64_t>(1, (a.n_in + kListChunk - 1) / kListChunk);
      hipLaunchKernelGGL(k_mxv_list_prep, dim3(g), dim3(kCompactThreads), 0, s, a);
    } else {
      CompactArgs ca;
      ca.nb = a.u_bm;
      ca.nw = a.nw_in;
      ca.nbits = a.n_in;
      ca.rp = a.push.rp;
      ca.list = a.list;
      ca.degpre = a.degpre;
      ca.rowstart = a.rowstart;
      ca.tiles = a.tiles;
      ca.status_cur = a.status;
      ca.status_next = a.status + a.nblk;
      ca.ctrl = a.ctrl;
      ca.gated = true;
      ca.gate = a.gate;
      ca.blk_part = a.n_in > 0 ? a.blk_part : nullptr;  // left by the first kernel
      launch_compact(ca, s);
    }
    if (!Sr<SR>::lor) hipLaunchKernelGGL(k_mxv_prep<SR>, dim3(gw_out), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_mxv_push<SR>, dim3(kExpandGrid), dim3(kBlock), 0, s, a);
    // the OR semiring's word form takes 64 output words per wave
    const bool word_merge = Sr<SR>::lor && (!a.has_mask || a.mask_struct || !a.m_val);
    const int gm = word_merge ? (int)std::max<int64_t>(
                                    1, (a.nw_out + 64 * kWavesPerBlock - 1) / (64 * kWavesPerBlock))
                              : gw_out;
    hipLaunchKernelGGL(k_mxv_merge<SR>, dim3(std::min(gm, 1 << 16)), dim3(kBlock), 0, s, a);
  }
  if (want_pull) {
    if (a.u_from_list)
      launch_list_to_bitmap(a.u_list, a.u_cnt, a.n_in, const_cast<uint64_t *>(a.u_bm), s, &a.gate);
    hipLaunchKernelGGL(k_mxv_sweep<SR>, dim3(kSweepGrid), dim3(kBlock), 0, s, a);
    if (a.pull.nsplit_rows > 0) {
      const int gf = (int)std::min<int64_t>((a.pull.nsplit_rows + kBlock - 1) / kBlock, kExpandGrid);
      hipLaunchKernelGGL(k_mxv_fixup<SR>, dim3(gf), dim3(kBlock), 0, s, a);
    }
  }
}

}  // namespace

void launch_mxv(const MxvArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (a.semiring) {
    case GRB_LOR_LAND_BOOL: run_mxv<GRB_LOR_LAND_BOOL>(a, s); break;
    case GRB_MIN_PLUS_FP32: run_mxv<GRB_MIN_PLUS_FP32>(a, s); break;
    case GRB_MIN_PLUS_FP64: run_mxv<GRB_MIN_PLUS_FP64>(a, s); break;
    case GRB_PLUS_TIMES_FP32: run_mxv<GRB_PLUS_TIMES_FP32>(a, s); break;
    case GRB_PLUS_TIMES_FP64: run_mxv<GRB_PLUS_TIMES_FP64>(a, s); break;
    case GRB_MIN_FIRST_INT32: run_mxv<GRB_MIN_FIRST_INT32>(a, s); break;
    default: run_mxv<GRB_MIN_SECOND_INT32>(a, s); break;
  }
}

}  // namespace grb
