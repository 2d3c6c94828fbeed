// Generic masked semiring products w<mask> = accum(w, A' u) (Section 3.3 of
// the paper; operand decomposition per its mxv figure), over the closed set
// of semirings of grb.h, in either direction:
// * push (SpMSpV): u's presence bitmap is compacted into a sorted list with
//   degree prefix (the traversal compaction kernel); merge-path tiles over
//   (entries + edges) scatter products into a temporary t with atomic
//   semiring adds, testing the mask at the scatter; a merge pass applies
//   accum / mask / REPLACE to w;
// * pull (masked SpMV, mask first): each wave owns one output bitmap word;
//   the allowed rows' adjacency is streamed as one concatenated list, 64
//   entries per step, reduced per row with a segmented scan (fixed order,
//   so floating-point results repeat bit for bit); LOR_LAND stops a row at
//   its first true product; rows longer than kHeavyDeg are cut into pieces
//   whose partial results a fix-up kernel (a wave per long row) combines in
//   a fixed order.
// The direction is chosen on the device (forced, or the descriptor's rule
// on the input's size and degree sum), every kernel of the path not taken
// returns at once.
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

__device__ __forceinline__ bool mask_allowed(const MxvArgs &a, int64_t i) {
  if (!a.has_mask) return true;
  bool m = bit_of(a.m_bm, i);
  if (m && !a.mask_struct) {
    switch (a.m_type) {
      case GRB_BOOL: m = ((const uint8_t *)a.m_val)[i] != 0; break;
      case GRB_INT32: m = ((const int32_t *)a.m_val)[i] != 0; break;
      case GRB_FP32: m = ((const float *)a.m_val)[i] != 0.0f; break;
      default: m = ((const double *)a.m_val)[i] != 0.0; break;
    }
  }
  return m != a.mask_comp;
}

__device__ __forceinline__ int mxv_dir(const MxvArgs &a) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  if (!a.can_push) return GRB_DIR_PULL;
  const int count = a.ctrl->count, sumdeg = a.ctrl->sumdeg;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n_in;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

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

__global__ void k_mxv_init(MxvArgs a) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = gt; i < 2 * (int64_t)a.nblk; i += (int64_t)gridDim.x * blockDim.x)
    a.status[i] = 0ull;
  // the control block (a few KB) cleared by the first workgroup's threads
  // together, 8 bytes each (all its fields are zero when cleared)
  static_assert(sizeof(Ctrl) % 8 == 0, "Ctrl is cleared in 8-byte words");
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < (int)(sizeof(Ctrl) / 8); k += blockDim.x)
      reinterpret_cast<uint64_t *>(a.ctrl)[k] = 0ull;
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
    if constexpr (!Sr<SR>::lor) {
      const int64_t i = w * 64 + ln;
      if (i < a.n_out) ((T *)a.t_val)[i] = Sr<SR>::identity();
    }
  }
}

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_push(MxvArgs a) {
  using T = typename Sr<SR>::T;
  __shared__ int s_deg[kPushTile + 1], s_rs[kPushTile + 1];
  __shared__ T s_val[kPushTile + 1];
  if (mxv_dir(a) != GRB_DIR_PUSH) return;
  const int ntiles = a.ctrl->ntiles, sumdeg = a.ctrl->sumdeg;
  const T *uv = (const T *)a.u_val;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int i0 = a.tiles[t], i1 = a.tiles[t + 1];
    const int ne = i1 - i0 + 1;
    for (int k = threadIdx.x; k < ne; k += kBlock) {
      const int j = a.list[i0 + k];
      s_deg[k] = a.degpre[i0 + k];
      s_rs[k] = a.rowstart[i0 + k];
      s_val[k] = uv[j];
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

template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_pull(MxvArgs a) {
  using T = typename Sr<SR>::T;
  __shared__ int s_mark[kWavesPerBlock][64];
  if (mxv_dir(a) != GRB_DIR_PULL) return;
  int *mark = s_mark[threadIdx.x >> 6];
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const T *uv = (const T *)a.u_val;
  T *w = (T *)a.w_val;
  for (int64_t wd = gw; wd < a.nw_out; wd += nwaves) {
    const int64_t i = wd * 64 + ln;
    const bool inb = i < a.n_out;
    const bool allowed = inb && mask_allowed(a, i);
    int cur = 0, end = 0;
    bool heavy = false;
    if (allowed) {
      cur = rp[i];
      end = rp[i + 1];
      heavy = end - cur > kHeavyDeg;
    }
    const bool act = allowed && !heavy;
    T acc;
    if constexpr (Sr<SR>::lor) acc = 0;
    else acc = Sr<SR>::identity();
    bool has = false;
    int cmin = 1 << 30;  // positions a row takes per step when rows are many
    if constexpr (Sr<SR>::lor) {
      // OR: the first two neighbours of every allowed row first (one row
      // per lane, from the prepared first-two array), so that rows settled
      // by them never stream; the stream below starts after them
      bool q0 = false, q1 = false, p0 = false, p1 = false;
      if (act) {
        const int2 f = a.pull.first2[i];
        q0 = f.x >= 0;
        q1 = f.y >= 0;
        p0 = q0 && bit_of(a.u_bm, f.x);
        p1 = q1 && bit_of(a.u_bm, f.y);
        if (p0 || p1) has = true;
        if ((p0 && uv[f.x] != 0 && mat_true(a.pull, cur)) ||
            (p1 && uv[f.y] != 0 && mat_true(a.pull, cur + 1)))
          acc = 1;
        cur = min(cur + 2, end);
      }
      // the probes' hit rate estimates the frontier's density d; a row
      // then streams about 2/d positions per step (its first frontier
      // entry is expected 1/d in), so that a dense frontier does not
      // gather the entries past the first
      const int np = __popcll(__ballot(q0)) + __popcll(__ballot(q1));
      const int nh = __popcll(__ballot(p0)) + __popcll(__ballot(p1));
      cmin = nh == 0 ? 64 : min(64, max(4, 2 * np / nh));
    }
    // kU steps of 64 stream positions are laid out first, then all their
    // loads issue together; products are reduced step by step in order.
    // OR takes one step at a time: a row stops at its first true product,
    // and larger batches would scan past it
    constexpr int kU = Sr<SR>::lor ? 1 : kUnroll;
    for (bool more = true; more;) {
      bool live = act;
      if constexpr (Sr<SR>::lor) live = live && acc == 0;  // OR saturates at true
      int64_t pos[kU];
      int row[kU], sev[kU], exv[kU];
      bool st[kU];
#pragma unroll
      for (int s = 0; s < kU; ++s) {
        pos[s] = -1;
        row[s] = 0;
        sev[s] = 0;
        exv[s] = 0;
        st[s] = false;
        if (!more) continue;
        int len = live ? end - cur : 0;
        if (Sr<SR>::lor && cmin < 64) {  // (a step holds 64 positions anyway)
          // at least a full step between the live rows
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
        const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
        if (ln < total) pos[s] = rcur + (ln - rexcl);
        row[s] = r;
        st[s] = starts;
        sev[s] = min(incl, 64);
        exv[s] = excl;
        if (starts) cur += sev[s] - excl;
      }
      int jv[kU];
#pragma unroll
      for (int s = 0; s < kU; ++s) jv[s] = pos[s] >= 0 ? ci[pos[s]] : -1;
      bool pres[kU];
#pragma unroll
      for (int s = 0; s < kU; ++s) pres[s] = jv[s] >= 0 && bit_of(a.u_bm, jv[s]);
      T prod[kU];
#pragma unroll
      for (int s = 0; s < kU; ++s) {
        if constexpr (Sr<SR>::lor) {
          prod[s] = pres[s] ? (T)(uv[jv[s]] != 0 && mat_true(a.pull, pos[s])) : (T)0;
        } else {
          prod[s] = pres[s] ? Sr<SR>::mul(mat_value<T>(a.pull, pos[s]), uv[jv[s]], a.pick_vec)
                            : Sr<SR>::identity();
        }
      }
#pragma unroll
      for (int s = 0; s < kU; ++s) {
        const uint64_t seg = st[s] ? (mask_below(sev[s]) & ~mask_below(exv[s])) : 0ull;
        const uint64_t pm = __ballot(pres[s]);
        if constexpr (Sr<SR>::lor) {
          const uint64_t tm = __ballot(prod[s] != 0);
          if (pm & seg) has = true;
          if (tm & seg) acc = 1;
        } else {
          const T x = wave_seg_scan(prod[s], row[s], Sr<SR>::identity(), SrAdd<SR>());
          const T segv = __shfl(x, st[s] ? sev[s] - 1 : 0);
          if (pm & seg) {
            has = true;
            acc = Sr<SR>::add(acc, segv);
          }
        }
      }
    }
    bool out_has = false;
    if (inb && !heavy) {
      T out = acc;
      out_has = epilogue<SR>(a, i, allowed, has, acc, &out);
      if (out_has) w[i] = out;
    }
    const uint64_t hmask = __ballot(heavy);
    const uint64_t bits = __ballot(out_has);
    if (ln == 0) a.w_bm[wd] = (bits & ~hmask) | (a.w_bm[wd] & hmask);
  }
  // pieces of long rows: partial results, combined in piece order later
  T *hv = (T *)a.hp_val;
  for (int64_t h = gw; h < a.pull.nheavy; h += nwaves) {
    const int r = a.pull.heavy[2 * h], b = a.pull.heavy[2 * h + 1];
    bool pres_any = false;
    T acc;
    if constexpr (Sr<SR>::lor) acc = 0;
    else acc = Sr<SR>::identity();
    if (mask_allowed(a, r)) {
      const int e = min(b + kHeavyChunk, rp[r + 1]);
      bool done = false;
      for (int base = b; base < e && !done; base += 64 * kUnroll) {
        int jv[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          const int64_t pos = base + s * 64 + ln;
          jv[s] = pos < e ? ci[pos] : -1;
        }
        bool pres[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) pres[s] = jv[s] >= 0 && bit_of(a.u_bm, jv[s]);
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          const int64_t pos = base + s * 64 + ln;
          T prod;
          if constexpr (Sr<SR>::lor) {
            prod = pres[s] ? (T)(uv[jv[s]] != 0 && mat_true(a.pull, pos)) : (T)0;
          } else {
            prod = pres[s] ? Sr<SR>::mul(mat_value<T>(a.pull, pos), uv[jv[s]], a.pick_vec)
                           : Sr<SR>::identity();
          }
          if (__ballot(pres[s])) pres_any = true;
          if constexpr (Sr<SR>::lor) {
            if (!done && __ballot(prod != 0)) {
              acc = 1;
              done = true;
            }
          } else {
            T x = prod;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x = Sr<SR>::add(x, __shfl_xor(x, off));
            acc = Sr<SR>::add(acc, x);
          }
        }
      }
    }
    if (ln == 0) {
      hv[h] = acc;
      a.hp_has[h] = pres_any ? 1 : 0;
    }
  }
}

// One wave per long row: lane l combines the pieces l, l + 64, ... in order,
// then the lanes' results are combined in a fixed order.
template <int SR>
__global__ __launch_bounds__(kBlock) void k_mxv_pull_fixup(MxvArgs a) {
  using T = typename Sr<SR>::T;
  if (mxv_dir(a) != GRB_DIR_PULL) return;
  const T *hv = (const T *)a.hp_val;
  T *w = (T *)a.w_val;
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t k = gw; k < a.pull.nheavy_rows; k += nwaves) {
    const int r = a.pull.heavy_rows[3 * k], first = a.pull.heavy_rows[3 * k + 1],
              cnt = a.pull.heavy_rows[3 * k + 2];
    T acc;
    if constexpr (Sr<SR>::lor) acc = 0;
    else acc = Sr<SR>::identity();
    bool has = false;
    for (int p = ln; p < cnt; p += 64) {
      if (!a.hp_has[first + p]) continue;
      has = true;
      if constexpr (Sr<SR>::lor) acc = (T)(acc || hv[first + p]);
      else acc = Sr<SR>::add(acc, hv[first + p]);
    }
    has = __ballot(has) != 0ull;
    if constexpr (Sr<SR>::lor) {
      acc = (T)(__ballot(acc != 0) != 0ull);
    } else {
      acc = lane_last(wave_scan(acc, Sr<SR>::identity(), SrAdd<SR>()));
    }
    if (ln == 0) {
      const bool allowed = mask_allowed(a, r);
      T out = acc;
      const bool out_has = epilogue<SR>(a, r, allowed, has, acc, &out);
      const unsigned long long bit = 1ull << (r & 63);
      if (out_has) {
        w[r] = out;
        atomicOr((unsigned long long *)&a.w_bm[r >> 6], bit);
      } else {
        atomicAnd((unsigned long long *)&a.w_bm[r >> 6], ~bit);
      }
    }
  }
}

template <int SR>
void run_mxv(const MxvArgs &a, hipStream_t s) {
  // per-word kernels: one output word per wave (each word is a dependent
  // chain of loads, so the words run side by side)
  const int gw_out = (int)std::max<int64_t>(
      1, std::min<int64_t>((a.nw_out + kWavesPerBlock - 1) / kWavesPerBlock, 1 << 16));
  hipLaunchKernelGGL(k_mxv_init, dim3(64), dim3(256), 0, s, a);
  const bool want_push = a.can_push && a.forced != GRB_DIR_PULL;
  const bool want_pull = a.can_pull && a.forced != GRB_DIR_PUSH;
  if (want_push) {
    CompactArgs ca;
    ca.nb = a.u_bm;
    ca.nw = a.nw_in;
    ca.rp = a.push.rp;
    ca.list = a.list;
    ca.degpre = a.degpre;
    ca.rowstart = a.rowstart;
    ca.tiles = a.tiles;
    ca.status_cur = a.status;
    ca.status_next = a.status + a.nblk;
    ca.ctrl = a.ctrl;
    launch_compact(ca, s);
    hipLaunchKernelGGL(k_mxv_prep<SR>, dim3(gw_out), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_mxv_push<SR>, dim3(kExpandGrid), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_mxv_merge<SR>, dim3(gw_out), dim3(kBlock), 0, s, a);
  }
  if (want_pull) {
    hipLaunchKernelGGL(k_mxv_pull<SR>, dim3(gw_out), dim3(kBlock), 0, s, a);
    if (a.pull.nheavy_rows > 0) {
      const int gf = (int)std::min<int64_t>(
          (a.pull.nheavy_rows + kWavesPerBlock - 1) / kWavesPerBlock, kExpandGrid);
      hipLaunchKernelGGL(k_mxv_pull_fixup<SR>, dim3(gf), dim3(kBlock), 0, s, a);
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
