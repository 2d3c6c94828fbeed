// PageRank iteration kernels (Section 7.3 of the paper: pull form, SpMV
// every iteration because the vector never gets sparse), and the adaptive
// form (PageRankDelta, named in Sections 5.1 and 7.3): the mask holds the
// vertices that have converged, whose values stay frozen, so only the rows
// of the others are computed and the work of an iteration is the in-edges
// of its active rows.
//
// Load balance: each wave takes a run of bitmap words of rows (64
// consecutive rows of the CSR of A^T each), runs of about equal work built
// by grb_matrix_prepare, one word at a time, and streams the word's
// in-edges as one concatenated list, 64 positions per step: the rows'
// prefix ends sit in LDS, each lane finds the row of its position by
// bisection (so the steps are independent and kSweepUnroll of them have
// their loads in flight together), and a segmented sum per step adds each row's
// segment to the row's LDS accumulator, in step order;
// rows longer than kPushSplit are cut into fixed pieces that any wave
// takes, and a second kernel (one wave per long row) adds each long
// row's pieces in a fixed order.  Summation order is fixed, so fp32 and fp64 results are bitwise
// reproducible run to run.  The dangling mass and the L1 change are reduced
// per workgroup and then in a fixed order in the fix-up kernel, which also
// decides convergence on the device.
//
// Adaptive: three rotating activity bitmaps (this iteration, the previous
// one, the next one).  A wave owns the words of its run, so it writes each
// word of the next bitmap with one store (long rows stay set there and
// their kernel clears the bit of a row that freezes).  A vertex frozen in
// the previous iteration copies its x into the other buffer once; from
// then on both buffers hold it.  The dangling mass of frozen vertices is
// kept as a running sum on the device.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

template <class T>
__device__ __forceinline__ T rank_update(const PrArgs &a, T t, T dn) {
  const T alpha = (T)a.alpha;
  const T base = (T)((1.0 - a.alpha) / (double)a.n);
  return base + alpha * (t + dn);
}

// Sums each of the kPrFields partials over the workgroup (fixed order);
// thread 0 writes them to out[kPrFields * blockIdx.x + f].
__device__ __forceinline__ void block_partials(double (&v)[kPrFields], double *out) {
  __shared__ double s_red[kWavesPerBlock][kPrFields];
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < kPrFields; ++f) {
    v[f] = wave_sum_f64(v[f]);
    if ((threadIdx.x & 63) == 0) s_red[wid][f] = v[f];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int f = 0; f < kPrFields; ++f) {
      double t = 0;
      for (int i = 0; i < kWavesPerBlock; ++i) t += s_red[i][f];
      out[kPrFields * blockIdx.x + f] = t;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_pr_init(PrArgs a) {
  T *p = (T *)a.p;
  T *xn = (T *)a.xn;
  const T p0 = (T)(1.0 / (double)a.n);
  double dang = 0;
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * kBlock;
  for (int64_t v = tid; v < a.n; v += nt) {
    p[v] = p0;
    const int od = a.out_rp[v + 1] - a.out_rp[v];
    if (od == 0) {
      xn[v] = (T)0;
      dang += (double)p0;
    } else {
      xn[v] = p0 / (T)od;
    }
  }
  // adaptive: every vertex is active in the first iteration and counts as
  // active in the one before it (so nothing is carried over)
  if (a.act_cur) {
    for (int64_t w = tid; w < a.nw; w += nt) {
      const int64_t valid = a.n - w * 64;
      const uint64_t m = valid >= 64 ? ~0ull : mask_below((int)valid);
      a.act_cur[w] = m;
      a.act_prev[w] = m;
    }
  }
  double v[kPrFields] = {0.0, dang, 0.0, 0.0, 0.0, 0.0};
  block_partials(v, a.blk_part);
}

template <class T, bool AD>
__global__ __launch_bounds__(kBlock) void k_pr_iter(PrArgs a) {
  __shared__ int s_end[kWavesPerBlock][64];
  __shared__ int s_base[kWavesPerBlock][64];
  __shared__ T s_acc[kWavesPerBlock][64];
  if (a.ctrl->converged) return;
  const int wid = threadIdx.x >> 6;
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const T *x = (const T *)a.x;
  T *xn = (T *)a.xn;
  T *p = (T *)a.p;
  const T dn = (T)(a.ctrl->D / (double)a.n);
  double delta = 0, dang = 0, dfz = 0, after = 0, upd = 0, edges = 0;
  // rows up to kPushSplit long: the wave's run of words (about equal work
  // per run), one word of rows at a time
  for (int64_t part = gw; part < kWaveParts; part += nwaves) {
    const int64_t wlo = a.pull.wpart[part], whi = a.pull.wpart[part + 1];
    for (int64_t w = wlo; w < whi; ++w) {
      const int64_t v = w * 64 + ln;
      const bool inb = v < a.n;
      uint64_t on_m = ~0ull;
      if (AD) {
        on_m = a.act_cur[w];
        const uint64_t was = a.act_prev[w];
        // frozen in the previous iteration: x enters the other buffer once
        if (inb && (((was & ~on_m) >> ln) & 1ull)) xn[v] = x[v];
        if (!on_m) {  // the word's rows are all frozen
          if (ln == 0) a.act_nxt[w] = 0ull;
          continue;
        }
      }
      const bool on = inb && ((on_m >> ln) & 1ull);
      int cur = 0, end = 0;
      bool split = false;
      if (on) {
        cur = rp[v];
        end = rp[v + 1];
        split = end - cur > kPushSplit;
        if (AD) {
          upd += 1.0;
          edges += (double)(end - cur);
        }
      }
      const bool act = on && !split;
      // the word's rows' in-edges as one list of `total` positions; the
      // prefix ends of the rows go to LDS once, and every 64-position step
      // finds its rows there by bisection, so no step waits on the one before
      // and the loads of kSweepUnroll steps are in flight together
      const int len = act ? end - cur : 0;
      const int incl = wave_incl_scan(len);
      const int total = lane_last(incl);
      s_end[wid][ln] = incl;
      s_base[wid][ln] = cur - (incl - len);  // position q of this row's edges: base + q
      s_acc[wid][ln] = (T)0;
      wave_lds_sync();
      for (int q0 = 0; q0 < total; q0 += 64 * kSweepUnroll) {
        int row[kSweepUnroll], c[kSweepUnroll];
        bool last[kSweepUnroll];
  #pragma unroll
        for (int s = 0; s < kSweepUnroll; ++s) {
          const int q = q0 + s * 64 + ln;
          row[s] = -1;
          last[s] = false;
          c[s] = -1;
          if (q < total) {
            int r = 0;
  #pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
              if (s_end[wid][r + step - 1] <= q) r += step;
            row[s] = r;
            last[s] = q + 1 == s_end[wid][r] || ln == 63;
            c[s] = s_base[wid][r] + q;
          }
        }
  #pragma unroll
        for (int s = 0; s < kSweepUnroll; ++s) c[s] = c[s] >= 0 ? ci[c[s]] : -1;
        T val[kSweepUnroll];
  #pragma unroll
        for (int s = 0; s < kSweepUnroll; ++s) val[s] = c[s] >= 0 ? x[c[s]] : (T)0;
  #pragma unroll
        for (int s = 0; s < kSweepUnroll; ++s) {
          const T y = seg_sum_scan<T>(val[s], row[s]);
          if (last[s]) atomicAdd(&s_acc[wid][row[s]], y);  // one segment per row and step
        }
      }
      wave_lds_sync();
      const T acc = s_acc[wid][ln];
      bool keep = false;
      if (act) {
        const T po = p[v];
        const T pn = rank_update<T>(a, acc, dn);
        const double ch = fabs((double)pn - (double)po);
        delta += ch;
        p[v] = pn;
        const int od = a.out_rp[v + 1] - a.out_rp[v];
        if (od == 0) {
          xn[v] = (T)0;
          dang += (double)pn;
        } else {
          xn[v] = pn / (T)od;
        }
        if (AD) {
          keep = !(ch <= a.eps * (double)po);
          if (!keep && od == 0) dfz += (double)pn;
        }
      }
      if (AD) {
        // long rows stay set; their kernel clears the bit if they freeze
        const uint64_t nx = __ballot(keep || (on && split));
        if (ln == 0) {
          a.act_nxt[w] = nx;
          after += (double)__popcll(nx);
        }
      }
    }
  }
  // pieces of long rows (kPushSplit edges each), spread over the waves and
  // two at a time; each piece's sum goes to its slot for the fix-up kernel
  static_assert(kPushSplit == 64 * kUnroll, "a piece is one unrolled step");
  T *hp = (T *)a.heavy_part;
  for (int64_t h0 = gw; h0 < a.pull.nsplit; h0 += 2 * nwaves) {
    int pb[2], pe[2];
    int64_t ph[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ph[q] = h0 + q * nwaves;
      pb[q] = pe[q] = 0;
      if (ph[q] < a.pull.nsplit) {
        const int r = a.pull.split[2 * ph[q]];
        if (!AD || bit_of(a.act_cur, r)) {  // frozen rows: no work
          pb[q] = a.pull.split[2 * ph[q] + 1];
          pe[q] = min(pb[q] + kPushSplit, rp[r + 1]);
        }
      }
    }
    int c[2][kUnroll];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int pos = pb[q] + s * 64 + ln;
        c[q][s] = pos < pe[q] ? ci[pos] : -1;
      }
    T val[2][kUnroll];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) val[q][s] = c[q][s] >= 0 ? x[c[q][s]] : (T)0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T sum = (val[q][0] + val[q][1]) + (val[q][2] + val[q][3]);
      sum = lane_last(wave_scan(sum, (T)0, OpAdd()));  // fixed order
      if (ln == 0 && ph[q] < a.pull.nsplit) hp[ph[q]] = sum;
    }
  }
  double pv[kPrFields] = {delta, dang, dfz, after, upd, edges};
  block_partials(pv, a.blk_part);
}

// Long rows: one wave per row adds the row's pieces (lane l the pieces
// l, l + 64, ... in order, then a fixed-order reduction over the lanes) and
// updates its rank; per-workgroup partials follow those of the SpMV kernel.
template <class T, bool AD>
__global__ __launch_bounds__(kBlock) void k_pr_long(PrArgs a) {
  if (a.ctrl->converged) return;
  const T dn = (T)(a.ctrl->D / (double)a.n);
  const T *hp = (const T *)a.heavy_part;
  T *p = (T *)a.p;
  T *xn = (T *)a.xn;
  const int ln = threadIdx.x & 63;
  double delta = 0, dang = 0, dfz = 0, after = 0;
  const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (i < a.pull.nsplit_rows) {
    const int r = a.pull.split_rows[3 * i], first = a.pull.split_rows[3 * i + 1],
              cnt = a.pull.split_rows[3 * i + 2];
    if (!AD || bit_of(a.act_cur, r)) {
      T part = (T)0;
      for (int k = ln; k < cnt; k += 64) part += hp[first + k];
      const T acc = lane_last(wave_scan(part, (T)0, OpAdd()));
      if (ln == 0) {
        const T po = p[r];
        const T pn = rank_update<T>(a, acc, dn);
        const double ch = fabs((double)pn - (double)po);
        delta = ch;
        p[r] = pn;
        const int od = a.out_rp[r + 1] - a.out_rp[r];
        if (od == 0) {
          xn[r] = (T)0;
          dang = (double)pn;
        } else {
          xn[r] = pn / (T)od;
        }
        if (AD && ch <= a.eps * (double)po) {  // freezes: clear its bit
          atomicAnd((unsigned long long *)&a.act_nxt[r >> 6], ~(1ull << (r & 63)));
          after = -1.0;
          if (od == 0) dfz = (double)pn;
        }
      }
    }
  }
  double pv[kPrFields] = {delta, dang, dfz, after, 0.0, 0.0};
  block_partials(pv, a.blk_part + kPrFields * a.nblk);
}

// One workgroup: reduces the per-workgroup partials in a fixed order and
// updates the control block (dangling mass, L1 change, convergence; for
// the adaptive form also the frozen dangling mass, the active count and the
// iteration's record).
template <class T>
__global__ __launch_bounds__(1024) void k_pr_fixup(PrArgs a, int init) {
  __shared__ double s_v[16][kPrFields];
  if (!init && a.ctrl->converged) return;
  double v[kPrFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int nparts = init ? a.nblk : a.nblk + a.nblk_long;
  for (int i = threadIdx.x; i < nparts; i += 1024)
#pragma unroll
    for (int f = 0; f < kPrFields; ++f) v[f] += a.blk_part[kPrFields * i + f];
#pragma unroll
  for (int f = 0; f < kPrFields; ++f) {
    v[f] = wave_sum_f64(v[f]);
    if ((threadIdx.x & 63) == 0) s_v[threadIdx.x >> 6][f] = v[f];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kPrFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int f = 0; f < kPrFields; ++f) t[f] += s_v[i][f];
    Ctrl *c = a.ctrl;
    if (init) {
      c->D = t[1];
      c->Dfz = 0.0;
      c->active = a.act_cur ? a.n : 0;
      c->iters = 0;
      c->converged = 0;
      c->delta = 0.0;
    } else {
      const double dfz_old = a.act_cur ? c->Dfz : 0.0;
      c->D = t[1] + dfz_old;
      c->delta = t[0];
      if (a.act_cur) {
        c->Dfz = dfz_old + t[2];
        c->active = (int64_t)t[3];
        if (a.stats && c->iters < kStatsCap) {
          int64_t *r = a.stats + (size_t)c->iters * kStatFields;
          r[0] = (int64_t)t[4];
          r[1] = (int64_t)t[5];
          r[2] = GRB_DIR_PULL;
          r[3] = (int64_t)t[3];
        }
      }
      c->iters += 1;
      if (t[0] < a.tol) c->converged = 1;
      if (a.act_cur && c->active == 0) c->converged = 1;
    }
  }
}

}  // namespace

int pr_long_grid(int64_t nsplit_rows) {
  return (int)((nsplit_rows + kWavesPerBlock - 1) / kWavesPerBlock);  // a wave per row
}

void launch_pr_init(int is_fp64, const PrArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (is_fp64) {
    hipLaunchKernelGGL(k_pr_init<double>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_pr_fixup<double>, dim3(1), dim3(1024), 0, s, a, 1);
  } else {
    hipLaunchKernelGGL(k_pr_init<float>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_pr_fixup<float>, dim3(1), dim3(1024), 0, s, a, 1);
  }
}

template <class T, bool AD>
static void pr_iter_launch(const PrArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_pr_iter<T, AD>), dim3(a.nblk), dim3(kBlock), 0, s, a);
  if (a.nblk_long > 0)
    hipLaunchKernelGGL((k_pr_long<T, AD>), dim3(a.nblk_long), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_pr_fixup<T>, dim3(1), dim3(1024), 0, s, a, 0);
}

void launch_pr_iter(int is_fp64, const PrArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const bool ad = a.act_cur != nullptr;
  if (is_fp64) {
    if (ad) pr_iter_launch<double, true>(a, s);
    else pr_iter_launch<double, false>(a, s);
  } else {
    if (ad) pr_iter_launch<float, true>(a, s);
    else pr_iter_launch<float, false>(a, s);
  }
}

}  // namespace grb
