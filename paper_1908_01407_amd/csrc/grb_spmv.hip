// PageRank iteration kernels (Section 7.3 of the paper: pull form, SpMV
// every iteration because the vector never gets sparse).
//
// Load balance: each wave takes a run of bitmap words of rows (64
// consecutive rows of the CSR of A^T each), runs of about equal work built
// by grb_matrix_prepare, one word per step, and
// streams their in-edges as one concatenated list, kUnroll x 64 edges per
// step, with a segmented sum per row (wave-level load-balanced search);
// rows longer than kPushSplit are cut into fixed pieces that any wave
// takes, and a second kernel (one thread per long row) adds each long
// row's pieces in order.  Summation order is fixed, so fp32 and fp64 results are bitwise
// reproducible run to run.  The dangling mass and the L1 change are reduced
// per workgroup and then in a fixed order in the fix-up kernel, which also
// decides convergence on the device.
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

template <class T>
__device__ __forceinline__ void block_partials(double delta, double dang, double *out) {
  __shared__ double s_red[kWavesPerBlock][2];
  delta = wave_sum_f64(delta);
  dang = wave_sum_f64(dang);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[wid][0] = delta;
    s_red[wid][1] = dang;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double d0 = 0, d1 = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      d0 += s_red[i][0];
      d1 += s_red[i][1];
    }
    out[2 * blockIdx.x + 0] = d0;
    out[2 * blockIdx.x + 1] = d1;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_pr_init(PrArgs a) {
  T *p = (T *)a.p;
  T *xn = (T *)a.xn;
  const T p0 = (T)(1.0 / (double)a.n);
  double dang = 0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * kBlock) {
    p[v] = p0;
    const int od = a.out_rp[v + 1] - a.out_rp[v];
    if (od == 0) {
      xn[v] = (T)0;
      dang += (double)p0;
    } else {
      xn[v] = p0 / (T)od;
    }
  }
  block_partials<T>(0.0, dang, a.blk_part);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_pr_iter(PrArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  if (a.ctrl->converged) return;
  int *mark = s_mark[threadIdx.x >> 6];
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const T *x = (const T *)a.x;
  T *xn = (T *)a.xn;
  T *p = (T *)a.p;
  const T dn = (T)(a.ctrl->D / (double)a.n);
  double delta = 0, dang = 0;
  // rows up to kPushSplit long: the wave's run of words (about equal work
  // per run), one word of rows per step; kUnroll x 64 edges per step (slot
  // positions first, then all gathers, then the segmented sums in slot order)
  const int64_t wlo = gw < kWaveParts ? a.pull.wpart[gw] : 0;
  const int64_t whi = gw < kWaveParts ? a.pull.wpart[gw + 1] : 0;
  for (int64_t w = wlo; w < whi; ++w) {
    const int64_t v = w * 64 + ln;
    const bool inb = v < a.n;
    int cur = 0, end = 0;
    bool split = false;
    if (inb) {
      cur = rp[v];
      end = rp[v + 1];
      split = end - cur > kPushSplit;
    }
    const bool act = inb && !split;
    if (!act) end = cur;
    T acc = (T)0;
    for (bool more = true; more;) {
      int pos[kUnroll], row[kUnroll], se[kUnroll];
      bool st[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        pos[s] = -1;
        row[s] = 0;
        se[s] = 0;
        st[s] = false;
        if (!more) continue;
        const int len = end - cur;
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
        se[s] = min(incl, 64);
        if (starts) cur += se[s] - excl;
      }
      int c[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) c[s] = pos[s] >= 0 ? ci[pos[s]] : -1;
      T val[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) val[s] = c[s] >= 0 ? x[c[s]] : (T)0;
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const T y = seg_sum_scan<T>(val[s], row[s]);
        const T seg = __shfl(y, st[s] ? se[s] - 1 : 0);
        if (st[s]) acc += seg;
      }
    }
    if (act) {
      const T pn = rank_update<T>(a, acc, dn);
      delta += fabs((double)pn - (double)p[v]);
      p[v] = pn;
      const int od = a.out_rp[v + 1] - a.out_rp[v];
      if (od == 0) {
        xn[v] = (T)0;
        dang += (double)pn;
      } else {
        xn[v] = pn / (T)od;
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
        pb[q] = a.pull.split[2 * ph[q] + 1];
        pe[q] = min(pb[q] + kPushSplit, rp[r + 1]);
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
  block_partials<T>(delta, dang, a.blk_part);
}

// Long rows: one thread per row adds the row's pieces in order and updates
// its rank; per-workgroup partials follow those of the SpMV kernel.
template <class T>
__global__ __launch_bounds__(kBlock) void k_pr_long(PrArgs a) {
  if (a.ctrl->converged) return;
  const T dn = (T)(a.ctrl->D / (double)a.n);
  const T *hp = (const T *)a.heavy_part;
  T *p = (T *)a.p;
  T *xn = (T *)a.xn;
  double delta = 0, dang = 0;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < a.pull.nsplit_rows) {
    const int r = a.pull.split_rows[3 * i], first = a.pull.split_rows[3 * i + 1],
              cnt = a.pull.split_rows[3 * i + 2];
    T acc = (T)0;
    for (int k = 0; k < cnt; ++k) acc += hp[first + k];
    const T pn = rank_update<T>(a, acc, dn);
    delta = fabs((double)pn - (double)p[r]);
    p[r] = pn;
    const int od = a.out_rp[r + 1] - a.out_rp[r];
    if (od == 0) {
      xn[r] = (T)0;
      dang = (double)pn;
    } else {
      xn[r] = pn / (T)od;
    }
  }
  block_partials<T>(delta, dang, a.blk_part + 2 * a.nblk);
}

// One workgroup: reduces the per-workgroup partials in a fixed order and
// updates the control block (dangling mass, L1 change, convergence).
template <class T>
__global__ __launch_bounds__(1024) void k_pr_fixup(PrArgs a, int init) {
  __shared__ double s_d[16], s_g[16];
  if (!init && a.ctrl->converged) return;
  double delta = 0, dang = 0;
  const int nparts = init ? a.nblk : a.nblk + a.nblk_long;
  for (int i = threadIdx.x; i < nparts; i += 1024) {
    delta += a.blk_part[2 * i];
    dang += a.blk_part[2 * i + 1];
  }
  delta = wave_sum_f64(delta);
  dang = wave_sum_f64(dang);
  if ((threadIdx.x & 63) == 0) {
    s_d[threadIdx.x >> 6] = delta;
    s_g[threadIdx.x >> 6] = dang;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double d = 0, g = 0;
    for (int i = 0; i < 16; ++i) {
      d += s_d[i];
      g += s_g[i];
    }
    a.ctrl->D = g;
    if (init) {
      a.ctrl->iters = 0;
      a.ctrl->converged = 0;
      a.ctrl->delta = 0.0;
    } else {
      a.ctrl->delta = d;
      a.ctrl->iters += 1;
      if (d < a.tol) a.ctrl->converged = 1;
    }
  }
}

}  // namespace

int pr_long_grid(int64_t nsplit_rows) {
  return (int)((nsplit_rows + kBlock - 1) / kBlock);
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

void launch_pr_iter(int is_fp64, const PrArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (is_fp64) {
    hipLaunchKernelGGL(k_pr_iter<double>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    if (a.nblk_long > 0)
      hipLaunchKernelGGL(k_pr_long<double>, dim3(a.nblk_long), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_pr_fixup<double>, dim3(1), dim3(1024), 0, s, a, 0);
  } else {
    hipLaunchKernelGGL(k_pr_iter<float>, dim3(a.nblk), dim3(kBlock), 0, s, a);
    if (a.nblk_long > 0)
      hipLaunchKernelGGL(k_pr_long<float>, dim3(a.nblk_long), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_pr_fixup<float>, dim3(1), dim3(1024), 0, s, a, 0);
  }
}

}  // namespace grb
