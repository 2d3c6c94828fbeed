// Masked sparse matrix-matrix product in the dot-product form,
// C = (A B^T) .* M, and triangle counting as its reduction to a scalar
// (Sections 6.3.4 (masked SpGEMM) and 7.5: with L the strict lower triangle
// of a symmetric adjacency, the triangle count is the sum of L L^T .* L).
//
// Only the entries the mask holds are computed: C(i, j) for j in M(i, :) is
// the sum over k of A(i, k) * B(j, k), i.e. the intersection of row i of A
// with row j of B (B is given by its rows, the columns of B^T).  The
// paper's kernel gives one warp a row of the mask and binary-searches the
// column of B for each element of A's row.  Here one wave takes a row i of
// the mask (rows dealt out round-robin), copies row i of A into its own LDS
// segment once, and streams the rows j of B named by the mask row as one
// concatenated list, kUnroll x 64 entries per step (the same wave-level
// load-balanced search as the pull kernels); every entry k is looked up in
// the LDS copy by binary search.  A row of A longer than the LDS segment is
// searched in place in global memory.  With the vertices numbered by
// decreasing degree, a row of L holds only neighbours of at least the
// row's degree, at most sqrt(2 nnz) of them, so the searched rows fit the
// segment and the streamed rows are the short rows of high-degree vertices
// that every wave re-reads from the caches.
//
// Triangle counting fuses the reduction into the product (the kernel
// fusion the paper names as open work): nothing of C is written, each wave
// counts its hits, and one atomic per workgroup adds the total.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

// first index in col[0, d) holding a value >= k (ascending list)
template <class P>
__device__ __forceinline__ int lower_pos(P col, int d, int32_t k) {
  int lo = 0, len = d;
  while (len > 0) {
    const int half = len >> 1;
    if (col[lo + half] < k) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// product of A(i, k) and B(j, k) under the semiring's multiply: 1 for
// PLUS_PAIR (structure only), a * b for PLUS_TIMES
template <class V>
struct Mul {
  __device__ __forceinline__ static V get(const void *aval, int64_t ia, const void *bval,
                                          int64_t ib) {
    return ((const V *)aval)[ia] * ((const V *)bval)[ib];
  }
};
template <>
struct Mul<int> {
  __device__ __forceinline__ static int get(const void *, int64_t, const void *, int64_t) {
    return 1;
  }
};

// COUNT: add the hits into *a.count (V must be int, PLUS_PAIR); otherwise
// write C(i, j) = sum of the products to c[e] for every mask entry e.
template <class V, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_mxm_dot(MxmArgs a) {
  __shared__ int32_t s_col[kWavesPerBlock][kMxmLds];
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ unsigned long long s_cnt[kWavesPerBlock];
  const int wid = threadIdx.x >> 6;
  const int ln = threadIdx.x & 63;
  int32_t *lcol = s_col[wid];
  int *mark = s_mark[wid];
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *mrp = a.M.rp, *mci = a.M.ci;
  const int32_t *arp = a.A.rp, *aci = a.A.ci;
  const int32_t *brp = a.B.rp, *bci = a.B.ci;
  V *c = (V *)a.c;
  unsigned long long hits = 0;  // COUNT: wave-uniform
  for (int64_t i = gw; i < a.nrows; i += nwaves) {
    const int mb = mrp[i], me = mrp[i + 1];
    if (mb == me) continue;
    const int ab = arp[i];
    const int da = arp[i + 1] - ab;
    if (da == 0) {  // empty row of A: every entry of the row is zero
      if (!COUNT)
        for (int e = mb + ln; e < me; e += 64) c[e] = (V)0;
      continue;
    }
    const bool in_lds = da <= kMxmLds;
    if (in_lds) {
      for (int t = ln; t < da; t += 64) lcol[t] = aci[ab + t];
      wave_lds_sync();
    }
    // the mask row's entries, 64 at a time (one per lane)
    for (int e0 = mb; e0 < me; e0 += 64) {
      const int e = e0 + ln;
      const bool has = e < me;
      int cur = 0, end = 0;
      if (has) {
        const int j = mci[e];
        cur = brp[j];
        end = brp[j + 1];
      }
      V acc = (V)0;
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
        int32_t kk[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) kk[s] = pos[s] >= 0 ? bci[pos[s]] : -1;
        int at[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          at[s] = -1;
          if (kk[s] >= 0) {
            const int p = in_lds ? lower_pos(lcol, da, kk[s]) : lower_pos(aci + ab, da, kk[s]);
            const int32_t got = p < da ? (in_lds ? lcol[p] : aci[ab + p]) : -1;
            if (got == kk[s]) at[s] = p;
          }
        }
        if (COUNT) {
#pragma unroll
          for (int s = 0; s < kUnroll; ++s) hits += (unsigned long long)__popcll(__ballot(at[s] >= 0));
        } else {
#pragma unroll
          for (int s = 0; s < kUnroll; ++s) {
            const V v = at[s] >= 0 ? Mul<V>::get(a.A.val, (int64_t)ab + at[s], a.B.val, pos[s])
                                   : (V)0;
            const V y = seg_sum_scan<V>(v, row[s]);
            const V seg = __shfl(y, st[s] ? se[s] - 1 : 0);
            if (st[s]) acc += seg;
          }
        }
      }
      if (!COUNT && has) c[e] = acc;
    }
    if (in_lds) wave_lds_sync();  // the next row overwrites the segment
  }
  if (COUNT) {
    if (ln == 0) s_cnt[wid] = hits;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) t += s_cnt[w];
      if (t) atomicAdd(a.count, t);
    }
  }
}

// Structure-only product (PLUS_PAIR: C(i, j) = |A(i, :) and B(j, :)|) and
// the fused triangle count.  Membership in row i of A is a bit test: each
// wave keeps a bitmap of kPairBits columns in LDS, sets the bits of row i's
// entries below kPairBits, and keeps the rest of the row (its tail, the
// entries at or above kPairBits; rows are sorted, so they come last) as a
// sorted LDS list searched by bisection.  Under the degree numbering the
// columns of a row are the ids of higher-degree vertices, which are small
// numbers, so nearly every probe is a bit test.  Rows of B with at least
// kPairLong entries are streamed one at a time, 64 x kUnroll entries per
// step with no per-step bookkeeping; shorter ones go through the
// load-balanced concatenated stream.
__device__ __forceinline__ bool pair_hit(const uint32_t *bm, const int32_t *tail, int dt,
                                         bool tail_lds, const int32_t *gtail, int32_t k) {
  if (k < kPairBits) return (bm[k >> 5] >> (k & 31)) & 1u;
  if (dt == 0) return false;
  const int p = tail_lds ? lower_pos(tail, dt, k) : lower_pos(gtail, dt, k);
  return p < dt && (tail_lds ? tail[p] : gtail[p]) == k;
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void k_mxm_pair(MxmArgs a) {
  __shared__ uint32_t s_bm[kWavesPerBlock][kPairBits / 32];
  __shared__ int32_t s_tail[kWavesPerBlock][kPairTail];
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ unsigned long long s_cnt[kWavesPerBlock];
  const int wid = threadIdx.x >> 6;
  const int ln = threadIdx.x & 63;
  uint32_t *bm = s_bm[wid];
  int32_t *tail = s_tail[wid];
  int *mark = s_mark[wid];
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *mrp = a.M.rp, *mci = a.M.ci;
  const int32_t *arp = a.A.rp, *aci = a.A.ci;
  const int32_t *brp = a.B.rp, *bci = a.B.ci;
  int *c = (int *)a.c;
  for (int t = ln; t < kPairBits / 32; t += 64) bm[t] = 0u;
  wave_lds_sync();
  unsigned long long hits = 0;  // COUNT: wave-uniform
  for (int64_t i = gw; i < a.nrows; i += nwaves) {
    const int mb = mrp[i], me = mrp[i + 1];
    if (mb == me) continue;
    const int ab = arp[i];
    const int da = arp[i + 1] - ab;
    if (da == 0) {
      if (!COUNT)
        for (int e = mb + ln; e < me; e += 64) c[e] = 0;
      continue;
    }
    // bits of the entries below kPairBits (a prefix of the sorted row)
    int t0 = 0;
    for (int t = 0; t < da; t += 64) {
      const int32_t k = t + ln < da ? aci[ab + t + ln] : INT32_MAX;
      const bool low = k < kPairBits;
      if (low) atomicOr(&bm[k >> 5], 1u << (k & 31));
      t0 += __popcll(__ballot(low));
    }
    const int dt = da - t0;
    const bool tail_lds = dt <= kPairTail;
    if (tail_lds)
      for (int t = ln; t < dt; t += 64) tail[t] = aci[ab + t0 + t];
    wave_lds_sync();
    const int32_t *gtail = aci + ab + t0;
    for (int e0 = mb; e0 < me; e0 += 64) {
      const int e = e0 + ln;
      const bool has = e < me;
      int cur = 0, end = 0;
      if (has) {
        const int j = mci[e];
        cur = brp[j];
        end = brp[j + 1];
      }
      int acc = 0;
      // long rows of B, one at a time
      uint64_t lm = __ballot(has && end - cur >= kPairLong);
      while (lm) {
        const int l = __ffsll((unsigned long long)lm) - 1;
        lm &= lm - 1;
        const int rb = __shfl(cur, l), re = __shfl(end, l);
        int cnt = 0;
        for (int p0 = rb; p0 < re; p0 += 64 * kPairUnroll) {
          int32_t kk[kPairUnroll];
#pragma unroll
          for (int s = 0; s < kPairUnroll; ++s) {
            const int p = p0 + s * 64 + ln;
            kk[s] = p < re ? bci[p] : -1;
          }
#pragma unroll
          for (int s = 0; s < kPairUnroll; ++s)
            cnt += __popcll(__ballot(kk[s] >= 0 && pair_hit(bm, tail, dt, tail_lds, gtail, kk[s])));
        }
        if (COUNT) hits += (unsigned long long)cnt;
        else if (ln == l) acc += cnt;
      }
      // short rows as one concatenated stream
      if (has && end - cur >= kPairLong) end = cur;
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
        int32_t kk[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) kk[s] = pos[s] >= 0 ? bci[pos[s]] : -1;
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          const bool hit = kk[s] >= 0 && pair_hit(bm, tail, dt, tail_lds, gtail, kk[s]);
          if (COUNT) {
            hits += (unsigned long long)__popcll(__ballot(hit));
          } else {
            const int y = seg_sum_scan<int>(hit ? 1 : 0, row[s]);
            const int seg = __shfl(y, st[s] ? se[s] - 1 : 0);
            if (st[s]) acc += seg;
          }
        }
      }
      if (!COUNT && has) c[e] = acc;
    }
    // clear the row's bits for the next row
    wave_lds_sync();
    for (int t = ln; t < t0; t += 64) bm[aci[ab + t] >> 5] = 0u;
    wave_lds_sync();
  }
  if (COUNT) {
    if (ln == 0) s_cnt[wid] = hits;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) t += s_cnt[w];
      if (t) atomicAdd(a.count, t);
    }
  }
}

}  // namespace

void launch_mxm_dot(const MxmArgs &a, bool count, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const dim3 g(kExpandGrid), b(kBlock);
  if (count) {
    hipLaunchKernelGGL((k_mxm_pair<true>), g, b, 0, s, a);
  } else if (a.vt != GRB_FP32 && a.vt != GRB_FP64) {
    hipLaunchKernelGGL((k_mxm_pair<false>), g, b, 0, s, a);
  } else if (a.vt == GRB_FP32) {
    hipLaunchKernelGGL((k_mxm_dot<float, false>), g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_mxm_dot<double, false>), g, b, 0, s, a);
  }
}

}  // namespace grb
