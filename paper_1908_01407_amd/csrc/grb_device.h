// Device helpers for wave64 (gfx950): scans, reductions, bitmap tests,
// scoped atomics and the slot-to-row map of the wave-level load-balanced
// search used by every pull kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace grb {

__device__ __forceinline__ uint64_t mask_below(int k) {
  return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
}

__device__ __forceinline__ bool bit_of(const uint64_t *bm, int64_t v) {
  return (bm[v >> 6] >> (v & 63)) & 1ull;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int ln = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (ln >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ int wave_max_scan(int x) {
  const int ln = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (ln >= off) x = max(x, y);
  }
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fminf(x, __shfl_xor(x, off));
  return x;
}

// Orders this wave's LDS traffic (lanes of one wave exchange data through LDS).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The bitmap words [lo, hi) a wave owns in a grid-wide sweep: one
// contiguous run per wave, so lanes can load 64 of them at once.
__device__ __forceinline__ void wave_words(int64_t nw, int64_t gw, int64_t nwaves, int64_t &lo,
                                           int64_t &hi) {
  const int64_t per = (nw + nwaves - 1) / nwaves;
  lo = gw * per;
  hi = lo + per < nw ? lo + per : nw;
}

// Wave-level load-balanced search: lane `l` owns a row whose remaining
// edges occupy slots [excl, excl + len) of a concatenated stream.  For every
// slot s in [0, 64) this returns the lane whose row covers s (the row that
// starts at the largest start <= s).  `mark` is 64 ints of LDS private to the
// wave.  Slot 0 is always covered when any row is non-empty.
__device__ __forceinline__ int slot_rows(int *mark, bool starts, int excl) {
  const int ln = threadIdx.x & 63;
  mark[ln] = -1;
  wave_lds_sync();
  if (starts) mark[excl] = ln;
  wave_lds_sync();
  const int r = wave_max_scan(mark[ln]);
  wave_lds_sync();
  return r;
}

// Position of the n-th (0-based) set bit of x, found by halving the window
// with popcounts; x must have more than n set bits.
__device__ __forceinline__ int nth_set_bit(uint64_t x, int n) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const int c = __popcll((x >> pos) & mask_below(w));
    if (n >= c) {
      n -= c;
      pos += w;
    }
  }
  return pos;
}

// Wave-local compaction of a bitmap: lane l holds word m (bitmap word index
// `word`), its popcount `cnt` and the inclusive scan `incl` of the counts.
// Returns the vertex of slot b + lane of the enumeration of all set bits in
// lane order (-1 past the end, `total` = the last lane's incl).
__device__ __forceinline__ int64_t queue_slot(int *mark, uint64_t m, int cnt, int incl, int total,
                                              int b, int64_t word) {
  const int ln = threadIdx.x & 63;
  const int excl = incl - cnt;
  const bool starts = cnt > 0 && incl > b && excl < b + 64;
  const int k = slot_rows(mark, starts, excl > b ? excl - b : 0);
  const uint64_t mk = __shfl(m, k);
  const int ek = __shfl(excl, k);
  const int64_t wk = __shfl(word, k);
  const int sl = b + ln;
  return sl < total ? wk * 64 + nth_set_bit(mk, sl - ek) : -1;
}

// Lanes hold (word, bits) where lanes with equal words are contiguous.
// Returns to the first lane of each run of equal words the OR of the run's
// bits, to every other lane 0.
__device__ __forceinline__ uint64_t run_head_or(int64_t word, uint64_t bits) {
  const int ln = threadIdx.x & 63;
  const int64_t prev = __shfl_up(word, 1);
  const bool head = ln == 0 || prev != word;
  const int rid = wave_max_scan(head ? ln : -1);
  uint64_t x = bits;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_down(x, off);
    const int ry = __shfl_down(rid, off);
    if (ln + off < 64 && ry == rid) x |= y;
  }
  return head ? x : 0ull;
}

// Inclusive min-scan over slots restricted to runs of equal row id.
__device__ __forceinline__ float seg_min_scan(float x, int row) {
  const int ln = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const float y = __shfl_up(x, off);
    const int ry = __shfl_up(row, off);
    if (ln >= off && ry == row) x = fminf(x, y);
  }
  return x;
}

template <class T>
__device__ __forceinline__ T seg_sum_scan(T x, int row) {
  const int ln = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off);
    const int ry = __shfl_up(row, off);
    if (ln >= off && ry == row) x += y;
  }
  return x;
}

// Device-coherent atomic store / load of a 64-bit word.  Relaxed ordering:
// the word itself carries everything the reader needs, so no other memory
// has to be made visible with it (release/acquire at device scope would
// write back / invalidate the per-XCD L2 caches on every call).
__device__ __forceinline__ void store_relaxed_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed_u64(uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// atomic min for floats of either sign (returns the previous value)
__device__ __forceinline__ float atomic_min_f32(float *a, float v) {
  if (!(v < 0.0f)) return __int_as_float(atomicMin((int *)a, __float_as_int(v)));
  return __uint_as_float(atomicMax((unsigned *)a, __float_as_uint(v)));
}

__device__ __forceinline__ double atomic_min_f64(double *a, double v) {
  if (!(v < 0.0)) {
    return __longlong_as_double(
        atomicMin((long long *)a, (long long)__double_as_longlong(v)));
  }
  return __longlong_as_double((long long)atomicMax(
      (unsigned long long *)a, (unsigned long long)__double_as_longlong(v)));
}

}  // namespace grb
