// Device helpers for wave64 (gfx950): scans, reductions, bitmap tests,
// scoped atomics and the slot-to-row map of the wave-level load-balanced
// search used by every pull kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "grb_internal.h"

namespace grb {

__device__ __forceinline__ uint64_t mask_below(int k) {
  return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
}

__device__ __forceinline__ bool bit_of(const uint64_t *bm, int64_t v) {
  return (bm[v >> 6] >> (v & 63)) & 1ull;
}

// ---- lane movement with DPP ---------------------------------------------
// Inclusive scans run Hillis-Steele over the wave with DPP moves instead of
// LDS shuffles: row_shr:1,2,4,8 within each row of 16 lanes, then
// row_bcast:15 (lane 15 of a row into the next row, rows 1 and 3) and
// row_bcast:31 (lane 31 into rows 2 and 3).  A lane whose source is outside
// its row, or whose row is masked off, receives `old` (the operation's
// identity).  All 64 lanes must be active.
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppBcast15 = 0x142, kDppBcast31 = 0x143;
constexpr int kDppWaveShl1 = 0x130;  // lane i receives lane i + 1
constexpr int kDppWaveShr1 = 0x138;  // lane i receives lane i - 1

template <int C, int R>
__device__ __forceinline__ int dpp_move(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, C, R, 0xf, false);
}
template <int C, int R>
__device__ __forceinline__ float dpp_move(float old, float v) {
  return __int_as_float(dpp_move<C, R>(__float_as_int(old), __float_as_int(v)));
}
template <int C, int R>
__device__ __forceinline__ uint64_t dpp_move(uint64_t old, uint64_t v) {
  const int lo = dpp_move<C, R>((int)(uint32_t)old, (int)(uint32_t)v);
  const int hi = dpp_move<C, R>((int)(uint32_t)(old >> 32), (int)(uint32_t)(v >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}
template <int C, int R>
__device__ __forceinline__ int64_t dpp_move(int64_t old, int64_t v) {
  return (int64_t)dpp_move<C, R>((uint64_t)old, (uint64_t)v);
}
template <int C, int R>
__device__ __forceinline__ double dpp_move(double old, double v) {
  return __longlong_as_double(
      (long long)dpp_move<C, R>((uint64_t)__double_as_longlong(old), (uint64_t)__double_as_longlong(v)));
}

// inclusive scan of `op` (identity `id`) over the 64 lanes
template <class T, class Op>
__device__ __forceinline__ T wave_scan(T x, T id, Op op) {
  x = op(x, dpp_move<kDppShr1, 0xf>(id, x));
  x = op(x, dpp_move<kDppShr2, 0xf>(id, x));
  x = op(x, dpp_move<kDppShr4, 0xf>(id, x));
  x = op(x, dpp_move<kDppShr8, 0xf>(id, x));
  x = op(x, dpp_move<kDppBcast15, 0xa>(id, x));
  x = op(x, dpp_move<kDppBcast31, 0xc>(id, x));
  return x;
}

// inclusive scan restricted to runs of equal `seg` (runs must be contiguous
// and seg >= 0)
template <class T, class Op>
__device__ __forceinline__ T wave_seg_scan(T x, int seg, T id, Op op) {
#define GRB_SEG_STEP(C, R)                          \
  {                                                 \
    const T y = dpp_move<C, R>(id, x);              \
    const int sy = dpp_move<C, R>(-1, seg);         \
    if (sy == seg) x = op(x, y);                    \
  }
  GRB_SEG_STEP(kDppShr1, 0xf)
  GRB_SEG_STEP(kDppShr2, 0xf)
  GRB_SEG_STEP(kDppShr4, 0xf)
  GRB_SEG_STEP(kDppShr8, 0xf)
  GRB_SEG_STEP(kDppBcast15, 0xa)
  GRB_SEG_STEP(kDppBcast31, 0xc)
#undef GRB_SEG_STEP
  return x;
}

// value of lane 63 (uniform)
__device__ __forceinline__ int lane_last(int x) { return __builtin_amdgcn_readlane(x, 63); }
__device__ __forceinline__ float lane_last(float x) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ __forceinline__ double lane_last(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

struct OpAdd {
  template <class T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  __device__ __forceinline__ int operator()(int a, int b) const { return a > b ? a : b; }
};
struct OpMinF {
  __device__ __forceinline__ float operator()(float a, float b) const { return fminf(a, b); }
};
struct OpOr {
  __device__ __forceinline__ uint64_t operator()(uint64_t a, uint64_t b) const { return a | b; }
};

__device__ __forceinline__ int wave_incl_scan(int x) { return wave_scan(x, 0, OpAdd()); }

__device__ __forceinline__ int wave_max_scan(int x) { return wave_scan(x, INT_MIN, OpMax()); }

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

// minimum over the wave, returned to every lane
__device__ __forceinline__ float wave_min(float x) {
  return lane_last(wave_scan(x, __int_as_float(0x7f800000), OpMinF()));
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

// Lanes hold (word, bits) where lanes with equal words are contiguous
// (word < 0: no bits).  Returns to the last lane of each run of equal words
// the OR of the run's bits (0 elsewhere) and sets `tail` to the index of the
// last lane of this lane's run.
__device__ __forceinline__ uint64_t run_tail_or(int64_t word, uint64_t bits, int &tail) {
  const int ln = threadIdx.x & 63;
  const int64_t prev = dpp_move<kDppWaveShr1, 0xf>(word ^ 1, word);
  const int64_t next = dpp_move<kDppWaveShl1, 0xf>(word ^ 1, word);
  const bool head = prev != word;
  const bool last = next != word;
  const int rid = wave_max_scan(head ? ln : -1);  // first lane of the run
  const uint64_t x = wave_seg_scan(bits, rid, (uint64_t)0, OpOr());
  const uint64_t tails = __ballot(last);
  tail = __ffsll((unsigned long long)(tails & ~mask_below(ln))) - 1;
  return last ? x : 0ull;
}

// Inclusive min-scan over slots restricted to runs of equal row id.
__device__ __forceinline__ float seg_min_scan(float x, int row) {
  return wave_seg_scan(x, row, __int_as_float(0x7f800000), OpMinF());
}

template <class T>
__device__ __forceinline__ T seg_sum_scan(T x, int row) {
  return wave_seg_scan(x, row, (T)0, OpAdd());
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

// ---- multi-workgroup loops ---------------------------------------------------
// Device-coherent (agent-scope) 32-bit load and store, for what one
// workgroup of a loop hands to another within one kernel.
__device__ __forceinline__ int ld_coherent(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier j of a multi-workgroup loop, called by one thread per workgroup
// after the workgroup's memory operations have completed: one arrival on
// the shared counter, then a wait bounded by wait_ticks of the 100 MHz
// real-time clock.  A workgroup that waits longer gives the barrier up by
// writing j + 1 into the counter's high half, with a compare-and-swap
// against the word it read, so that it cannot give up a barrier the last
// arrival completed in the meantime.  Every workgroup reaches the same
// outcome: 1 when all have arrived, 0 when the barrier was given up (every
// workgroup has then still done its work before barrier j, and all of them
// leave the loop at barrier j).  Arrivals must stay below 2^32.
__device__ __forceinline__ int coop_barrier(unsigned long long *bar, int groups, int64_t j,
                                            uint64_t wait_ticks) {
  const unsigned long long target = (unsigned long long)groups * (unsigned long long)(j + 1);
  const unsigned long long mark = (unsigned long long)(j + 1) << 32;
  __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const unsigned long long w = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((w >> 32) != 0ull) return 0;  // given up (only barrier j can be)
    if ((w & 0xffffffffull) >= target) return 1;
    if (wall_clock64() - t0 >= wait_ticks) {
      unsigned long long e = w;
      if (__hip_atomic_compare_exchange_strong(bar, &e, w | mark, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        return 0;
    } else {
      __builtin_amdgcn_s_sleep(1);
    }
  }
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

// Direction of a generic product (Section 4.3.1, Table 5), evaluated by a
// wave from the first kernel's (count, degree sum) partials, or read from
// the word an earlier kernel of the product left; forced directions and
// single-orientation matrices need neither.  All 64 lanes must be active;
// every lane gets the same answer.
__device__ __forceinline__ int gate_dir(const DirGate &g) {
  if (g.forced) return g.forced;
  if (!g.can_pull) return GRB_DIR_PUSH;
  if (!g.can_push) return GRB_DIR_PULL;
  if (g.decided) {  // left by an earlier kernel of the product
    const int dd = *g.decided;
    if (dd) return dd;
  }
  const int ln = threadIdx.x & 63;
  int64_t c = 0, d = 0;
#pragma unroll
  for (int k = 0; k < kMxvParts / 64; ++k) {
    c += g.part[2 * (k * 64 + ln)];
    d += g.part[2 * (k * 64 + ln) + 1];
  }
  c = wave_sum64(c);
  d = wave_sum64(d);
  const bool pull = g.rule == GRB_SWITCH_EXACT ? (int64_t)g.denom * d > g.nnz
                                               : (int64_t)g.denom * c > g.n_in;
  const int dir = pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
  // every evaluating wave stores the same value; a kernel launched later in
  // the product reads it
  if (g.decided && ln == 0) *g.decided = dir;
  return dir;
}

}  // namespace grb
