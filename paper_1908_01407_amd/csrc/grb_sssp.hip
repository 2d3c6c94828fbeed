// SSSP (Section 7.2 of the paper): Bellman-Ford over the min-plus semiring
// with the frontier sparsified to the vertices whose distance improved in
// the previous round; stop when no distance improves.  One kernel per
// round, like the BFS levels:
// * push: one wave per frontier word streams the frontier rows' out-edges
//   (concatenated, 64 per step) and relaxes dist[v] with an atomicMin on
//   the float's bits (distances are >= 0, so the bit patterns order like
//   the values); rows longer than kPushSplit use the static pieces;
// * pull: one wave per word of candidate rows (rows with in-edges) streams
//   their in-edges and takes a segmented minimum of dist[u] + w(u,v) over
//   frontier neighbours u; a row's owner writes its own distance; rows
//   longer than kHeavyDeg are split into pieces that use atomicMin;
// * every improved vertex sets its bit in the next frontier; the first
//   setter counts it (size and degree sum for the direction choice).
// Relaxations read the current distances in place, so a round may already
// use a distance lowered earlier in the same round; any such order reaches
// the same fixed point, the exact shortest distances.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

__device__ __forceinline__ int decide(const SsspArgs &a, int count, int sumdeg) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

// Marks v improved for the next round; the first marker counts it.
__device__ __forceinline__ void mark_improved(const SsspArgs &a, int v, int &fc, int &fd) {
  const uint64_t b = 1ull << (v & 63);
  if (a.fnxt[v >> 6] & b) return;
  const uint64_t old = atomicOr((unsigned long long *)&a.fnxt[v >> 6], (unsigned long long)b);
  if (old & b) return;
  fc += 1;
  fd += a.push.rp[v + 1] - a.push.rp[v];
}

__device__ __forceinline__ void relax(const SsspArgs &a, int v, float nd, int &fc, int &fd) {
  if (!(nd < a.dist[v])) return;  // plain read: a filter, the atomic decides
  const int old = atomicMin((int *)&a.dist[v], __float_as_int(nd));
  if (nd < __int_as_float(old)) mark_improved(a, v, fc, fd);
}

__device__ void sssp_push(const SsspArgs &a, int *mark, int &fc, int &fd) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    if (ln == 0) a.fclr[w] = 0ull;
    const uint64_t fw = a.fcur[w];
    if (fw == 0ull) continue;
    const int64_t u = w * 64 + ln;
    int cur = 0, end = 0;
    float du = 0.0f;
    if ((fw >> ln) & 1ull) {
      cur = rp[u];
      end = rp[u + 1];
      du = a.dist[u];
      if (end - cur > kPushSplit) end = cur;  // long rows: static pieces below
    }
    for (;;) {
      const int len = end - cur;
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
      const float rdu = __shfl(du, r);
      if (ln < total) {
        const int pos = rcur + (ln - rexcl);
        relax(a, ci[pos], rdu + a.wpush[pos], fc, fd);
      }
      if (starts) cur += min(incl, 64) - excl;
    }
  }
  for (int64_t h0 = gw * 64; h0 < a.push.nsplit; h0 += nwaves * 64) {
    const int64_t h = h0 + ln;
    int u = -1, b = 0;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      b = a.push.split[2 * h + 1];
    }
    uint64_t act = __ballot(u >= 0 && bit_of(a.fcur, u));
    while (act) {
      const int k = __ffsll((unsigned long long)act) - 1;
      act &= act - 1;
      const int pu = __shfl(u, k), pb = __shfl(b, k);
      const float du = a.dist[pu];
      const int e = min(pb + kPushSplit, rp[pu + 1]);
      for (int base = pb; base < e; base += 64) {
        const int pos = base + ln;
        if (pos < e) relax(a, ci[pos], du + a.wpush[pos], fc, fd);
      }
    }
  }
}

__device__ void sssp_pull(const SsspArgs &a, int *mark, int &fc, int &fd) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const float inf = __int_as_float(0x7f800000);
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    if (ln == 0) a.fclr[w] = 0ull;
    const uint64_t cand = ~a.iso[w];
    if (cand == 0ull) continue;
    const int64_t v = w * 64 + ln;
    bool act = (cand >> ln) & 1ull;
    int cur = 0, end = 0;
    if (act) {
      cur = rp[v];
      end = rp[v + 1];
      if (end - cur > kHeavyDeg) act = false;  // long rows: split pieces below
    }
    const int deg0 = end - cur;
    float best = inf;
    for (;;) {
      const int len = act ? end - cur : 0;
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
      float x = inf;
      if (ln < total) {
        const int pos = rcur + (ln - rexcl);
        const int c = ci[pos];
        if (bit_of(a.fcur, c)) x = a.dist[c] + a.wpull[pos];
      }
      x = seg_min_scan(x, r);
      const int se = min(incl, 64);
      const float segmin = __shfl(x, starts ? se - 1 : 0);
      if (starts) {
        best = fminf(best, segmin);
        cur += se - excl;
      }
    }
    bool improved = false;
    if (act && best < a.dist[v]) {
      a.dist[v] = best;
      improved = true;
      fc += 1;
      fd += a.same_csr ? deg0 : a.push.rp[v + 1] - a.push.rp[v];
    }
    const uint64_t ib = __ballot(improved);
    if (ib && ln == 0) atomicOr((unsigned long long *)&a.fnxt[w], (unsigned long long)ib);
  }
  for (int64_t h = gw; h < a.pull.nheavy; h += nwaves) {
    const int r = a.pull.heavy[2 * h], b = a.pull.heavy[2 * h + 1];
    const int e = min(b + kHeavyChunk, rp[r + 1]);
    float best = inf;
    for (int base = b; base < e; base += 64) {
      const int pos = base + ln;
      if (pos < e) {
        const int c = ci[pos];
        if (bit_of(a.fcur, c)) best = fminf(best, a.dist[c] + a.wpull[pos]);
      }
    }
    best = wave_min(best);
    if (ln == 0) relax(a, r, best, fc, fd);
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_round(SsspArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int s_count, s_sumdeg;
  __shared__ int s_red[kWavesPerBlock][2];
  if (threadIdx.x == 0) {
    int c = 0, sd = 0;
    for (int t = 0; t < kCntStripes; ++t) {
      c += a.cnt_cur[2 * t];
      sd += a.cnt_cur[2 * t + 1];
    }
    s_count = c;
    s_sumdeg = sd;
    if (blockIdx.x == 0) {
      for (int i = 0; i < kCntSlots; ++i) a.cnt_clr[i] = 0;
      if (c > 0) {
        a.ctrl->nlev = a.d + 1;
        if (a.stats && a.d < kStatsCap) {
          a.stats[a.d * kStatFields + 0] = c;
          a.stats[a.d * kStatFields + 1] = sd;
          a.stats[a.d * kStatFields + 2] = decide(a, c, sd);
        }
      }
    }
  }
  __syncthreads();
  if (s_count == 0) return;
  const int dir = decide(a, s_count, s_sumdeg);
  int fc = 0, fd = 0;
  if (dir == GRB_DIR_PUSH) sssp_push(a, s_mark[threadIdx.x >> 6], fc, fd);
  else sssp_pull(a, s_mark[threadIdx.x >> 6], fc, fd);
  fc = wave_sum(fc);
  fd = wave_sum(fd);
  if ((threadIdx.x & 63) == 0) {
    s_red[threadIdx.x >> 6][0] = fc;
    s_red[threadIdx.x >> 6][1] = fd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, sd = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      c += s_red[i][0];
      sd += s_red[i][1];
    }
    if (c) {
      const int t = blockIdx.x % kCntStripes;
      atomicAdd(&a.cnt_nxt[2 * t], c);
      atomicAdd(&a.cnt_nxt[2 * t + 1], sd);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_start(SsspArgs a, int32_t source, uint64_t *f1,
                                                       uint64_t *f2) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    bool iso = true;
    if (v < a.n) {
      iso = a.can_pull ? (a.pull.rp[v + 1] == a.pull.rp[v]) : false;
      a.dist[v] = (v == source) ? 0.0f : __int_as_float(0x7f800000);
    }
    const uint64_t isom = __ballot(iso);
    if (ln == 0) {
      a.iso[w] = isom;
      a.fcur[w] = (w == (source >> 6)) ? (1ull << (source & 63)) : 0ull;
      f1[w] = 0ull;
      f2[w] = 0ull;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < kCntSlots; ++i) {
      a.cnt_cur[i] = 0;
      a.cnt_nxt[i] = 0;
      a.cnt_clr[i] = 0;
    }
    a.ctrl->nlev = 0;
    a.cnt_cur[0] = 1;
    a.cnt_cur[1] = a.push.rp[source + 1] - a.push.rp[source];
  }
}

}  // namespace

void launch_sssp_start(const SsspArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                       void *stream) {
  int64_t g = (a.nw + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_sssp_start, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, a,
                     source, f1, f2);
}

void launch_sssp_round(const SsspArgs &a, void *stream) {
  hipLaunchKernelGGL(k_sssp_round, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
