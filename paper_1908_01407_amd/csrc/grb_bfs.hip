// Direction-optimised BFS (Algorithm 1 and Section 7.1 of the paper) with
// one kernel per level.
//
// Each level is f <- A^T f .* not(visited) over the Boolean semiring, run as
// push (SpMSpV from the frontier's out-edges) or pull (masked SpMV over the
// unvisited rows, stopping a row at its first frontier neighbour), chosen on
// the device from the frontier's size and degree sum (the switch rule of the
// descriptor).  The frontier is only a bitmap, and one kernel does all of a
// level, so nothing sits between levels:
// * push gives each wave one frontier word and streams the out-edges of its
//   frontier rows as one concatenated list, 64 edges per step (the same
//   wave-level load-balanced search as pull); rows longer than kPushSplit
//   come from a static list of kPushSplit-edge pieces built by
//   grb_matrix_prepare, each piece active when its row is in the frontier;
// * a vertex is claimed by the first atomicOr on its visited bit; the
//   claimer writes its level and sets its bit in the next frontier bitmap;
// * the next frontier's size and degree sum are reduced per workgroup and
//   added into kCntStripes striped counters (few atomics per address);
// * bitmaps and counters rotate through three buffers: the level reads
//   buffer d, fills buffer d+1 and clears buffer d+2.
// Pull finds the smallest-id parent directly (ascending adjacency, first
// hit).  Push-discovered vertices get theirs from one pass after the last
// level: the first in-neighbour one level up in ascending order.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

__device__ __forceinline__ int decide(const BfsArgs &a, int count, int sumdeg) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

// Claims v (v < 0: nothing) for the next level; counts it in (fc, fd).
__device__ __forceinline__ void claim(const BfsArgs &a, int v, int &fc, int &fd) {
  if (v < 0 || bit_of(a.visited, v)) return;  // plain read: a filter, the atomic decides
  const uint64_t b = 1ull << (v & 63);
  const uint64_t old = atomicOr((unsigned long long *)&a.visited[v >> 6], (unsigned long long)b);
  if (old & b) return;
  a.levels[v] = a.d + 1;
  atomicOr((unsigned long long *)&a.fnxt[v >> 6], (unsigned long long)b);
  fc += 1;
  fd += a.push.rp[v + 1] - a.push.rp[v];
}

__device__ void bfs_push(const BfsArgs &a, int *mark, int &fc, int &fd) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    if (ln == 0) a.fclr[w] = 0ull;  // the bitmap two levels ahead
    const uint64_t fw = a.fcur[w];
    if (fw == 0ull) continue;
    const int64_t u = w * 64 + ln;
    int cur = 0, end = 0;
    if ((fw >> ln) & 1ull) {
      cur = rp[u];
      end = rp[u + 1];
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
      claim(a, ln < total ? ci[rcur + (ln - rexcl)] : -1, fc, fd);
      if (starts) cur += min(incl, 64) - excl;
    }
  }
  // static pieces of long rows: 64 pieces tested per step (one per lane),
  // then the wave streams the pieces whose row is in the frontier
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
      const int e = min(pb + kPushSplit, rp[pu + 1]);
      for (int base = pb; base < e; base += 64) {
        const int pos = base + ln;
        claim(a, pos < e ? ci[pos] : -1, fc, fd);
      }
    }
  }
}

__device__ void bfs_pull(const BfsArgs &a, int *mark, int &fc, int &fd) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    if (ln == 0) a.fclr[w] = 0ull;
    const uint64_t cand = ~a.visited[w];
    if (cand == 0ull) continue;
    const int64_t v = w * 64 + ln;
    bool act = (cand >> ln) & 1ull;
    int cur = 0, end = 0;
    if (act) {
      cur = rp[v];
      end = rp[v + 1];
      if (end - cur > kHeavyDeg) act = false;  // long rows: split pieces below
    }
    const int deg0 = end - cur;  // push degree when both orientations share one CSR
    bool found = false;
    int par = -1;
    if (act) {  // the first two neighbours of every row, in parallel
      const int c0 = cur < end ? ci[cur] : -1;
      const int c1 = cur + 1 < end ? ci[cur + 1] : -1;
      if (c0 >= 0 && bit_of(a.fcur, c0)) { found = true; par = c0; }
      else if (c1 >= 0 && bit_of(a.fcur, c1)) { found = true; par = c1; }
      cur = min(cur + 2, end);
    }
    for (;;) {  // the rest as one concatenated stream, 64 edges per step
      const int len = (act && !found) ? end - cur : 0;
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
      const bool valid = ln < total;
      const int c = valid ? ci[rcur + (ln - rexcl)] : -1;
      const uint64_t hm = __ballot(valid && bit_of(a.fcur, c));
      const int se = min(incl, 64);
      const uint64_t seg = starts ? (mask_below(se) & ~mask_below(excl)) : 0ull;
      const uint64_t h = hm & seg;
      const int fl = h ? (__ffsll((unsigned long long)h) - 1) : 0;
      const int pc = __shfl(c, fl);
      if (h) { found = true; par = pc; }
      if (starts) cur += se - excl;
    }
    const uint64_t fbits = __ballot(found);
    if (fbits == 0ull) continue;
    if (ln == 0) {
      atomicOr((unsigned long long *)&a.visited[w], (unsigned long long)fbits);
      atomicOr((unsigned long long *)&a.fnxt[w], (unsigned long long)fbits);
    }
    if (found) {
      a.levels[v] = a.d + 1;
      if (a.parents) a.parents[v] = par;
      fc += 1;
      fd += a.same_csr ? deg0 : a.push.rp[v + 1] - a.push.rp[v];
    }
  }
  // pieces of long rows; a row counts as a candidate unless it was reached
  // before this level (its level is then 0..d)
  for (int64_t h = gw; h < a.pull.nheavy; h += nwaves) {
    const int r = a.pull.heavy[2 * h], b = a.pull.heavy[2 * h + 1];
    const int lr = a.levels[r];
    if (lr >= 0 && lr <= a.d) continue;
    const int e = min(b + kHeavyChunk, rp[r + 1]);
    for (int base = b; base < e; base += 64) {
      const int pos = base + ln;
      const int c = pos < e ? ci[pos] : -1;
      const uint64_t hm = __ballot(c >= 0 && bit_of(a.fcur, c));
      if (hm) {
        const int pc = __shfl(c, __ffsll((unsigned long long)hm) - 1);
        if (ln == 0) {
          const uint64_t bit = 1ull << (r & 63);
          const uint64_t old =
              atomicOr((unsigned long long *)&a.visited[r >> 6], (unsigned long long)bit);
          if (a.parents) atomicMin((unsigned *)&a.parents[r], (unsigned)pc);
          if (!(old & bit)) {
            a.levels[r] = a.d + 1;
            atomicOr((unsigned long long *)&a.fnxt[r >> 6], (unsigned long long)bit);
            fc += 1;
            fd += a.push.rp[r + 1] - a.push.rp[r];
          }
        }
        break;
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_bfs_level(BfsArgs a) {
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
      // the buffer two levels ahead is cleared even when this level is
      // empty: it still holds the counts of the previous level
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
  const int count = s_count;
  if (count == 0) return;
  const int dir = decide(a, count, s_sumdeg);
  int fc = 0, fd = 0;
  if (dir == GRB_DIR_PUSH) bfs_push(a, s_mark[threadIdx.x >> 6], fc, fd);
  else bfs_pull(a, s_mark[threadIdx.x >> 6], fc, fd);
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

__global__ __launch_bounds__(kBlock) void k_bfs_start(BfsArgs a, int32_t source, uint64_t *f1,
                                                      uint64_t *f2) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    bool iso = true;
    if (v < a.n) {
      // no in-edges: a pull can never reach it (a push cannot either)
      iso = a.can_pull ? (a.pull.rp[v + 1] == a.pull.rp[v]) : false;
      a.levels[v] = (v == source) ? 0 : -1;
      if (a.parents) a.parents[v] = (v == source) ? source : -1;
    }
    const uint64_t isom = __ballot(iso || v == source);
    if (ln == 0) {
      a.visited[w] = isom;
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
    a.cnt_cur[0] = 1;  // level 0 = {source}
    a.cnt_cur[1] = a.push.rp[source + 1] - a.push.rp[source];
  }
}

// Smallest-id parent of every vertex reached by a push: the first
// in-neighbour (ascending) whose level is one less.
__global__ __launch_bounds__(kBlock) void k_bfs_parents(BfsArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  int *mark = s_mark[threadIdx.x >> 6];
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    int lv = -1;
    bool need = false;
    if (v < a.n) {
      lv = a.levels[v];
      need = lv > 0 && a.parents[v] < 0;
    }
    if (__ballot(need) == 0ull) continue;
    int cur = need ? rp[v] : 0, end = need ? rp[v + 1] : 0;
    const int tgt = lv - 1;
    bool found = false;
    int par = -1;
    for (;;) {
      const int len = (need && !found) ? end - cur : 0;
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r), rt = __shfl(tgt, r);
      const bool valid = ln < total;
      const int c = valid ? ci[rcur + (ln - rexcl)] : -1;
      const uint64_t hm = __ballot(valid && a.levels[c] == rt);
      const int se = min(incl, 64);
      const uint64_t seg = starts ? (mask_below(se) & ~mask_below(excl)) : 0ull;
      const uint64_t h = hm & seg;
      const int fl = h ? (__ffsll((unsigned long long)h) - 1) : 0;
      const int pc = __shfl(c, fl);
      if (h) { found = true; par = pc; }
      if (starts) cur += se - excl;
    }
    if (found) a.parents[v] = par;
  }
}

}  // namespace

void launch_bfs_start(const BfsArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                      void *stream) {
  int64_t g = (a.nw + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_bfs_start, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, a,
                     source, f1, f2);
}

void launch_bfs_level(const BfsArgs &a, void *stream) {
  hipLaunchKernelGGL(k_bfs_level, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

void launch_bfs_parents(const BfsArgs &a, void *stream) {
  hipLaunchKernelGGL(k_bfs_parents, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
