// SSSP (Section 7.2 of the paper): Bellman-Ford over the min-plus semiring
// with the frontier sparsified to the vertices whose distance improved in
// the previous round; stop when no distance improves.  One kernel per
// round, like the BFS levels:
// * push streams the out-edges of the frontier rows and relaxes dist[v]
//   with an atomicMin on the float's bits (distances are >= 0, so the bit
//   patterns order like the values);
// * pull streams the in-edges of every row that has any and takes a
//   segmented minimum of fd[u] + w(u,v), where fd holds the distances of
//   the frontier's vertices and +inf elsewhere (one gather per edge, no
//   bitmap test); the row's wave writes it with a plain store, and pieces
//   of long rows combine their minima with atomicMin;
// * every improved vertex sets its bit in the next frontier and its new
//   distance in the next fd vector (atomicMin); the first setter counts it
//   (size and degree sum for the direction choice).  fd vectors rotate with
//   the bitmaps; a round resets the entries of the buffer it clears.
// Relaxations read the current distances in place, so a round may already
// use a distance lowered earlier in the same round; any such order reaches
// the same fixed point, the exact shortest distances.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

// A pull round probes the frontier bitmap before gathering distances when
// fewer than nnz / kProbeDen edges leave the frontier (the share of the
// gathers the probe can skip; a frontier of hubs is small in vertices but
// not in edges), and loads weights for frontier members only below
// nnz / kSparseDen such edges.
constexpr int64_t kProbeDen = 4;
constexpr int64_t kSparseDen = 32;
enum PullMode { kGatherAll = 0, kProbe = 1, kProbeSparse = 2 };

__device__ __forceinline__ int decide(const SsspArgs &a, int count, int sumdeg) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

// Marks v improved for the next round; the first marker counts it.
__device__ __forceinline__ void mark_improved(const SsspArgs &a, int v, int &fc, int &fd,
                                              int &fl) {
  const uint64_t b = 1ull << (v & 63);
  if (a.fnxt[v >> 6] & b) return;
  const uint64_t old = atomicOr((unsigned long long *)&a.fnxt[v >> 6], (unsigned long long)b);
  if (old & b) return;
  const int pd = a.push.rp[v + 1] - a.push.rp[v];
  fc += 1;
  fd += pd;
  fl += pd > kPushSplit ? 1 : 0;
}

// Relaxes dist[c[s]] with nd[s] for s < kUnroll (c < 0: none).  The
// current distances are read first, all at once (a plain read is only a
// filter, the atomic decides).  Beside each atomic go the loads a success
// needs (the next frontier's word, the target's degree), and the marks of
// all s are issued before any is counted, so a batch waits a fixed number
// of times whatever its wins.
__device__ __forceinline__ void relax_batch(const SsspArgs &a, const int (&c)[kUnroll],
                                            const float (&nd)[kUnroll], int &fc, int &fd,
                                            int &fl) {
  float cd[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) cd[s] = c[s] >= 0 ? a.dist[c[s]] : 0.0f;
  int old[kUnroll], r0[kUnroll], r1[kUnroll];
  uint64_t w[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    old[s] = 0;
    r0[s] = r1[s] = 0;
    w[s] = ~0ull;
    if (c[s] >= 0 && nd[s] < cd[s]) {
      old[s] = atomicMin((int *)&a.dist[c[s]], __float_as_int(nd[s]));
      w[s] = a.fnxt[c[s] >> 6];
      r0[s] = a.push.rp[c[s]];
      r1[s] = a.push.rp[c[s] + 1];
    }
  }
  uint64_t o[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    o[s] = ~0ull;
    if (c[s] >= 0 && nd[s] < cd[s] && nd[s] < __int_as_float(old[s])) {
      atomicMin((int *)&a.fd_nxt[c[s]], __float_as_int(nd[s]));
      const uint64_t b = 1ull << (c[s] & 63);
      if (!(w[s] & b))
        o[s] = atomicOr((unsigned long long *)&a.fnxt[c[s] >> 6], (unsigned long long)b);
    }
  }
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    if (c[s] >= 0 && !(o[s] & (1ull << (c[s] & 63)))) {
      const int pd = r1[s] - r0[s];
      fc += 1;
      fd += pd;
      fl += pd > kPushSplit ? 1 : 0;
    }
  }
}

// Bitmap words are dealt out to the waves round-robin.  Push compacts the
// frontier bits of a wave's words into a queue of rows, pull takes the
// candidate rows one word at a time (lanes = the word's 64 rows).  Rows up
// to kPushSplit edges long are streamed by the wave as one concatenated
// list, kUnroll x 64 edges per step; longer rows come in static
// kPushSplit-edge pieces spread over all waves (both directions), so no
// wave is left with a hub.

// Clears the frontier bitmap two rounds ahead, word `mw` per lane, and
// resets the frontier distances of its vertices to +inf (coalesced: the
// wave writes one word's 64 entries at a time).
__device__ __forceinline__ void clear_behind(const SsspArgs &a, int64_t mw, bool valid) {
  const int ln = threadIdx.x & 63;
  uint64_t old = 0ull;
  if (valid) {
    old = a.fclr[mw];
    if (old) a.fclr[mw] = 0ull;
  }
  uint64_t nz = __ballot(old != 0ull);
  const float inf = __int_as_float(0x7f800000);
  while (nz) {
    const int k = __ffsll((unsigned long long)nz) - 1;
    nz &= nz - 1;
    const int64_t w = __shfl(mw, k);
    const uint64_t bits = __shfl(old, k);
    if ((bits >> ln) & 1ull) a.fd_clr[w * 64 + ln] = inf;
  }
}

__device__ void sssp_push(const SsspArgs &a, int *mark, bool long_rows, int &fc, int &fd,
                          int &fl) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  // words dealt out round-robin (wave gw takes words gw, gw + nwaves, ...);
  // their set bits are compacted into a queue of rows, 64 at a time
  for (int64_t w0 = gw; w0 < a.nw; w0 += 64 * nwaves) {
    const int64_t mw = w0 + (int64_t)ln * nwaves;
    clear_behind(a, mw, mw < a.nw);
    const uint64_t mf = mw < a.nw ? a.fcur[mw] : 0ull;
    const int cnt = __popcll(mf);
    const int qincl = wave_incl_scan(cnt);
    const int qtotal = lane_last(qincl);
    for (int b = 0; b < qtotal; b += 64) {
      const int64_t u = queue_slot(mark, mf, cnt, qincl, qtotal, b, mw);
      int cur = 0, end = 0;
      float du = 0.0f;
      if (u >= 0) {
        cur = rp[u];
        end = rp[u + 1];
        du = a.dist[u];
        if (end - cur > kPushSplit) end = cur;  // long rows: static pieces below
      }
      for (bool more = true; more;) {
        int cc[kUnroll];
        float nd[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          cc[s] = -1;
          nd[s] = 0.0f;
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
          const float rdu = __shfl(du, r);
          if (ln < total) {
            cc[s] = rcur + (ln - rexcl);
            nd[s] = rdu;
          }
          if (starts) cur += min(incl, 64) - excl;
        }
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          if (cc[s] >= 0) {
            const int pos = cc[s];
            cc[s] = ci[pos];
            nd[s] += a.wpush[pos];
          }
        }
        relax_batch(a, cc, nd, fc, fd, fl);
      }
    }
  }
  // static pieces of long rows, spread over the waves, 64 tested per step
  static_assert(kPushSplit == 64 * kUnroll, "a piece is one unrolled step");
  if (!long_rows) return;  // no row of the frontier has pieces
  for (int64_t hb = gw; hb < a.push.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int u = -1, b = 0, e = 0;
    float du = 0.0f;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      b = a.push.split[2 * h + 1];
      if (bit_of(a.fcur, u)) {
        e = min(b + kPushSplit, rp[u + 1]);
        du = a.dist[u];
      } else {
        u = -1;
      }
    }
    uint64_t act = __ballot(u >= 0);
    while (act) {
      const int k = __ffsll((unsigned long long)act) - 1;
      act &= act - 1;
      const int pb = __shfl(b, k), pe = __shfl(e, k);
      const float pdu = __shfl(du, k);
      int cc[kUnroll];
      float nd[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int pos = pb + s * 64 + ln;
        cc[s] = pos < pe ? ci[pos] : -1;
        nd[s] = pos < pe ? pdu + a.wpush[pos] : 0.0f;
      }
      relax_batch(a, cc, nd, fc, fd, fl);
    }
  }
}

// Pull-round candidate distances fd(c) + w(pos) of the stream positions pos
// (pos < 0: none) with column ids c (+inf off the frontier).  kGatherAll:
// the weights load with the ids and every id's distance is gathered (the
// fewest dependent loads: for frontiers that most edges leave).  kProbe:
// each id's frontier bit is read first (the bitmap is n/8 bytes and stays
// in cache) and only frontier members gather their distance.  kProbeSparse:
// as kProbe, and only members load their weight, beside the distance.
template <int K>
__device__ __forceinline__ void pull_terms(const SsspArgs &a, const int (&pos)[K], int mode,
                                           float (&t)[K]) {
  const float inf = __int_as_float(0x7f800000);
  int c[K];
  float w[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    c[s] = pos[s] >= 0 ? a.pull.ci[pos[s]] : -1;
    w[s] = (mode != kProbeSparse && pos[s] >= 0) ? a.wpull[pos[s]] : 0.0f;
  }
  if (mode == kGatherAll) {
#pragma unroll
    for (int s = 0; s < K; ++s) t[s] = (c[s] >= 0 ? a.fd_cur[c[s]] : inf) + w[s];
    return;
  }
  uint64_t fb[K];
#pragma unroll
  for (int s = 0; s < K; ++s) fb[s] = c[s] >= 0 ? a.fcur[c[s] >> 6] : 0ull;
  float d[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const bool in = c[s] >= 0 && ((fb[s] >> (c[s] & 63)) & 1ull);
    d[s] = in ? a.fd_cur[c[s]] : inf;
    if (mode == kProbeSparse && in) w[s] = a.wpull[pos[s]];
  }
#pragma unroll
  for (int s = 0; s < K; ++s) t[s] = d[s] + w[s];
}

__device__ void sssp_pull(const SsspArgs &a, int *mark, int mode, int &fc, int &fd, int &fl) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp;
  const float inf = __int_as_float(0x7f800000);
  // the wave's run of words (runs of about equal work, built by
  // grb_matrix_prepare: rows of similar degree have nearby ids)
  for (int64_t part = gw; part < kWaveParts; part += nwaves) {
    const int64_t wlo = a.pull.wpart[part], whi = a.pull.wpart[part + 1];
    for (int64_t w0 = wlo; w0 < whi; w0 += 64) {
      const int64_t mw = w0 + ln;
      clear_behind(a, mw, mw < whi);
      const uint64_t mc = mw < whi ? ~a.iso[mw] : 0ull;  // candidate rows: rows with in-edges
      uint64_t nzw = __ballot(mc != 0ull);
      while (nzw) {
        const int k = __ffsll((unsigned long long)nzw) - 1;
        nzw &= nzw - 1;
        const int64_t w = w0 + k;
        const uint64_t cand = __shfl(mc, k);
        const int64_t v = w * 64 + ln;
        bool act = (cand >> ln) & 1ull;
        int cur = 0, end = 0;
        if (act) {
          cur = rp[v];
          end = rp[v + 1];
          if (end - cur > kPushSplit) act = false;  // long rows: pieces below
        }
        if (!act) end = cur;
        const int deg0 = end - cur;
        float best = inf;
        // slot positions of kUnroll x 64 edges first, then their loads, then
        // the segmented minima over frontier neighbours (off the frontier a
        // candidate is +inf)
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
          float tv[kUnroll];
          pull_terms(a, pos, mode, tv);
  #pragma unroll
          for (int s = 0; s < kUnroll; ++s) {
            const float y = seg_min_scan(tv[s], row[s]);
            const float segmin = __shfl(y, st[s] ? se[s] - 1 : 0);
            if (st[s]) best = fminf(best, segmin);
          }
        }
        bool improved = false;
        if (act && best < a.dist[v]) {  // only this wave writes row v in a pull round
          a.dist[v] = best;
          a.fd_nxt[v] = best;
          improved = true;
          const int pd = a.same_csr ? deg0 : a.push.rp[v + 1] - a.push.rp[v];
          fc += 1;
          fd += pd;
          fl += pd > kPushSplit ? 1 : 0;
        }
        const uint64_t ib = __ballot(improved);
        if (ib && ln == 0) atomicOr((unsigned long long *)&a.fnxt[w], (unsigned long long)ib);
      }
    }
  }
  // pieces of long rows: each piece's minimum is combined with atomicMin;
  // two active pieces are loaded at once so their latencies overlap
  for (int64_t hb = gw; hb < a.pull.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int r = -1, b = 0, e = 0;
    if (h < a.pull.nsplit) {
      r = a.pull.split[2 * h];
      b = a.pull.split[2 * h + 1];
      e = min(b + kPushSplit, rp[r + 1]);
    }
    uint64_t act = __ballot(r >= 0);
    while (act) {
      int pr[2], pb[2], pe[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        pr[q] = -1;
        pb[q] = pe[q] = 0;
        if (act) {
          const int k = __ffsll((unsigned long long)act) - 1;
          act &= act - 1;
          pr[q] = __shfl(r, k);
          pb[q] = __shfl(b, k);
          pe[q] = __shfl(e, k);
        }
      }
      int pos[2][kUnroll];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          const int ps = pb[q] + s * 64 + ln;
          pos[q][s] = ps < pe[q] ? ps : -1;
        }
      float tv[2][kUnroll];
#pragma unroll
      for (int q = 0; q < 2; ++q) pull_terms(a, pos[q], mode, tv[q]);
      float best[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        best[q] = inf;
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) best[q] = fminf(best[q], tv[q][s]);
      }
      best[0] = wave_min(best[0]);
      best[1] = wave_min(best[1]);
      // lane q relaxes piece q's row
      const int myr = ln == 0 ? pr[0] : (ln == 1 ? pr[1] : -1);
      const float myb = ln == 0 ? best[0] : best[1];
      if (myr >= 0 && myb < inf) {
        const int old = atomicMin((int *)&a.dist[myr], __float_as_int(myb));
        if (myb < __int_as_float(old)) {
          atomicMin((int *)&a.fd_nxt[myr], __float_as_int(myb));
          mark_improved(a, myr, fc, fd, fl);
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_round(SsspArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int s_count, s_sumdeg, s_long;
  __shared__ int s_red[kWavesPerBlock][kCntFields];
  if (threadIdx.x == 0) {
    int c = 0, sd = 0, lr = 0;
    for (int t = 0; t < kCntStripes; ++t) {
      c += a.cnt_cur[kCntFields * t];
      sd += a.cnt_cur[kCntFields * t + 1];
      lr += a.cnt_cur[kCntFields * t + 2];
    }
    s_count = c;
    s_sumdeg = sd;
    s_long = lr;
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
  int fc = 0, fd = 0, fl = 0;
  if (dir == GRB_DIR_PUSH) sssp_push(a, s_mark[threadIdx.x >> 6], s_long > 0, fc, fd, fl);
  else {
    const int64_t e = s_sumdeg;  // edges that leave the frontier
    const int mode = e * kSparseDen < a.nnz ? kProbeSparse
                     : e * kProbeDen < a.nnz ? kProbe : kGatherAll;
    sssp_pull(a, s_mark[threadIdx.x >> 6], mode, fc, fd, fl);
  }
  fc = wave_sum(fc);
  fd = wave_sum(fd);
  fl = wave_sum(fl);
  if ((threadIdx.x & 63) == 0) {
    s_red[threadIdx.x >> 6][0] = fc;
    s_red[threadIdx.x >> 6][1] = fd;
    s_red[threadIdx.x >> 6][2] = fl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, sd = 0, lr = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      c += s_red[i][0];
      sd += s_red[i][1];
      lr += s_red[i][2];
    }
    if (c) {
      const int t = blockIdx.x % kCntStripes;
      atomicAdd(&a.cnt_nxt[kCntFields * t], c);
      atomicAdd(&a.cnt_nxt[kCntFields * t + 1], sd);
      if (lr) atomicAdd(&a.cnt_nxt[kCntFields * t + 2], lr);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_start(SsspArgs a, int32_t source, uint64_t *f1,
                                                       uint64_t *f2, float *fd1, float *fd2) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    bool iso = true;
    if (v < a.n) {
      iso = a.can_pull ? (a.pull.rp[v + 1] == a.pull.rp[v]) : false;
      const float inf = __int_as_float(0x7f800000);
      a.dist[v] = (v == source) ? 0.0f : inf;
      a.fd_cur[v] = (v == source) ? 0.0f : inf;
      fd1[v] = inf;
      fd2[v] = inf;
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
    const int ds = a.push.rp[source + 1] - a.push.rp[source];
    a.cnt_cur[0] = 1;
    a.cnt_cur[1] = ds;
    a.cnt_cur[2] = ds > kPushSplit ? 1 : 0;
  }
}

}  // namespace

void launch_sssp_start(const SsspArgs &a, int32_t source, uint64_t *f1, uint64_t *f2, float *fd1,
                       float *fd2, void *stream) {
  int64_t g = (a.nw + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_sssp_start, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, a,
                     source, f1, f2, fd1, fd2);
}

void launch_sssp_round(const SsspArgs &a, void *stream) {
  hipLaunchKernelGGL(k_sssp_round, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
