// Bucketed SSSP: the min-plus relaxation of Section 7.2 of the paper
// processed in distance order, a near-far form of delta-stepping.  The
// paper's Bellman-Ford rounds relax every improved vertex at once, which on
// high-diameter graphs (road networks, grids) relaxes each edge over a
// hundred times; here a round relaxes only the pending vertices whose
// distance lies below the current bucket's limit (B + 1) * delta, and the
// others wait in the pending set.  The bucket advances to the smallest
// pending bucket once no vertex is left below the limit.  Any order of
// relaxations reaches the same fixed point, so the distances are the exact
// shortest distances, identical to the Bellman-Ford rounds.
//
// One kernel per round, like the BFS levels and the Bellman-Ford rounds:
// * pending sets are bitmaps rotating through three buffers (read d, fill
//   d + 1, clear d + 2); each wave compacts the set bits of its words into a
//   queue of rows;
// * a queued row below the limit is relaxed (push, atomicMin on the float
//   bits) and leaves the set unless it improves again; a row above it is
//   carried into the next set;
// * the first setter of a bit counts the new member: near (below the
//   limit: size, degree sum, rows with pieces) or far (the smallest far
//   bucket), plus the pending total, all in striped counters.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

struct DCount {
  int near = 0, sd = 0, lng = 0, far = INT_MAX, pend = 0;
};

__device__ __forceinline__ int bucket_of(float d, float delta) { return (int)(d / delta); }

// Counts a new member of the next pending set with distance nd and out-
// degree pd.
__device__ __forceinline__ void count_new(const SsspArgs &a, int pd, float nd, float limit,
                                          DCount &c) {
  c.pend += 1;
  if (nd < limit) {
    c.near += 1;
    c.sd += pd;
    c.lng += pd > kPushSplit ? 1 : 0;
  } else {
    c.far = min(c.far, bucket_of(nd, a.delta));
  }
}

// Relaxes dist[c[s]] with nd[s] (c < 0: none); all reads, then all atomics,
// each beside the loads its success needs (the pending set's word, the
// target's degree), then all marks, then the counts.
__device__ __forceinline__ void relax_near(const SsspArgs &a, const int (&c)[kUnroll],
                                           const float (&nd)[kUnroll], float limit, DCount &cnt) {
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
      const uint64_t b = 1ull << (c[s] & 63);
      if (!(w[s] & b))
        o[s] = atomicOr((unsigned long long *)&a.fnxt[c[s] >> 6], (unsigned long long)b);
    }
  }
#pragma unroll
  for (int s = 0; s < kUnroll; ++s)
    if (c[s] >= 0 && !(o[s] & (1ull << (c[s] & 63)))) count_new(a, r1[s] - r0[s], nd[s], limit, cnt);
}

__device__ void delta_push(const SsspArgs &a, int *mark, float limit, bool pieces, DCount &cnt) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  for (int64_t w0 = gw; w0 < a.nw; w0 += 64 * nwaves) {
    const int64_t mw = w0 + (int64_t)ln * nwaves;
    uint64_t mf = 0ull;
    if (mw < a.nw) {
      a.fclr[mw] = 0ull;  // the set two rounds ahead
      mf = a.fcur[mw];
    }
    const int qc = __popcll(mf);
    const int qincl = wave_incl_scan(qc);
    const int qtotal = lane_last(qincl);
    for (int b = 0; b < qtotal; b += 64) {
      const int64_t u = queue_slot(mark, mf, qc, qincl, qtotal, b, mw);
      const float du = u >= 0 ? a.dist[u] : 0.0f;
      const bool active = u >= 0 && du < limit;
      // rows above the limit stay pending: one atomicOr per word (queued
      // rows are ascending), each lane then learns whether it was first
      const bool carry = u >= 0 && !active;
      const int64_t cw = carry ? (u >> 6) : -1;
      int tail;
      const uint64_t run = run_tail_or(cw, carry ? (1ull << (u & 63)) : 0ull, tail);
      uint64_t oldw = 0ull;
      if (run && cw >= 0) oldw = atomicOr((unsigned long long *)&a.fnxt[cw], (unsigned long long)run);
      oldw = __shfl(oldw, tail);
      if (carry && !((oldw >> (u & 63)) & 1ull)) {
        cnt.pend += 1;
        cnt.far = min(cnt.far, bucket_of(du, a.delta));
      }
      int cur = 0, end = 0;
      if (active) {
        cur = rp[u];
        end = rp[u + 1];
        if (end - cur > kPushSplit) end = cur;  // long rows: pieces below
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
        relax_near(a, cc, nd, limit, cnt);
      }
    }
  }
  if (!pieces) return;
  // pieces of long rows below the limit, spread over the waves
  static_assert(kPushSplit == 64 * kUnroll, "a piece is one unrolled step");
  for (int64_t hb = gw; hb < a.push.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int u = -1, pbeg = 0, pend = 0;
    float du = 0.0f;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      pbeg = a.push.split[2 * h + 1];
      if (bit_of(a.fcur, u)) {
        du = a.dist[u];
        if (du < limit) pend = min(pbeg + kPushSplit, rp[u + 1]);
        else u = -1;
      } else {
        u = -1;
      }
    }
    uint64_t act = __ballot(u >= 0);
    while (act) {
      const int k = __ffsll((unsigned long long)act) - 1;
      act &= act - 1;
      const int pb = __shfl(pbeg, k), pe = __shfl(pend, k);
      const float pdu = __shfl(du, k);
      int cc[kUnroll];
      float nd[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int pos = pb + s * 64 + ln;
        cc[s] = pos < pe ? ci[pos] : -1;
        nd[s] = pos < pe ? pdu + a.wpush[pos] : 0.0f;
      }
      relax_near(a, cc, nd, limit, cnt);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_delta_round(SsspArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int s_bucket, s_pend, s_pieces;
  __shared__ int s_red[kWavesPerBlock][kDeltaFields];
  if (threadIdx.x == 0) {
    int nr = 0, sd = 0, lg = 0, far = INT_MAX, pend = 0;
    for (int t = 0; t < kCntStripes; ++t) {
      nr += a.cnt_cur[kDeltaFields * t];
      sd += a.cnt_cur[kDeltaFields * t + 1];
      lg += a.cnt_cur[kDeltaFields * t + 2];
      far = min(far, a.cnt_cur[kDeltaFields * t + 3]);
      pend += a.cnt_cur[kDeltaFields * t + 4];
    }
    // stay in the bucket while it has members, else move to the nearest
    // pending bucket
    const int bucket = nr > 0 ? a.ctrl->bucket : far;
    s_bucket = bucket;
    s_pend = pend;
    // a row below the limit may be long although no long row was counted
    // near (its distance can drop after its first insertion), so the pieces
    // are skipped only when the graph has none
    s_pieces = a.push.nsplit > 0 ? 1 : 0;
    if (blockIdx.x == 0) {
      for (int t = 0; t < kCntStripes; ++t) {
        for (int f = 0; f < kDeltaFields; ++f)
          a.cnt_clr[kDeltaFields * t + f] = f == 3 ? INT_MAX : 0;
      }
      if (pend > 0) {
        a.ctrl->nlev = a.d + 1;
        a.ctrl->bucket = bucket;
        if (a.stats && a.d < kStatsCap) {
          a.stats[a.d * kStatFields + 0] = pend;
          a.stats[a.d * kStatFields + 1] = sd;
          a.stats[a.d * kStatFields + 2] = GRB_DIR_PUSH;
          a.stats[a.d * kStatFields + 3] = bucket;
        }
      }
    }
  }
  __syncthreads();
  if (s_pend == 0) return;
  const float limit = (float)(s_bucket + 1) * a.delta;
  DCount c;
  delta_push(a, s_mark[threadIdx.x >> 6], limit, s_pieces != 0, c);
  c.near = wave_sum(c.near);
  c.sd = wave_sum(c.sd);
  c.lng = wave_sum(c.lng);
  c.pend = wave_sum(c.pend);
  c.far = lane_last(wave_scan(c.far, INT_MAX, [](int x, int y) { return x < y ? x : y; }));
  if ((threadIdx.x & 63) == 0) {
    const int wv = threadIdx.x >> 6;
    s_red[wv][0] = c.near;
    s_red[wv][1] = c.sd;
    s_red[wv][2] = c.lng;
    s_red[wv][3] = c.far;
    s_red[wv][4] = c.pend;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0, sd = 0, lg = 0, far = INT_MAX, pend = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      nr += s_red[i][0];
      sd += s_red[i][1];
      lg += s_red[i][2];
      far = min(far, s_red[i][3]);
      pend += s_red[i][4];
    }
    if (pend) {
      const int t = blockIdx.x % kCntStripes;
      if (nr) {
        atomicAdd(&a.cnt_nxt[kDeltaFields * t], nr);
        atomicAdd(&a.cnt_nxt[kDeltaFields * t + 1], sd);
        if (lg) atomicAdd(&a.cnt_nxt[kDeltaFields * t + 2], lg);
      }
      if (far != INT_MAX) atomicMin(&a.cnt_nxt[kDeltaFields * t + 3], far);
      atomicAdd(&a.cnt_nxt[kDeltaFields * t + 4], pend);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_delta_start(SsspArgs a, int32_t source,
                                                             uint64_t *f1, uint64_t *f2) {
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int ln = threadIdx.x & 63;
  const float inf = __int_as_float(0x7f800000);
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    if (v < a.n) a.dist[v] = (v == source) ? 0.0f : inf;
    if (ln == 0) {
      a.fcur[w] = (w == (source >> 6)) ? (1ull << (source & 63)) : 0ull;
      f1[w] = 0ull;
      f2[w] = 0ull;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < kDeltaSlots; ++i) {
      const int v = (i % kDeltaFields) == 3 ? INT_MAX : 0;
      a.cnt_cur[i] = v;
      a.cnt_nxt[i] = v;
      a.cnt_clr[i] = v;
    }
    const int ds = a.push.rp[source + 1] - a.push.rp[source];
    a.cnt_cur[0] = 1;  // the source: near in bucket 0, pending
    a.cnt_cur[1] = ds;
    a.cnt_cur[2] = ds > kPushSplit ? 1 : 0;
    a.cnt_cur[4] = 1;
    a.ctrl->nlev = 0;
    a.ctrl->bucket = 0;
  }
}

}  // namespace

void launch_sssp_delta_start(const SsspArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                             void *stream) {
  int64_t g = (a.nw + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_sssp_delta_start, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream,
                     a, source, f1, f2);
}

void launch_sssp_delta_round(const SsspArgs &a, void *stream) {
  hipLaunchKernelGGL(k_sssp_delta_round, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream,
                     a);
}

}  // namespace grb
