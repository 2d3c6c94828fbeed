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

// ---- one-workgroup bucket rounds while the pending set is small -----------
// The pending set as two LDS lists (consumed / filled: vertex, row start,
// degree) with membership bits in two bitmaps (F0, F1), so a vertex joins
// the filled list once per round.  A round: each thread takes entries of the
// consumed list, clears their bits, reads their distance together with
// their first out-edges; an entry below the bucket's limit relaxes its edges
// (atomicMin on the float bits, the target's row extents loaded beside it)
// and every improved target joins the filled list; an entry above the limit
// is carried.  The bucket moves to the nearest pending one when no member
// below the limit is left.  A pending set too large for the lists goes to
// the wide round kernel as its bitmap and counters.
__device__ __forceinline__ void small_insert(bool want, int x, int rs, int dg, float dx, float limit,
                                             float delta, uint64_t *fill, int (*s_v)[kSmallCap],
                                             int (*s_rs)[kSmallCap], int (*s_dg)[kSmallCap],
                                             int *s_n, int *s_near, int *s_sd, int *s_lng,
                                             int *s_far, int nb) {
  const int ln = threadIdx.x & 63;
  bool first = false;
  if (want) {
    const uint64_t bit = 1ull << (x & 63);
    first = !(atomicOr((unsigned long long *)&fill[x >> 6], (unsigned long long)bit) & bit);
  }
  const uint64_t fm = __ballot(first);
  if (fm == 0ull) return;
  int base = 0;
  if (ln == 0) base = atomicAdd(&s_n[nb], __popcll(fm));
  base = __shfl(base, 0);
  const bool nr = first && dx < limit;
  const int c_near = wave_sum(nr ? 1 : 0), c_sd = wave_sum(nr ? dg : 0);
  const int c_lng = wave_sum(nr && dg > kPushSplit ? 1 : 0);
  int far = (first && !nr) ? bucket_of(dx, delta) : INT_MAX;
  far = lane_last(wave_scan(far, INT_MAX, [](int p, int q) { return p < q ? p : q; }));
  if (ln == 0) {
    if (c_near) {
      atomicAdd(&s_near[nb], c_near);
      atomicAdd(&s_sd[nb], c_sd);
      if (c_lng) atomicAdd(&s_lng[nb], c_lng);
    }
    if (far != INT_MAX) atomicMin(&s_far[nb], far);
  }
  if (first) {
    const int slot = base + __popcll(fm & mask_below(ln));
    if (slot < kSmallCap) {
      s_v[nb][slot] = x;
      s_rs[nb][slot] = rs;
      s_dg[nb][slot] = dg;
    }
    // (a member past the lists' capacity stays in the bitmap only: the set
    // then goes to the wide kernel, which reads the bitmap)
  }
}

__global__ __launch_bounds__(kSmallThreads) void k_sssp_delta_small(SsspArgs a, int32_t source,
                                                                    int64_t max_rounds,
                                                                    uint64_t *F0, uint64_t *F1,
                                                                    uint64_t *F2) {
  __shared__ int s_v[2][kSmallCap], s_rs[2][kSmallCap], s_dg[2][kSmallCap];
  __shared__ int s_n[2], s_near[2], s_sd[2], s_lng[2], s_far[2];
  __shared__ int s_bucket;
  const int tid = threadIdx.x;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  const float delta = a.delta;
  uint64_t *const bm[2] = {F0, F1};
  if (tid == 0) {
    const int dg = rp[source + 1] - rp[source];
    s_v[0][0] = source;
    s_rs[0][0] = rp[source];
    s_dg[0][0] = dg;
    s_n[0] = 1;
    s_near[0] = 1;
    s_sd[0] = dg;
    s_lng[0] = dg > kPushSplit ? 1 : 0;
    s_far[0] = INT_MAX;
    s_bucket = 0;
  }
  __syncthreads();
  int64_t d = 0;
  int b = 0;
  bool spill = false;
  for (;;) {
    const int n = s_n[b];
    if (n == 0 || d >= max_rounds) break;
    if (n > kSmallSpill || s_sd[b] > kSmallEdges) {
      spill = true;
      break;
    }
    const int bucket = s_near[b] > 0 ? s_bucket : s_far[b];
    __syncthreads();  // every thread has read the counters of list b
    if (tid == 0) {
      s_bucket = bucket;
      s_n[b ^ 1] = s_near[b ^ 1] = s_sd[b ^ 1] = s_lng[b ^ 1] = 0;
      s_far[b ^ 1] = INT_MAX;
      a.ctrl->nlev = (int)d + 1;
      a.ctrl->bucket = bucket;
      if (a.stats && d < kStatsCap) {
        a.stats[d * kStatFields + 0] = n;
        a.stats[d * kStatFields + 1] = s_sd[b];
        a.stats[d * kStatFields + 2] = GRB_DIR_PUSH;
        a.stats[d * kStatFields + 3] = bucket;
      }
    }
    __syncthreads();
    const float limit = (float)(bucket + 1) * delta;
    uint64_t *const cons = bm[d & 1], *const fill = bm[(d + 1) & 1];
    for (int base = 0; base < n; base += 4 * kSmallThreads) {
      int v[4], rs[4], dg[4];
      float dv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = base + k * kSmallThreads + tid;
        v[k] = -1;
        rs[k] = dg[k] = 0;
        dv[k] = 0.0f;
        if (i < n) {
          v[k] = s_v[b][i];
          rs[k] = s_rs[b][i];
          dg[k] = s_dg[b][i];
          atomicAnd((unsigned long long *)&cons[v[k] >> 6], ~(1ull << (v[k] & 63)));
          dv[k] = a.dist[v[k]];
        }
      }
      // carried: members above the limit stay pending
#pragma unroll
      for (int k = 0; k < 4; ++k)
        small_insert(v[k] >= 0 && !(dv[k] < limit), v[k], rs[k], dg[k], dv[k], limit, delta, fill,
                     s_v, s_rs, s_dg, s_n, s_near, s_sd, s_lng, s_far, b ^ 1);
      int mx = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (v[k] >= 0 && dv[k] < limit) mx = max(mx, dg[k]);
      for (int q0 = 0; __syncthreads_or(q0 < mx); q0 += 4) {
        int c[16];
        float nd[16];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool ok = v[k] >= 0 && dv[k] < limit && q0 + q < dg[k];
            c[k * 4 + q] = ok ? ci[rs[k] + q0 + q] : -1;
            nd[k * 4 + q] = ok ? dv[k] + a.wpush[rs[k] + q0 + q] : 0.0f;
          }
        int old[16], r0[16], r1[16];
#pragma unroll
        for (int x = 0; x < 16; ++x) {
          old[x] = 0;
          r0[x] = r1[x] = 0;
          if (c[x] >= 0) {
            old[x] = atomicMin((int *)&a.dist[c[x]], __float_as_int(nd[x]));
            r0[x] = rp[c[x]];
            r1[x] = rp[c[x] + 1];
          }
        }
#pragma unroll
        for (int x = 0; x < 16; ++x)
          small_insert(c[x] >= 0 && nd[x] < __int_as_float(old[x]), c[x], r0[x], r1[x] - r0[x],
                       nd[x], limit, delta, fill, s_v, s_rs, s_dg, s_n, s_near, s_sd, s_lng,
                       s_far, b ^ 1);
      }
    }
    __syncthreads();
    ++d;
    b ^= 1;
  }
  if (spill) {
    // the pending set of round d: its bitmap (F[d % 2]) becomes the wide
    // kernel's F[d % 3]; every other buffer is zero; counters and bucket
    uint64_t *const F[3] = {F0, F1, F2};
    uint64_t *src = F[d % 2], *dst = F[d % 3];
    if (src != dst)
      for (int64_t w = tid; w < a.nw; w += kSmallThreads) {
        dst[w] = src[w];
        src[w] = 0ull;
      }
    for (int i = tid; i < 3 * kDeltaSlots; i += kSmallThreads)
      a.ctrl->lists[i] = (i % kDeltaFields) == 3 ? INT_MAX : 0;
    __syncthreads();
    if (tid == 0) {
      int32_t *cnt = a.ctrl->lists + (d % 3) * kDeltaSlots;
      cnt[0] = s_near[b];
      cnt[1] = s_sd[b];
      cnt[2] = s_lng[b];
      cnt[3] = s_far[b];
      cnt[4] = s_n[b];
      a.ctrl->bucket = s_bucket;
    }
  }
  if (tid == 0) {
    a.ctrl->small_levels = (int)d;
    a.ctrl->spilled = spill ? 1 : 0;
  }
}

}  // namespace

void launch_sssp_delta_small(const SsspArgs &a, int32_t source, int64_t max_rounds,
                             uint64_t *const F[3], void *stream) {
  hipLaunchKernelGGL(k_sssp_delta_small, dim3(1), dim3(kSmallThreads), 0, (hipStream_t)stream, a,
                     source, max_rounds, F[0], F[1], F[2]);
}

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
