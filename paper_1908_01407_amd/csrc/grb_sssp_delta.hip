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

// multi-workgroup loop of this file: workgroups, queue segments (one per
// wave), segment counts read per lane of one wave
constexpr int kCoopGrid = kCoopGridSssp;
constexpr int kCoopSegs = kCoopGrid * (kCoopThreads / 64);
constexpr int kCoopSegsPerLane = kCoopSegs / 64;
static_assert(kCoopSegs % 64 == 0 && kCoopSegs <= kCoopSegsMax,
              "segment counts are read by one wave");

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
    if (a.coop) {  // the multi-workgroup loop's first queue: {source}, near
      a.coop->bar = 0ull;
      for (int i = 0; i < kCoopSegsMax; ++i) {
        a.coop->cnt[0][i] = a.coop->esum[0][i] = a.coop->near[0][i] = 0;
        a.coop->far[0][i] = INT_MAX;
      }
      a.coop->cnt[0][0] = 1;
      a.coop->near[0][0] = 1;
      a.coop->esum[0][0] = ds;
      a.qv[0] = source;
      a.qe[0] = ((uint64_t)(uint32_t)ds << 32) | (uint32_t)a.push.rp[source];
    }
  }
}

// ---- multi-workgroup bucket rounds while the pending set is small ----------
// The pending set as a queue in device memory (one segment per wave of the
// loop; entries: vertex, row start | degree << 32) with membership bits in
// F0 / F1 (round d consumes F[d & 1] and fills F[(d + 1) & 1]).  A vertex
// may be queued more than once in a round (each improvement queues it); the
// consumer whose atomicAnd clears its membership bit takes it, and the
// other copies are skipped.  A round: workgroup w takes the entries
// [w n / G, (w + 1) n / G), a thread per entry, which clears the member's
// bit and reads its distance together with its first four out-edges and
// weights; a member below the bucket's limit relaxes its edges (atomicMin
// on the float bits, the target's row extents loaded beside) and queues
// every target it improved, a member above it is queued again (carried).
// Per wave: entries queued, near ones (below the limit), their degree sum,
// the smallest bucket of the others.  The bucket moves to the nearest
// pending one when no near member is left.  A pending set that outgrows
// the segments (or the loop's edge limit) goes to the round kernel.
// Queues in the wave's segment of the next queue (slots counted in wcnt);
// every queued vertex gets its membership bit, also past the segment's end.
__device__ __forceinline__ void coop_queue(bool want, int x, int rs, int dg, float dx, float limit,
                                           float delta, uint64_t *fill, int32_t *qv, uint64_t *qe,
                                           int seg, int &wcnt, int &wnear, int &wsd, int &wfar) {
  const int ln = threadIdx.x & 63;
  const uint64_t m = __ballot(want);
  if (m == 0ull) return;
  const bool nr = want && dx < limit;
  wnear += wave_sum(nr ? 1 : 0);
  wsd += wave_sum(nr ? dg : 0);
  const int far = (want && !nr) ? bucket_of(dx, delta) : INT_MAX;
  wfar = min(wfar, lane_last(wave_scan(far, INT_MAX, [](int p, int q) { return p < q ? p : q; })));
  if (want) {
    const int slot = wcnt + __popcll(m & mask_below(ln));
    atomicOr((unsigned long long *)&fill[x >> 6], 1ull << (x & 63));
    if (slot < seg) {
      st_coherent(qv + slot, x);
      store_relaxed_u64(qe + slot, ((uint64_t)(uint32_t)dg << 32) | (uint32_t)rs);
    }
  }
  wcnt += __popcll(m);
}

__global__ __launch_bounds__(kCoopThreads) void k_sssp_delta_coop(SsspArgs a, int64_t max_rounds,
                                                                  uint64_t wait_ticks,
                                                                  uint64_t *F0, uint64_t *F1) {
  __shared__ int s_pre[kCoopSegs + 1];
  __shared__ int s_n, s_near, s_sd, s_far, s_ovf, s_go;
  const int tid = threadIdx.x, ln = tid & 63;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  const float *wt = a.wpush;
  CoopCtl *cc = a.coop;
  const int w = (int)blockIdx.x;
  const int my_seg = w * (kCoopThreads / 64) + (tid >> 6);
  const int seg = a.qseg, qsize = kCoopSegs * seg;
  const float delta = a.delta;
  int bucket = 0;
  int64_t d = 0;
  bool spill = false;
  for (;;) {
    const int sl = (int)(d & 1);
    if (tid < 64) {  // the round's queue: segment counts and their prefix, totals
      // lane l holds segments kCoopSegsPerLane * l + r
      int c[kCoopSegsPerLane], csum = 0, nr = 0, e = 0, f = INT_MAX;
      bool over = false;
#pragma unroll
      for (int r = 0; r < kCoopSegsPerLane; ++r) {
        const int sg = kCoopSegsPerLane * tid + r;
        c[r] = ld_coherent(&cc->cnt[sl][sg]);
        nr += ld_coherent(&cc->near[sl][sg]);
        e += ld_coherent(&cc->esum[sl][sg]);
        f = min(f, ld_coherent(&cc->far[sl][sg]));
        csum += c[r];
        over |= c[r] > seg;
      }
      const int incl = wave_incl_scan(csum);
      int run = incl - csum;
#pragma unroll
      for (int r = 0; r < kCoopSegsPerLane; ++r) {
        run += c[r];
        s_pre[kCoopSegsPerLane * tid + r + 1] = run;
      }
      const int tot = lane_last(incl), nt = wave_sum(nr), et = wave_sum(e);
      const int ft = lane_last(wave_scan(f, INT_MAX, [](int p, int q) { return p < q ? p : q; }));
      const bool ovf = __ballot(over) != 0ull;
      if (tid == 0) {
        s_pre[0] = 0;
        s_n = tot;
        s_near = nt;
        s_sd = et;
        s_far = ft;
        s_ovf = ovf ? 1 : 0;
      }
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0 || d >= max_rounds) break;
    if (s_ovf || s_sd > kCoopEdges || d >= kCoopMaxLevels) {
      spill = true;
      break;
    }
    bucket = s_near > 0 ? bucket : s_far;
    if (w == 0 && tid == 0) {
      a.ctrl->nlev = (int)d + 1;
      a.ctrl->bucket = bucket;
      if (a.stats && d < kStatsCap) {
        a.stats[d * kStatFields + 0] = n;
        a.stats[d * kStatFields + 1] = s_sd;
        a.stats[d * kStatFields + 2] = GRB_DIR_PUSH;
        a.stats[d * kStatFields + 3] = bucket;
      }
    }
    const float limit = (float)(bucket + 1) * delta;
    uint64_t *const cons = sl ? F1 : F0, *const fill = sl ? F0 : F1;
    const int qin = sl * qsize, qout = (sl ^ 1) * qsize + my_seg * seg;
    int32_t *const qvo = a.qv + qout;
    uint64_t *const qeo = a.qe + qout;
    const int lo = (int)((int64_t)n * w / kCoopGrid);
    const int hi = (int)((int64_t)n * (w + 1) / kCoopGrid);
    int wcnt = 0, wnear = 0, wsd = 0, wfar = INT_MAX;  // uniform over the wave
    for (int base = lo; base < hi; base += kCoopThreads) {
      const int i = base + tid;
      int v = -1, rs = 0, dg = 0;
      if (i < hi) {
        int s = 0;  // segment holding entry i: the last s with s_pre[s] <= i
#pragma unroll
        for (int step = kCoopSegs / 2; step > 0; step >>= 1)
          if (s_pre[s + step] <= i) s += step;
        const int at = qin + s * seg + (i - s_pre[s]);
        v = ld_coherent(a.qv + at);
        const uint64_t e = load_relaxed_u64(a.qe + at);
        rs = (int)(uint32_t)e;
        dg = (int)(e >> 32);
      }
      bool take = false;
      float dv = 0.0f;
      int c0[4];
      float w0[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c0[q] = -1;
        w0[q] = 0.0f;
      }
      if (v >= 0) {
        const uint64_t bit = 1ull << (v & 63);
        const uint64_t was = atomicAnd((unsigned long long *)&cons[v >> 6], ~bit);
        dv = __int_as_float(ld_coherent((const int32_t *)&a.dist[v]));
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < dg) {
            c0[q] = ci[rs + q];
            w0[q] = wt[rs + q];
          }
        take = (was & bit) != 0ull;
      }
      const bool relax = take && dv < limit;
      // carried: a member above the limit stays pending
      coop_queue(take && !relax, v, rs, dg, dv, limit, delta, fill, qvo, qeo, seg, wcnt, wnear,
                 wsd, wfar);
      for (int q0 = 0; __ballot(relax && q0 < dg) != 0ull; q0 += 4) {
        int c[4];
        float nd[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = relax && q0 + q < dg;
          c[q] = !ok ? -1 : (q0 == 0 ? c0[q] : ci[rs + q0 + q]);
          nd[q] = !ok ? 0.0f : dv + (q0 == 0 ? w0[q] : wt[rs + q0 + q]);
        }
        int old[4], r0[4], r1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          old[q] = 0;
          r0[q] = r1[q] = 0;
          if (c[q] >= 0) {
            old[q] = atomicMin((int *)&a.dist[c[q]], __float_as_int(nd[q]));
            r0[q] = rp[c[q]];
            r1[q] = rp[c[q] + 1];
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          coop_queue(c[q] >= 0 && nd[q] < __int_as_float(old[q]), c[q], r0[q], r1[q] - r0[q],
                     nd[q], limit, delta, fill, qvo, qeo, seg, wcnt, wnear, wsd, wfar);
      }
    }
    // the wave's segment counters go with its entries; the barrier follows
    // once every memory operation of the workgroup is done
    if (ln == 0) {
      st_coherent(&cc->cnt[sl ^ 1][my_seg], wcnt);
      st_coherent(&cc->near[sl ^ 1][my_seg], wnear);
      st_coherent(&cc->esum[sl ^ 1][my_seg], wsd);
      st_coherent(&cc->far[sl ^ 1][my_seg], wfar);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) s_go = coop_barrier(&cc->bar, kCoopGrid, d, wait_ticks);
    __syncthreads();
    ++d;
    if (!s_go) {
      // barrier given up: the pending set of round d (complete: every
      // workgroup finished round d - 1) goes to the round kernel
      spill = true;
      break;
    }
  }
  if (w == 0 && tid == 0) {
    a.ctrl->small_levels = (int)d;
    a.ctrl->spilled = spill ? 1 : 0;
  }
}

// After the loop spilled at round h = ctrl->small_levels: its pending set
// (bitmap F[h & 1] of F0 / F1) becomes the round kernel's F[h % 3] (every
// other buffer is zero), with the counters and bucket of round h.
__global__ __launch_bounds__(kBlock) void k_sssp_delta_coop_handover(SsspArgs a, uint64_t *F0,
                                                                      uint64_t *F1,
                                                                      uint64_t *F2) {
  if (!a.ctrl->spilled) return;
  const int64_t h = a.ctrl->small_levels;
  uint64_t *const F[3] = {F0, F1, F2};
  uint64_t *src = F[h & 1], *dst = F[h % 3];
  if (src != dst)
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < a.nw;
         w += (int64_t)gridDim.x * kBlock) {
      dst[w] = src[w];
      src[w] = 0ull;
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int sl = (int)(h & 1);
    int nq = 0, nr = 0, sd = 0, far = INT_MAX;
    for (int s = 0; s < kCoopSegs; ++s) {
      nq += a.coop->cnt[sl][s];
      nr += a.coop->near[sl][s];
      sd += a.coop->esum[sl][s];
      far = min(far, a.coop->far[sl][s]);
    }
    for (int i = 0; i < 3 * kDeltaSlots; ++i)
      a.ctrl->lists[i] = (i % kDeltaFields) == 3 ? INT_MAX : 0;
    int32_t *cnt = a.ctrl->lists + (h % 3) * kDeltaSlots;
    cnt[0] = nr;
    cnt[1] = sd;
    cnt[2] = 0;  // rows are at most kCoopMaxDeg long
    cnt[3] = far;
    cnt[4] = nq;
  }
}

}  // namespace

void launch_sssp_delta_coop(const SsspArgs &a, int64_t max_rounds, uint64_t *const F[3],
                            uint64_t wait_ticks, void *stream) {
  hipLaunchKernelGGL(k_sssp_delta_coop, dim3(kCoopGrid), dim3(kCoopThreads), 0,
                     (hipStream_t)stream, a, max_rounds, wait_ticks, F[0], F[1]);
  int64_t g = (a.nw + kBlock - 1) / kBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_sssp_delta_coop_handover, dim3((unsigned)g), dim3(kBlock), 0,
                     (hipStream_t)stream, a, F[0], F[1], F[2]);
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
