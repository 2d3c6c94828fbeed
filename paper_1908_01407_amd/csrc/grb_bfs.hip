// Direction-optimised BFS (Algorithm 1 and Section 7.1 of the paper) with
// one kernel per level.
//
// Each level is f <- A^T f .* not(visited) over the Boolean semiring, run as
// push (SpMSpV from the frontier's out-edges) or pull (masked SpMV over the
// unvisited rows, stopping a row at its first frontier neighbour), chosen on
// the device from the frontier's size and degree sum (the switch rule of the
// descriptor).  The frontier is only a bitmap, and one kernel does all of a
// level, so nothing sits between levels:
// * push gives each wave a run of frontier words and streams the out-edges
//   of its frontier rows as one concatenated list (the same wave-level
//   load-balanced search as pull); rows longer than kPushSplit come from a
//   static list of kPushSplit-edge pieces built by grb_matrix_prepare,
//   spread over all waves, each piece active when its row is in the
//   frontier;
// * a vertex is claimed by the first atomicOr on its visited bit; the
//   claimer writes its level and sets its bit in the next frontier bitmap;
// * the next frontier's size and degree sum are reduced per workgroup and
//   added into kCntStripes striped counters (few atomics per address);
// * bitmaps and counters rotate through three buffers: the level reads
//   buffer d, fills buffer d+1 and clears buffer d+2.
// Pull finds the smallest-id parent directly (ascending adjacency, first
// hit).  A push from a one-vertex frontier writes that vertex as parent.
// Vertices found by a push of several vertices get theirs in the next
// level's kernel, where they are the frontier: the smallest in-neighbour
// one level up, offered edge by edge while that level pushes over the same
// CSR, else found by a pass over their in-edges (first hit in ascending
// order); a standalone pass covers the last level when the level cap stops
// the search.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

// multi-workgroup loop of this file: workgroups, queue segments (one per
// wave), segment counts read per lane of one wave
constexpr int kCoopGrid = kCoopGridBfs;
constexpr int kCoopSegs = kCoopGrid * (kCoopThreads / 64);
constexpr int kCoopSegsPerLane = kCoopSegs / 64;
static_assert(kCoopSegs % 64 == 0 && kCoopSegs <= kCoopSegsMax,
              "segment counts are read by one wave");

__device__ __forceinline__ int decide(const BfsArgs &a, int count, int sumdeg) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

// Finishes the claims won by this lane: level, next-frontier bit, counts.
// dg[s]: out-degree of target c[s], loaded by the caller together with its
// visited word (before the claim is decided, so no load follows it).
// With a one-vertex frontier (`single`) that vertex, par[s], is the only
// parent a target can have, and it is written at once.
// `next_set`: the caller has already set the targets' next-frontier bits.
__device__ __forceinline__ void claim_won(const BfsArgs &a, const int (&c)[kUnroll],
                                          const bool (&won)[kUnroll], const int (&par)[kUnroll],
                                          const int (&dg)[kUnroll], bool single, bool next_set,
                                          int &fc, int &fd, int &fl) {
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    if (won[s]) {
      a.levels[c[s]] = a.d + 1;
      if (single && a.parents) a.parents[c[s]] = par[s];
      if (!next_set)
        atomicOr((unsigned long long *)&a.fnxt[c[s] >> 6], 1ull << (c[s] & 63));
      fc += 1;
      fd += dg[s];
      fl += dg[s] > kPushSplit ? 1 : 0;
    }
  }
}

// Row extents of the targets still unvisited at the filter read (0 for the
// others: a visited target cannot be won), issued beside the claim atomics,
// whose latency covers theirs.
__device__ __forceinline__ void target_degrees(const BfsArgs &a, const int (&c)[kUnroll],
                                               const bool (&open)[kUnroll], int (&d0)[kUnroll],
                                               int (&d1)[kUnroll]) {
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    d0[s] = open[s] ? a.push.rp[c[s]] : 0;
    d1[s] = open[s] ? a.push.rp[c[s] + 1] : 0;
  }
}

// Parents of the frontier while a push expands it (symmetric graphs, whose
// out-edges are the in-edges): an expanded edge (u, v) with v one level
// above u offers v as u's parent, and the smallest offer wins (parents[u]
// is -1 until then, the largest value as unsigned).  lv[s]: level of c[s],
// loaded by the caller together with its visited words.
__device__ __forceinline__ void offer_parents(const BfsArgs &a, const int (&c)[kUnroll],
                                              const int (&par)[kUnroll], const int (&lv)[kUnroll]) {
#pragma unroll
  for (int s = 0; s < kUnroll; ++s)
    if (c[s] >= 0 && lv[s] == a.d - 1)
      atomicMin((unsigned int *)&a.parents[par[s]], (unsigned int)c[s]);
}

// Claims the targets c[0..kUnroll) (-1: none) from a stream that may hold
// one target twice.  The visited words of all of them are read first (a
// plain read is only a filter, the atomic decides) and all atomics are
// issued before any result is used, so their latencies overlap; the row
// extents of the unvisited targets are loaded beside them.
__device__ __forceinline__ void claim_batch(const BfsArgs &a, const int (&c)[kUnroll],
                                            const int (&par)[kUnroll], bool single, bool offer,
                                            int &fc, int &fd, int &fl) {
  uint64_t vw[kUnroll];
  int lv[kUnroll], d0[kUnroll], d1[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    vw[s] = c[s] >= 0 ? a.visited[c[s] >> 6] : ~0ull;
    lv[s] = (offer && c[s] >= 0) ? a.levels[c[s]] : -2;
  }
  if (offer) offer_parents(a, c, par, lv);
  bool open[kUnroll];
  uint64_t old[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    open[s] = c[s] >= 0 && !((vw[s] >> (c[s] & 63)) & 1ull);
    old[s] = ~0ull;
    if (open[s])
      old[s] = atomicOr((unsigned long long *)&a.visited[c[s] >> 6], 1ull << (c[s] & 63));
  }
  target_degrees(a, c, open, d0, d1);
  bool won[kUnroll];
  int dg[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    won[s] = c[s] >= 0 && !((old[s] >> (c[s] & 63)) & 1ull);
    dg[s] = d1[s] - d0[s];
  }
  claim_won(a, c, won, par, dg, single, false, fc, fd, fl);
}

// Claims the targets of one piece of a row: ascending and distinct, so the
// lanes whose targets share a visited word sit side by side and one atomicOr
// per word serves them all (issued by the run's last lane, whose previous
// value of the word every lane of the run then reads).
__device__ __forceinline__ void claim_piece(const BfsArgs &a, const int (&c)[kUnroll],
                                            const int (&par)[kUnroll], bool single, bool offer,
                                            int &fc, int &fd, int &fl) {
  uint64_t vw[kUnroll];
  int lv[kUnroll], d0[kUnroll], d1[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    vw[s] = c[s] >= 0 ? a.visited[c[s] >> 6] : ~0ull;
    lv[s] = (offer && c[s] >= 0) ? a.levels[c[s]] : -2;
  }
  if (offer) offer_parents(a, c, par, lv);
  bool want[kUnroll];
  uint64_t old[kUnroll], run[kUnroll];
  int64_t wd[kUnroll];
  int tail[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    want[s] = c[s] >= 0 && !((vw[s] >> (c[s] & 63)) & 1ull);
    wd[s] = want[s] ? (int64_t)(c[s] >> 6) : -1;
    run[s] = run_tail_or(wd[s], want[s] ? (1ull << (c[s] & 63)) : 0ull, tail[s]);
    old[s] = 0ull;
    if (run[s] && wd[s] >= 0)
      old[s] = atomicOr((unsigned long long *)&a.visited[wd[s]], (unsigned long long)run[s]);
  }
  target_degrees(a, c, want, d0, d1);
  bool won[kUnroll];
  int dg[kUnroll];
#pragma unroll
  for (int s = 0; s < kUnroll; ++s) {
    const uint64_t ow = __shfl(old[s], tail[s]);
    won[s] = want[s] && !((ow >> (c[s] & 63)) & 1ull);
    dg[s] = d1[s] - d0[s];
    // the run's tail also sets the won bits of the next frontier at once
    if (run[s] && wd[s] >= 0 && (run[s] & ~old[s]))
      atomicOr((unsigned long long *)&a.fnxt[wd[s]], (unsigned long long)(run[s] & ~old[s]));
  }
  claim_won(a, c, won, par, dg, single, true, fc, fd, fl);
}

// Each wave loads 64 bitmap words at once (one per lane) and compacts their
// set bits into a queue of rows, taken 64 at a time (one row per lane).  The
// edges of rows up to kPushSplit (push) or kHeavyDeg (pull) long are streamed
// as one concatenated list; longer rows come in static pieces spread over
// all waves, so a hub is expanded by hundreds of waves at once.

__device__ __forceinline__ void bfs_push(const BfsArgs &a, int *mark, bool long_rows, bool single,
                                         bool offer, int &fc, int &fd, int &fl) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  // words dealt out round-robin (wave gw takes words gw, gw + nwaves, ...)
  // so that runs of high-degree rows spread over the waves
  for (int64_t w0 = gw; w0 < a.nw; w0 += 64 * nwaves) {
    const int64_t mw = w0 + (int64_t)ln * nwaves;
    uint64_t mf = 0ull;
    if (mw < a.nw) {
      a.fclr[mw] = 0ull;  // the bitmap two levels ahead
      mf = a.fcur[mw];
    }
    const int cnt = __popcll(mf);
    const int incl = wave_incl_scan(cnt);
    const int total = lane_last(incl);
    for (int b = 0; b < total; b += 64) {
      const int64_t u = queue_slot(mark, mf, cnt, incl, total, b, mw);
      int cur = 0, end = 0;
      if (u >= 0) {
        cur = rp[u];
        end = rp[u + 1];
        if (end - cur > kPushSplit) end = cur;  // long rows: static pieces below
      }
      // the rows' out-edges as one concatenated stream, kUnroll x 64 edges
      // per step
      const int uid = (int)u;
      for (bool more = true; more;) {
        int c[kUnroll], par[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          c[s] = -1;
          par[s] = -1;
          if (!more) continue;
          const int len = end - cur;
          const int incl2 = wave_incl_scan(len);
          const int tot2 = lane_last(incl2);
          if (tot2 == 0) {
            more = false;
            continue;
          }
          const int excl = incl2 - len;
          const bool starts = len > 0 && excl < 64;
          const int r = slot_rows(mark, starts, excl);
          const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
          par[s] = __shfl(uid, r);
          if (ln < tot2) c[s] = rcur + (ln - rexcl);
          if (starts) cur += min(incl2, 64) - excl;
        }
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) c[s] = c[s] >= 0 ? ci[c[s]] : -1;
        claim_batch(a, c, par, single, offer, fc, fd, fl);
      }
    }
  }
  // static pieces of long rows, spread over the waves (wave gw owns pieces
  // gw, gw + nwaves, ...), 64 tested per step; a piece whose row is in the
  // frontier is streamed by the whole wave, kUnroll x 64 edges at once
  static_assert(kPushSplit == 64 * kUnroll, "a push piece is one unrolled step");
  if (!long_rows) return;  // no row of the frontier has pieces
  for (int64_t hb = gw; hb < a.push.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int u = -1, b = 0, e = 0;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      b = a.push.split[2 * h + 1];
      if (bit_of(a.fcur, u)) e = min(b + kPushSplit, rp[u + 1]);
      else u = -1;
    }
    uint64_t act = __ballot(u >= 0);
    while (act) {
      const int k = __ffsll((unsigned long long)act) - 1;
      act &= act - 1;
      const int pb = __shfl(b, k), pe = __shfl(e, k), pu = __shfl(u, k);
      int c[kUnroll], par[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int pos = pb + s * 64 + ln;
        c[s] = pos < pe ? ci[pos] : -1;
        par[s] = pu;
      }
      claim_piece(a, c, par, single, offer, fc, fd, fl);
    }
  }
}

// Records rows found in a pull: rows of one bitmap word sit in consecutive
// lanes (ascending ids), so one atomicOr per word and bitmap serves them.
__device__ __forceinline__ void pull_found(const BfsArgs &a, bool found, int64_t v, int par,
                                           int deg, int &fc, int &fd, int &fl) {
  const int64_t vw = found ? (v >> 6) : -1;
  int tail;
  const uint64_t hb = run_tail_or(vw, found ? (1ull << (v & 63)) : 0ull, tail);
  if (hb && vw >= 0) {
    atomicOr((unsigned long long *)&a.visited[vw], (unsigned long long)hb);
    atomicOr((unsigned long long *)&a.fnxt[vw], (unsigned long long)hb);
  }
  if (found) {
    a.levels[v] = a.d + 1;
    if (a.parents) a.parents[v] = par;
    const int pd = a.same_csr ? deg : a.push.rp[v + 1] - a.push.rp[v];
    fc += 1;
    fd += pd;
    fl += pd > kPushSplit ? 1 : 0;
  }
}

// Pull stream of the unsettled rows (one per lane: `act`, remaining
// positions [rc, re)) as one concatenated list, K steps of 64 positions
// laid out and loaded at once (K > 1 when the probes found the frontier
// sparse, so that rows rarely stop early); the steps are then read in
// order, so a row's first frontier neighbour (its smallest id: columns
// ascend) is its parent.
template <int K>
__device__ __forceinline__ void pull_stream(const BfsArgs &a, int *mark, bool act, int &rc, int re,
                                            bool &found, int &par) {
  const int ln = threadIdx.x & 63;
  const int32_t *ci = a.pull.ci;
  for (bool more = true; more;) {
    int pos[K], sev[K], exv[K];
    bool st[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      pos[s] = -1;
      sev[s] = exv[s] = 0;
      st[s] = false;
      if (!more) continue;
      const int len = (act && !found) ? re - rc : 0;
      const int incl = wave_incl_scan(len);
      const int total = lane_last(incl);
      if (total == 0) {
        more = false;
        continue;
      }
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(rc, r), rexcl = __shfl(excl, r);
      if (ln < total) pos[s] = rcur + (ln - rexcl);
      sev[s] = min(incl, 64);
      exv[s] = excl;
      st[s] = starts;
      if (starts) rc += sev[s] - excl;
    }
    int c[K];
#pragma unroll
    for (int s = 0; s < K; ++s) c[s] = pos[s] >= 0 ? ci[pos[s]] : -1;
    uint64_t fw[K];
#pragma unroll
    for (int s = 0; s < K; ++s) fw[s] = c[s] >= 0 ? a.fcur[c[s] >> 6] : 0ull;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const uint64_t hm = __ballot(c[s] >= 0 && ((fw[s] >> (c[s] & 63)) & 1ull));
      const uint64_t seg = st[s] ? (mask_below(sev[s]) & ~mask_below(exv[s])) : 0ull;
      const uint64_t h = hm & seg;
      const int first = h ? (__ffsll((unsigned long long)h) - 1) : 0;
      const int pc = __shfl(c[s], first);
      if (h && !found) {
        found = true;
        par = pc;
      }
    }
  }
}

__device__ __forceinline__ void bfs_pull(const BfsArgs &a, int *mark, int &fc, int &fd, int &fl) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  int64_t lo, hi;
  wave_words(a.nw, gw, nwaves, lo, hi);
  for (int64_t w0 = lo; w0 < hi; w0 += 64) {
    const int64_t mw = w0 + ln;
    uint64_t mc = 0ull;  // candidate rows: not visited
    if (mw < hi) {
      a.fclr[mw] = 0ull;
      mc = ~a.visited[mw];
    }
    const int cnt = __popcll(mc);
    const int incl = wave_incl_scan(cnt);
    const int total = lane_last(incl);
    // kPullRows queued rows per lane: the loads of their first two
    // neighbours are issued together
    for (int b = 0; b < total; b += 64 * kPullRows) {
      int64_t v[kPullRows];
      int cur[kPullRows], end[kPullRows];
      bool act[kPullRows];
#pragma unroll
      for (int q = 0; q < kPullRows; ++q) {
        v[q] = b + q * 64 < total ? queue_slot(mark, mc, cnt, incl, total, b + q * 64, mw) : -1;
        act[q] = v[q] >= 0;
      }
      // row extents and the first two neighbours (a separate array read
      // in row order), all issued together
      int c0[kPullRows], c1[kPullRows];
#pragma unroll
      for (int q = 0; q < kPullRows; ++q) {
        cur[q] = act[q] ? rp[v[q]] : 0;
        end[q] = act[q] ? rp[v[q] + 1] : 0;
        const int2 f = act[q] ? a.pull.first2[v[q]] : make_int2(-1, -1);
        c0[q] = f.x;
        c1[q] = f.y;
      }
#pragma unroll
      for (int q = 0; q < kPullRows; ++q)
        if (end[q] - cur[q] > kHeavyDeg || end[q] == cur[q]) {  // pieces / empty
          act[q] = false;
          c0[q] = c1[q] = -1;
        }
      uint64_t b0[kPullRows], b1[kPullRows];
#pragma unroll
      for (int q = 0; q < kPullRows; ++q) {
        b0[q] = c0[q] >= 0 ? a.fcur[c0[q] >> 6] : 0ull;
        b1[q] = c1[q] >= 0 ? a.fcur[c1[q] >> 6] : 0ull;
      }
      // rows settled by their first two neighbours; the others (with more
      // edges left) are counted per batch for the stream below
      uint64_t rest[kPullRows];
      int nrest = 0, np = 0, nh = 0;
#pragma unroll
      for (int q = 0; q < kPullRows; ++q) {
        bool found = false;
        int par = -1;
        const bool h0 = c0[q] >= 0 && ((b0[q] >> (c0[q] & 63)) & 1ull);
        const bool h1 = c1[q] >= 0 && ((b1[q] >> (c1[q] & 63)) & 1ull);
        np += __popcll(__ballot(c0[q] >= 0)) + __popcll(__ballot(c1[q] >= 0));
        nh += __popcll(__ballot(h0)) + __popcll(__ballot(h1));
        if (h0) {
          found = true;
          par = c0[q];
        } else if (h1) {
          found = true;
          par = c1[q];
        }
        pull_found(a, found, v[q], par, end[q] - cur[q], fc, fd, fl);
        rest[q] = __ballot(act[q] && !found && end[q] - cur[q] > 2);
        nrest += __popcll(rest[q]);
      }
      // the unsettled rows of all batches, compacted 64 at a time, stream
      // their remaining edges as one concatenated list with early exit
      for (int sb = 0; sb < nrest; sb += 64) {
        const int j = sb + ln;  // this lane's place among the unsettled rows
        int64_t rv = -1;
        int rc = 0, re = 0;
        int before = 0;
#pragma unroll
        for (int q = 0; q < kPullRows; ++q) {
          const int cq = __popcll(rest[q]);
          const int li = (j >= before && j < before + cq) ? nth_set_bit(rest[q], j - before) : 0;
          const int64_t sv = __shfl(v[q], li);
          const int sc = __shfl(cur[q], li), se_ = __shfl(end[q], li);
          if (j >= before && j < before + cq) {
            rv = sv;
            rc = sc + 2;
            re = se_;
          }
          before += cq;
        }
        const bool act2 = rv >= 0;
        const int deg2 = re - (rc - 2);
        bool found = false;
        int par = -1;
        // a frontier the probes found below 1/8 dense: four steps at once
        if (8 * nh < np) pull_stream<kUnroll>(a, mark, act2, rc, re, found, par);
        else pull_stream<1>(a, mark, act2, rc, re, found, par);
        pull_found(a, found, rv, par, deg2, fc, fd, fl);
      }
    }
  }
  // pieces of long rows; a row counts as a candidate unless it was reached
  // before this level (its level is then 0..d): a piece's claim must not
  // hide the row from its other pieces, whose first frontier neighbour may
  // have a smaller id.  kUnroll x 64 edges are loaded at once and searched
  // for the first frontier neighbour in order; the parent is the minimum
  // over the pieces.
  // Wave gw owns pieces gw, gw + nwaves, ...: 64 of them are tested at once
  // (one per lane), then the wave streams the live ones.
  for (int64_t hb = gw; hb < a.pull.nheavy; hb += 64 * nwaves) {
    const int64_t hh = hb + (int64_t)ln * nwaves;
    int hr = -1, hbeg = 0, hend = 0;
    if (hh < a.pull.nheavy) {
      hr = a.pull.heavy[2 * hh];
      hbeg = a.pull.heavy[2 * hh + 1];
      const int lr = a.levels[hr];
      if (lr >= 0 && lr <= a.d) hr = -1;
      else hend = min(hbeg + kHeavyChunk, rp[hr + 1]);
    }
    uint64_t live = __ballot(hr >= 0);
    while (live) {
      const int k = __ffsll((unsigned long long)live) - 1;
      live &= live - 1;
      const int r = __shfl(hr, k), b = __shfl(hbeg, k), e = __shfl(hend, k);
      for (int base = b; base < e; base += 64 * kUnroll) {
        int c[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) {
          const int pos = base + s * 64 + ln;
          c[s] = pos < e ? ci[pos] : -1;
        }
        uint64_t fwd[kUnroll];
#pragma unroll
        for (int s = 0; s < kUnroll; ++s) fwd[s] = c[s] >= 0 ? a.fcur[c[s] >> 6] : 0ull;
        int pc = -1;
#pragma unroll
        for (int s = kUnroll - 1; s >= 0; --s) {
          const uint64_t hm = __ballot(c[s] >= 0 && ((fwd[s] >> (c[s] & 63)) & 1ull));
          if (hm) pc = __shfl(c[s], __ffsll((unsigned long long)hm) - 1);
        }
        if (pc >= 0) {
          if (ln == 0) {
            const uint64_t bit = 1ull << (r & 63);
            const uint64_t old =
                atomicOr((unsigned long long *)&a.visited[r >> 6], (unsigned long long)bit);
            if (a.parents) atomicMin((unsigned *)&a.parents[r], (unsigned)pc);
            if (!(old & bit)) {
              a.levels[r] = a.d + 1;
              atomicOr((unsigned long long *)&a.fnxt[r >> 6], (unsigned long long)bit);
              const int pd = a.push.rp[r + 1] - a.push.rp[r];
              fc += 1;
              fd += pd;
              fl += pd > kPushSplit ? 1 : 0;
            }
          }
          break;
        }
      }
    }
  }
}

// Smallest-id parent of every vertex reached by a push: the first
// in-neighbour (ascending) whose level is one less.  A wave compacts the
// vertices that need a parent in 8 words of its run into a queue, 64 at a
// time; the first two in-neighbours of every queued row are tested in
// parallel, the rest streamed as one concatenated list.
__device__ __forceinline__ void parents_pass(const BfsArgs &a, int *mark) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  int64_t lo, hi;
  wave_words(a.nw, gw, nwaves, lo, hi);
  for (int64_t w0 = lo; w0 < hi; w0 += 8) {
    // the vertices of 8 words that still need a parent: reached (level > 0)
    // and without one; all 16 loads per lane are issued together
    uint64_t nm[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t v = (w0 + k) * 64 + ln;
      const bool inb = w0 + k < hi && v < a.n;
      const int lv = inb ? a.levels[v] : -1;
      const int pv = inb ? a.parents[v] : 0;
      nm[k] = __ballot(lv > 0 && pv < 0);
    }
    uint64_t mq = 0ull;  // lane k < 8 holds word w0 + k's mask
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (ln == k) mq = nm[k];
    const int cnt = __popcll(mq);
    const int incl = wave_incl_scan(cnt);
    const int total = lane_last(incl);
    for (int b = 0; b < total; b += 64) {
      const int64_t v = queue_slot(mark, mq, cnt, incl, total, b, w0 + ln);
      const bool need = v >= 0;
      int cur = need ? rp[v] : 0;
      const int end = need ? rp[v + 1] : 0;
      const int tgt = need ? a.levels[v] - 1 : -3;
      bool found = false;
      int par = -1;
      if (need) {
        const int2 f = a.pull.first2[v];
        const int c0 = f.x;
        const int c1 = f.y;
        const int l0 = c0 >= 0 ? a.levels[c0] : -2;
        const int l1 = c1 >= 0 ? a.levels[c1] : -2;
        if (l0 == tgt) { found = true; par = c0; }
        else if (l1 == tgt) { found = true; par = c1; }
        cur = min(cur + 2, end);
      }
      for (;;) {
        const int len = (need && !found) ? end - cur : 0;
        const int incl2 = wave_incl_scan(len);
        const int tot2 = lane_last(incl2);
        if (tot2 == 0) break;
        const int excl = incl2 - len;
        const bool starts = len > 0 && excl < 64;
        const int r = slot_rows(mark, starts, excl);
        const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r), rt = __shfl(tgt, r);
        const bool valid = ln < tot2;
        const int c = valid ? ci[rcur + (ln - rexcl)] : -1;
        const uint64_t hm = __ballot(valid && a.levels[c] == rt);
        const int se = min(incl2, 64);
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
}

// Parents of this level's frontier when a push of more than one vertex
// found it: for each frontier vertex v (queued from the frontier words, dealt
// out round-robin), the first in-neighbour one level up in ascending order.
__device__ __forceinline__ void frontier_parents(const BfsArgs &a, int *mark) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const int tgt = a.d - 1;
  for (int64_t w0 = gw; w0 < a.nw; w0 += 64 * nwaves) {
    const int64_t mw = w0 + (int64_t)ln * nwaves;
    const uint64_t mf = mw < a.nw ? a.fcur[mw] : 0ull;
    const int cnt = __popcll(mf);
    const int incl = wave_incl_scan(cnt);
    const int total = lane_last(incl);
    for (int b = 0; b < total; b += 64) {
      const int64_t v = queue_slot(mark, mf, cnt, incl, total, b, mw);
      const bool need = v >= 0;
      int cur = need ? rp[v] : 0;
      const int end = need ? rp[v + 1] : 0;
      bool found = false;
      int par = -1;
      if (need) {
        const int2 f = a.pull.first2[v];
        const int c0 = f.x;
        const int c1 = f.y;
        const int l0 = c0 >= 0 ? a.levels[c0] : -2;
        const int l1 = c1 >= 0 ? a.levels[c1] : -2;
        if (l0 == tgt) { found = true; par = c0; }
        else if (l1 == tgt) { found = true; par = c1; }
        cur = min(cur + 2, end);
      }
      for (;;) {
        const int len = (need && !found) ? end - cur : 0;
        const int incl2 = wave_incl_scan(len);
        const int tot2 = lane_last(incl2);
        if (tot2 == 0) break;
        const int excl = incl2 - len;
        const bool starts = len > 0 && excl < 64;
        const int r = slot_rows(mark, starts, excl);
        const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
        const bool valid = ln < tot2;
        const int c = valid ? ci[rcur + (ln - rexcl)] : -1;
        const uint64_t hm = __ballot(valid && a.levels[c] == tgt);
        const int se = min(incl2, 64);
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
}

// Parents of the frontier from the previous one: every vertex at level
// d - 1 offers itself (atomicMin) to its out-neighbours at level d, whose
// parents then hold the smallest such id (the claim's winner is one of
// them).  Chosen over the in-edge pass above when the previous frontier's
// degree sum and a scan of the levels cost less than this frontier's
// in-edges.  Rows of at most kPushSplit edges: 64 vertices per wave step,
// the selected rows' edges as one concatenated stream; longer rows through
// the push CSR's pieces, dealt to the waves with a stride.
__device__ __forceinline__ void prev_offers(const BfsArgs &a, int *mark) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  const int tgt = a.d - 1;
  for (int64_t b0 = gw * 64; b0 < a.n; b0 += nwaves * 64) {
    const int64_t u = b0 + ln;
    const bool sel = u < a.n && a.levels[u] == tgt;
    int cur = sel ? rp[u] : 0;
    const int end = sel ? rp[u + 1] : 0;
    if (end - cur > kPushSplit) cur = end;  // pieces below
    for (;;) {
      const int len = end - cur;
      const int incl = wave_incl_scan(len);
      const int total = lane_last(incl);
      if (total == 0) break;
      const int excl = incl - len;
      const bool starts = len > 0 && excl < 64;
      const int r = slot_rows(mark, starts, excl);
      const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
      if (ln < total) {
        const int v = ci[rcur + (ln - rexcl)];
        if (a.levels[v] == a.d) atomicMin((unsigned *)&a.parents[v], (unsigned)(b0 + r));
      }
      if (starts) cur += min(incl, 64) - excl;
    }
  }
  for (int64_t hb = gw; hb < a.push.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int u = -1, b = 0, e = 0;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      b = a.push.split[2 * h + 1];
      if (a.levels[u] == tgt) e = min(b + kPushSplit, rp[u + 1]);
      else u = -1;
    }
    for (uint64_t act = __ballot(u >= 0); act; act &= act - 1) {
      const int k = __ffsll((unsigned long long)act) - 1;
      const int pb = __shfl(b, k), pe = __shfl(e, k), pu = __shfl(u, k);
      int v[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) {
        const int pos = pb + s * 64 + ln;
        v[s] = pos < pe ? ci[pos] : -1;
      }
      int lv[kUnroll];
#pragma unroll
      for (int s = 0; s < kUnroll; ++s) lv[s] = v[s] >= 0 ? a.levels[v[s]] : -1;
#pragma unroll
      for (int s = 0; s < kUnroll; ++s)
        if (lv[s] == a.d) atomicMin((unsigned *)&a.parents[v[s]], (unsigned)pu);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_bfs_parents(BfsArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  parents_pass(a, s_mark[threadIdx.x >> 6]);
}

__global__ __launch_bounds__(kBlock) void k_bfs_level(BfsArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int s_count, s_sumdeg, s_long, s_open, s_prev_sd;
  __shared__ int s_red[kWavesPerBlock][kCntFields];
  if (threadIdx.x == 0) {
    s_open = a.parents ? a.ctrl->pushed[a.d % 3] : 0;
    s_prev_sd = s_open ? a.ctrl->pushed_sd[a.d % 3] : 0;
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
      // the buffer two levels ahead is cleared even when this level is
      // empty: it still holds the counts of the previous level
      for (int i = 0; i < kCntSlots; ++i) a.cnt_clr[i] = 0;
      if (c > 0) {
        a.ctrl->nlev = a.d + 1;
        // the next frontier's parents stay open when a push of several
        // vertices finds it
        a.ctrl->pushed[(a.d + 1) % 3] = (decide(a, c, sd) == GRB_DIR_PUSH && c > 1) ? 1 : 0;
        a.ctrl->pushed_sd[(a.d + 1) % 3] = sd;
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
  int fc = 0, fd = 0, fl = 0;
  // parents of this frontier, when a push of several vertices found it: a
  // push over the same CSR offers them while it expands the frontier;
  // otherwise the previous frontier offers them again when its degree sum
  // and a scan of the levels cost less than this frontier's in-edges, and
  // else a pass over those in-edges finds them first
  const bool offer = s_open && dir == GRB_DIR_PUSH && a.same_csr;
  if (s_open && !offer) {
    if ((int64_t)s_prev_sd + a.n / 16 < (int64_t)s_sumdeg) prev_offers(a, s_mark[threadIdx.x >> 6]);
    else frontier_parents(a, s_mark[threadIdx.x >> 6]);
  }
  if (dir == GRB_DIR_PUSH)
    bfs_push(a, s_mark[threadIdx.x >> 6], s_long > 0, count == 1, offer, fc, fd, fl);
  else
    bfs_pull(a, s_mark[threadIdx.x >> 6], fc, fd, fl);
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

__global__ __launch_bounds__(kBlock) void k_bfs_start(BfsArgs a, int32_t source, uint64_t *f1,
                                                      uint64_t *f2) {
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * kBlock;
  // levels and parents: -1 (source: 0 and itself), four vertices per
  // 16-byte store when both arrays allow it
  const bool vec = ((uintptr_t)a.levels % 16 == 0) &&
                   (!a.parents || (uintptr_t)a.parents % 16 == 0);
  const int64_t n4 = vec ? a.n / 4 : 0;
  for (int64_t i = tid; i < n4; i += nt) {
    int4 l = make_int4(-1, -1, -1, -1), p = l;
    if ((source >> 2) == i) {
      const int k = source & 3;
      if (k == 0) { l.x = 0; p.x = source; }
      else if (k == 1) { l.y = 0; p.y = source; }
      else if (k == 2) { l.z = 0; p.z = source; }
      else { l.w = 0; p.w = source; }
    }
    reinterpret_cast<int4 *>(a.levels)[i] = l;
    if (a.parents) reinterpret_cast<int4 *>(a.parents)[i] = p;
  }
  for (int64_t v = n4 * 4 + tid; v < a.n; v += nt) {
    a.levels[v] = (v == source) ? 0 : -1;
    if (a.parents) a.parents[v] = (v == source) ? source : -1;
  }
  // visited = rows a pull can never reach (no in-edges; padding) + source
  const int64_t sw = source >> 6;
  const uint64_t sb = 1ull << (source & 63);
  for (int64_t w = tid; w < a.nw; w += nt) {
    uint64_t vis;
    if (a.can_pull) {
      vis = a.pull.iso[w];
    } else {
      const int64_t valid = a.n - w * 64;  // bits past n are padding
      vis = valid >= 64 ? 0ull : ~mask_below((int)valid);
    }
    a.visited[w] = vis | (w == sw ? sb : 0ull);
    a.fcur[w] = w == sw ? sb : 0ull;
    f1[w] = 0ull;
    f2[w] = 0ull;
  }
  if (tid == 0) {
    for (int i = 0; i < kCntSlots; ++i) {
      a.cnt_cur[i] = 0;
      a.cnt_nxt[i] = 0;
      a.cnt_clr[i] = 0;
    }
    a.ctrl->nlev = 0;
    a.ctrl->pushed[0] = a.ctrl->pushed[1] = a.ctrl->pushed[2] = 0;
    const int ds = a.push.rp[source + 1] - a.push.rp[source];
    a.cnt_cur[0] = 1;  // level 0 = {source}
    a.cnt_cur[1] = ds;
    a.cnt_cur[2] = ds > kPushSplit ? 1 : 0;
    if (a.coop) {  // the multi-workgroup loop's first queue: {source}
      a.coop->bar = 0ull;
      for (int i = 0; i < kCoopSegsMax; ++i) a.coop->cnt[0][i] = a.coop->esum[0][i] = 0;
      a.coop->cnt[0][0] = 1;
      a.coop->esum[0][0] = ds;
      a.qv[0] = source;
      a.qe[0] = ((uint64_t)(uint32_t)ds << 32) | (uint32_t)a.push.rp[source];
    }
  }
}

// ---- multi-workgroup level loop for small frontiers -------------------------
// Level d: workgroup w takes the entries [w nc / G, (w + 1) nc / G) of the
// level's queue, a thread per entry.  The queue has one segment per wave of
// the loop; an entry is found through the prefix of the segments' counts.
// The thread writes the entry's level (deferred from the level that found
// it, so the store overlaps this level's loads), claims the targets of four
// out-edges per step with one atomicOr on their visited words (their row
// extents loaded beside), and queues the winners in its wave's segment of
// the next queue.  Entries past a segment's capacity get their level and go
// straight into the next frontier's bitmap (the loop then spills that
// frontier).  No counter is shared: each wave stores its segment's count
// and degree sum with its entries, before the barrier.
__global__ __launch_bounds__(kCoopThreads) void k_bfs_coop(BfsArgs a, int64_t max_levels,
                                                           uint64_t wait_ticks, uint64_t *F0,
                                                           uint64_t *F1, uint64_t *F2) {
  __shared__ int s_pre[kCoopSegs + 1];
  __shared__ int s_nc, s_ne, s_ovf, s_go;
  const int tid = threadIdx.x, ln = tid & 63;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  CoopCtl *cc = a.coop;
  const int w = (int)blockIdx.x;
  const int my_seg = w * (kCoopThreads / 64) + (tid >> 6);
  const int seg = a.qseg, qsize = kCoopSegs * seg;
  int64_t d = 0;
  bool spill = false;
  for (;;) {
    const int sl = (int)(d & 1);
    if (tid < 64) {  // the level's queue: segment counts, their prefix, degree sums
      // lane l holds segments kCoopSegsPerLane * l + r
      int c[kCoopSegsPerLane], csum = 0, esum = 0;
      bool over = false;
#pragma unroll
      for (int r = 0; r < kCoopSegsPerLane; ++r) {
        c[r] = ld_coherent(&cc->cnt[sl][kCoopSegsPerLane * tid + r]);
        esum += ld_coherent(&cc->esum[sl][kCoopSegsPerLane * tid + r]);
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
      const int tot = lane_last(incl), etot = wave_sum(esum);
      const bool ovf = __ballot(over) != 0ull;
      if (tid == 0) {
        s_pre[0] = 0;
        s_nc = tot;
        s_ne = etot;
        s_ovf = ovf ? 1 : 0;
      }
    }
    __syncthreads();
    const int nc = s_nc, ne = s_ne;
    if (nc == 0 || d >= max_levels) break;
    // a frontier that outgrew its segments, or one the switch rule would
    // pull, goes to the level kernel
    if (s_ovf || ne > kCoopEdges || d >= kCoopMaxLevels || decide(a, nc, ne) == GRB_DIR_PULL) {
      spill = true;
      break;
    }
    if (w == 0 && tid == 0) {
      a.ctrl->nlev = (int)d + 1;
      if (a.stats && d < kStatsCap) {
        a.stats[d * kStatFields + 0] = nc;
        a.stats[d * kStatFields + 1] = ne;
        a.stats[d * kStatFields + 2] = GRB_DIR_PUSH;
      }
    }
    const int qin = sl * qsize, qout = (sl ^ 1) * qsize + my_seg * seg;
    const int sx = (int)((d + 1) % 3);
    uint64_t *fn = sx == 0 ? F0 : (sx == 1 ? F1 : F2);
    const int lo = (int)((int64_t)nc * w / kCoopGrid);
    const int hi = (int)((int64_t)nc * (w + 1) / kCoopGrid);
    int wcnt = 0, wsum = 0;  // this wave's appends (uniform over the wave)
    for (int base = lo; base < hi; base += kCoopThreads) {
      const int i = base + tid;
      int rs = 0, dg = 0;
      if (i < hi) {
        int s = 0;  // segment holding entry i: the last s with s_pre[s] <= i
#pragma unroll
        for (int step = kCoopSegs / 2; step > 0; step >>= 1)
          if (s_pre[s + step] <= i) s += step;
        const int at = qin + s * seg + (i - s_pre[s]);
        const int v = ld_coherent(a.qv + at);
        const uint64_t e = load_relaxed_u64(a.qe + at);
        rs = (int)(uint32_t)e;
        dg = (int)(e >> 32);
        if (d > 0) a.levels[v] = (int)d;
      }
      for (int q0 = 0; __ballot(q0 < dg) != 0ull; q0 += 4) {
        int c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = q0 + q < dg ? ci[rs + q0 + q] : -1;
        uint64_t old[4];
        int r0[4], r1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          old[q] = ~0ull;
          r0[q] = r1[q] = 0;
          if (c[q] >= 0) {
            old[q] = atomicOr((unsigned long long *)&a.visited[c[q] >> 6], 1ull << (c[q] & 63));
            r0[q] = rp[c[q]];
            r1[q] = rp[c[q] + 1];
          }
        }
        bool won[4];
        int nw = 0, wdeg = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          won[q] = c[q] >= 0 && !((old[q] >> (c[q] & 63)) & 1ull);
          nw += won[q] ? 1 : 0;
          wdeg += won[q] ? r1[q] - r0[q] : 0;
        }
        const int incl = wave_incl_scan(nw);
        const int tot = lane_last(incl);
        if (tot == 0) continue;
        int slot = wcnt + incl - nw;
        wcnt += tot;
        wsum += wave_sum(wdeg);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!won[q]) continue;
          if (slot < seg) {
            st_coherent(a.qv + qout + slot, c[q]);
            store_relaxed_u64(a.qe + qout + slot,
                              ((uint64_t)(uint32_t)(r1[q] - r0[q]) << 32) | (uint32_t)r0[q]);
          } else {
            a.levels[c[q]] = (int)d + 1;
            atomicOr((unsigned long long *)&fn[c[q] >> 6], 1ull << (c[q] & 63));
          }
          ++slot;
        }
      }
    }
    // the wave's segment count and degree sum go with its entries; the
    // barrier follows once every memory operation of the workgroup is done
    if (ln == 0) {
      st_coherent(&cc->cnt[sl ^ 1][my_seg], wcnt);
      st_coherent(&cc->esum[sl ^ 1][my_seg], wsum);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) s_go = coop_barrier(&cc->bar, kCoopGrid, d, wait_ticks);
    __syncthreads();
    ++d;
    if (!s_go) {
      // barrier given up: the frontier of level d (found by every
      // workgroup before the barrier) goes to the level kernel
      spill = true;
      break;
    }
  }
  if (w == 0 && tid == 0) {
    a.ctrl->small_levels = (int)d;
    a.ctrl->spilled = spill ? 1 : 0;
  }
}

// After the loop: the frontier it left in its queue (level h =
// ctrl->small_levels, whose levels are not written yet) gets its levels;
// when the loop spilled it, it also becomes the bitmap and counters of
// level h for the level kernel (the entries past a segment's capacity are
// in the bitmap already).
__global__ __launch_bounds__(kBlock) void k_bfs_coop_handover(BfsArgs a, int32_t source,
                                                               uint64_t *F0, uint64_t *F1,
                                                               uint64_t *F2) {
  const bool spilled = a.ctrl->spilled != 0;
  const int64_t h = a.ctrl->small_levels;
  uint64_t *fh = (h % 3 == 0) ? F0 : ((h % 3 == 1) ? F1 : F2);
  const int sl = (int)(h & 1), seg = a.qseg, qsize = kCoopSegs * seg;
  const int32_t *qv = a.qv + sl * qsize;
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < qsize; t += gridDim.x * kBlock) {
    const int s = t / seg, j = t - s * seg;
    if (j < a.coop->cnt[sl][s]) {
      const int v = qv[t];
      if (h > 0) a.levels[v] = (int)h;
      if (spilled) atomicOr((unsigned long long *)&fh[v >> 6], 1ull << (v & 63));
    }
  }
  if (spilled && blockIdx.x == 0 && threadIdx.x == 0) {
    // the start kernel's source bit in F0 is the only other bit set
    // (h > 0: the source is not in this frontier)
    if (h > 0) atomicAnd((unsigned long long *)&F0[source >> 6], ~(1ull << (source & 63)));
    int nq = 0, ne = 0;
    for (int s = 0; s < kCoopSegs; ++s) {
      nq += a.coop->cnt[sl][s];
      ne += a.coop->esum[sl][s];
    }
    for (int i = 0; i < 3 * kCntSlots; ++i) a.ctrl->lists[i] = 0;
    int32_t *cnt = a.ctrl->lists + (h % 3) * kCntSlots;
    cnt[0] = nq;
    cnt[1] = ne;
    cnt[2] = 0;  // rows are at most kCoopMaxDeg long
    a.ctrl->pushed[0] = a.ctrl->pushed[1] = a.ctrl->pushed[2] = 0;  // parents: final pass
  }
}

}  // namespace

void launch_bfs_coop(const BfsArgs &a, int32_t source, int64_t max_levels, uint64_t *const F[3],
                     uint64_t wait_ticks, void *stream) {
  hipLaunchKernelGGL(k_bfs_coop, dim3(kCoopGrid), dim3(kCoopThreads), 0, (hipStream_t)stream, a,
                     max_levels, wait_ticks, F[0], F[1], F[2]);
  const int g = (kCoopSegs * a.qseg + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_bfs_coop_handover, dim3(g < 1 ? 1 : g), dim3(kBlock), 0,
                     (hipStream_t)stream, a, source, F[0], F[1], F[2]);
}

void launch_bfs_start(const BfsArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                      void *stream) {
  int64_t g = (a.n / 4 + kBlock - 1) / kBlock;
  g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
  hipLaunchKernelGGL(k_bfs_start, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, a,
                     source, f1, f2);
}

void launch_bfs_level(const BfsArgs &a, void *stream) {
  hipLaunchKernelGGL(k_bfs_level, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

void launch_bfs_parents(const BfsArgs &a, void *stream) {
  // one wave per bitmap word
  int64_t g = (a.nw + kWavesPerBlock - 1) / kWavesPerBlock;
  g = g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g);
  hipLaunchKernelGGL(k_bfs_parents, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
