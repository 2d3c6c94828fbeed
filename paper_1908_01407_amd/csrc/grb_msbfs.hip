// Batched multi-source BFS: k traversals at once as a masked sparse matrix
// times bitmask-block product, next = (A^T or.and F) and not V (the paper's
// multi-nodeset traversal with mxm, Table 6 and Section 3.3; matrix-matrix
// direction optimisation is its stated future work, Section 9).
//
// F (frontier) and V (visited) are n x W blocks of uint64 words, vertex
// major: word j of vertex v holds queries 64j .. 64j+63.  A level runs one
// kernel over a 2-D grid: blockIdx.y picks a tile of kt query words.
// * pull: each wave owns 64 consecutive vertices; for the tile's words of
//   every vertex with an unvisited query, the in-edges are streamed as one
//   concatenated list, 64 per step, and the neighbours' frontier words are
//   OR-reduced per row with a segmented scan; a row stops as soon as every
//   unvisited query of the tile is found (early exit of the Boolean
//   semiring, per query word);
// * push: each wave owns one word of the "active vertex" bitmap; the
//   out-edges of active rows are streamed the same way and each target is
//   claimed with atomicOr on its visited word, so every (vertex, query) is
//   discovered exactly once; rows longer than kPushSplit use the static
//   256-edge pieces;
// * discoveries write their level (vertex-major output, coalesced per row)
//   and set the next frontier and the next active bitmap; frontier sizes
//   for the device-side direction choice go to striped counters.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

__device__ __forceinline__ uint64_t wave_seg_or(uint64_t x, int row) {
  return wave_seg_scan(x, row, (uint64_t)0, OpOr());
}

// valid queries of word j (the last word may be partial)
__device__ __forceinline__ uint64_t qmask(const MsbfsArgs &a, int j) {
  const int rem = (int)(a.k - (int64_t)j * 64);
  return rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
}

// Direction for the whole batch: the paper's rule on the frontier's
// (vertex, query) pairs against n*k, or the exact rule on the out-edges of
// the active (vertex, query word) pairs against nnz per word.
__device__ __forceinline__ int ms_decide(const MsbfsArgs &a, int64_t active, int64_t edges) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  const bool pull = a.rule == GRB_SWITCH_EXACT
                        ? (int64_t)a.denom * edges > a.nnz * (int64_t)a.W
                        : (int64_t)a.denom * active > a.n * a.k;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

// Writes level d+1 for the new bits of (v, word j) held by each lane:
// the wave visits every lane with new bits and stores its 64 levels with
// one coalesced store.
// In a session the level is relative to the query's start level, and the
// new bits are ORed into the workgroup's per-word "has a frontier bit"
// words (s_alive, indexed by word - first word of the pass).
__device__ __forceinline__ void write_levels(const MsbfsArgs &a, int64_t v, int j,
                                             uint64_t newbits, unsigned long long *s_alive) {
  const int ln = threadIdx.x & 63;
  uint64_t todo = __ballot(newbits != 0ull);
  const int j0 = blockIdx.y * a.kt;
  while (todo) {
    const int r = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const int64_t rv = __shfl(v, r);
    const int rj = __shfl(j, r);
    const uint64_t nb = __shfl(newbits, r);
    const int64_t q = (int64_t)rj * 64 + ln;
    if (((nb >> ln) & 1ull) && q < a.k)
      a.levels[rv * a.k + q] = a.d + 1 - (a.start ? a.start[q] : 0);
    if (a.alive_nxt && ln == 0) atomicOr(&s_alive[rj - j0], (unsigned long long)nb);
  }
}

// Claim the query bits `bits` of vertex v, word j, for the next level.
__device__ __forceinline__ uint64_t claim_bits(const MsbfsArgs &a, int64_t v, int j, uint64_t bits,
                                               int64_t &edges_acc) {
  if (bits == 0ull) return 0ull;
  uint64_t *vw = &a.V[v * a.W + j];
  bits &= ~*vw;  // plain read: a filter, the atomic decides
  if (bits == 0ull) return 0ull;
  const uint64_t old = atomicOr((unsigned long long *)vw, (unsigned long long)bits);
  const uint64_t nb = bits & ~old;
  if (nb) {
    const uint64_t pf = atomicOr((unsigned long long *)&a.Fn[v * a.W + j], (unsigned long long)nb);
    if (pf == 0ull) edges_acc += a.push.rp[v + 1] - a.push.rp[v];
    atomicOr((unsigned long long *)&a.actn[v >> 6], 1ull << (v & 63));
  }
  return nb;
}

// Pull over the pass's query words j0 .. j0 + nj - 1 (nj <= L <= 8): an edge
// occupies L consecutive lanes, one per query word, so the frontier words of
// a neighbour (consecutive in the vertex-major block) come in one coalesced
// load; S = 64 / L edges per sub-step, kUnroll sub-steps per step.  Rows
// (lanes of the row layout, 64 per bitmap word) keep their unvisited and
// found bits per word and stop once every unvisited query of the pass is
// found.  Rows longer than kPushSplit are left to the pieces below, which
// claim with atomics like push.
template <int L>
__device__ void ms_pull_rows(const MsbfsArgs &a, int *mark, int64_t &act_acc,
                             int64_t &edges_acc, unsigned long long *s_alive) {
  constexpr int S = 64 / L;
  const int ln = threadIdx.x & 63;
  const int sl = ln / L, jl = ln % L;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const int j0 = blockIdx.y * a.kt;
  const int nj = min(a.kt, a.W - j0);
  const bool jv = jl < nj;
  for (int64_t part = gw; part < kWaveParts; part += nwaves) {
    const int64_t wlo = a.pull.wpart[part], whi = a.pull.wpart[part + 1];
    for (int64_t w = wlo; w < whi; ++w) {
      const int64_t v = w * 64 + ln;
      const bool inb = v < a.n;
      int rs = 0, re = 0;
      if (inb) {
        rs = rp[v];
        re = rp[v + 1];
        if (re - rs > kPushSplit) re = rs;  // pieces
      }
      uint64_t need[L], acc[L];
      bool any = false;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        need[q] = 0ull;
        acc[q] = 0ull;
        if (q < nj && re > rs) need[q] = ~a.V[v * a.W + j0 + q] & qmask(a, j0 + q);
        any |= need[q] != 0ull;
      }
      if (__ballot(any) == 0ull) continue;
      int cur = rs;
      const int end = any ? re : rs;
      bool done = !any;
      for (bool more = true; more;) {
        // slot positions of kUnroll sub-steps (S edges each)
        int pos[kUnroll], row[kUnroll], se[kUnroll];
        bool st[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          pos[u] = -1;
          row[u] = 0;
          se[u] = 0;
          st[u] = false;
          if (!more) continue;
          const int len = done ? 0 : end - cur;
          const int incl = wave_incl_scan(len);
          const int total = lane_last(incl);
          if (total == 0) {
            more = false;
            continue;
          }
          const int excl = incl - len;
          const bool starts = len > 0 && excl < S;
          const int rr = slot_rows(mark, starts, excl);  // row of slot ln (ln < S used)
          const int r = __shfl(rr, sl);                 // row of this lane's slot
          const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
          if (sl < total) pos[u] = rcur + (sl - rexcl);
          row[u] = r;
          st[u] = starts;
          se[u] = min(incl, S);
          if (starts) cur += se[u] - excl;
        }
        uint64_t f[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int c = pos[u] >= 0 ? ci[pos[u]] : -1;
          f[u] = (c >= 0 && jv) ? a.F[(int64_t)c * a.W + j0 + jl] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          // OR over the slots of each row, per query word (lanes L apart)
          uint64_t x = f[u];
#pragma unroll
          for (int off = L; off < 64; off <<= 1) {
            const uint64_t y = __shfl_up(x, off);
            const int ry = __shfl_up(row[u], off);
            if (ln >= off && ry == row[u]) x |= y;
          }
          // the row's lane takes the OR from the last slot of its segment
          const int last = st[u] ? se[u] - 1 : 0;
#pragma unroll
          for (int q = 0; q < L; ++q) {
            const uint64_t segv = __shfl(x, last * L + q);
            if (st[u]) acc[q] |= segv;
          }
        }
        bool all = true;
#pragma unroll
        for (int q = 0; q < L; ++q) all &= (acc[q] & need[q]) == need[q];
        done = done || all;
      }
      // found bits: this wave owns row v in pull
      bool anyb = false;
      int64_t e_add = 0;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const uint64_t nb = acc[q] & need[q];
        if (nb) {
          a.V[v * a.W + j0 + q] |= nb;
          a.Fn[v * a.W + j0 + q] = nb;
          act_acc += __popcll(nb);
          anyb = true;
          e_add += a.push.rp[v + 1] - a.push.rp[v];
        }
        write_levels(a, v, j0 + q, nb, s_alive);
      }
      edges_acc += e_add;
      const uint64_t ab = __ballot(anyb);
      if (ab && ln == 0) atomicOr((unsigned long long *)&a.actn[w], (unsigned long long)ab);
    }
  }
  // pieces of long rows: OR of the piece's neighbours' frontier words, then
  // claims like push (kPushSplit edges: S per sub-step)
  for (int64_t h = gw; h < a.pull.nsplit; h += nwaves) {
    const int r = a.pull.split[2 * h], b = a.pull.split[2 * h + 1];
    const int e = min(b + kPushSplit, rp[r + 1]);
    uint64_t need = 0ull;
    if (jv) need = ~a.V[(int64_t)r * a.W + j0 + jl] & qmask(a, j0 + jl);
    if (__ballot(need != 0ull) == 0ull) continue;
    uint64_t acc = 0ull;
    for (int base = b; base < e; base += S * kUnroll) {
      uint64_t f[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int p = base + u * S + sl;
        const int c = p < e ? ci[p] : -1;
        f[u] = (c >= 0 && jv) ? a.F[(int64_t)c * a.W + j0 + jl] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc |= f[u];
      if (__ballot((acc & need) != need) == 0ull) break;  // every word complete
    }
    // OR over the slots (lanes L apart) and claim in lanes 0 .. L-1
#pragma unroll
    for (int off = L; off < 64; off <<= 1) acc |= __shfl_xor(acc, off);
    int64_t ea = 0;
    uint64_t nb = 0ull;
    if (sl == 0 && jv) nb = claim_bits(a, r, j0 + jl, acc & need, ea);
    act_acc += sl == 0 ? __popcll(nb) : 0;
    edges_acc += ea;
    write_levels(a, sl == 0 ? (int64_t)r : -1, j0 + jl, sl == 0 ? nb : 0ull, s_alive);
  }
}

__device__ void ms_pull(const MsbfsArgs &a, int *mark, int64_t &act_acc, int64_t &edges_acc,
                        unsigned long long *s_alive) {
  if (a.kt <= 1) ms_pull_rows<1>(a, mark, act_acc, edges_acc, s_alive);
  else if (a.kt <= 2) ms_pull_rows<2>(a, mark, act_acc, edges_acc, s_alive);
  else if (a.kt <= 4) ms_pull_rows<4>(a, mark, act_acc, edges_acc, s_alive);
  else ms_pull_rows<8>(a, mark, act_acc, edges_acc, s_alive);
}

__device__ void ms_push(const MsbfsArgs &a, int *mark, int64_t &act_acc, int64_t &edges_acc,
                        unsigned long long *s_alive) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.push.rp, *ci = a.push.ci;
  const int j0 = blockIdx.y * a.kt;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const uint64_t aw = a.act[w];
    if (aw == 0ull) continue;
    const int64_t u = w * 64 + ln;
    int rs = 0, re = 0;
    if ((aw >> ln) & 1ull) {
      rs = rp[u];
      re = rp[u + 1];
      if (re - rs > kPushSplit) re = rs;  // long rows: static pieces below
    }
    for (int jj = 0; jj < a.kt; ++jj) {
      const int j = j0 + jj;
      if (j >= a.W) break;
      const uint64_t fu = (re > rs) ? a.F[u * a.W + j] : 0ull;
      int cur = rs;
      const int end = fu ? re : rs;
      for (;;) {
        const int len = end - cur;
        const int incl = wave_incl_scan(len);
        const int total = lane_last(incl);
        if (total == 0) break;
        const int excl = incl - len;
        const bool starts = len > 0 && excl < 64;
        const int r = slot_rows(mark, starts, excl);
        const int rcur = __shfl(cur, r), rexcl = __shfl(excl, r);
        const uint64_t rf = __shfl(fu, r);
        int64_t tv = -1;
        uint64_t nb = 0ull;
        if (ln < total) {
          tv = ci[rcur + (ln - rexcl)];
          nb = claim_bits(a, tv, j, rf, edges_acc);
          act_acc += __popcll(nb);
        }
        write_levels(a, tv, j, nb, s_alive);
        if (starts) cur += min(incl, 64) - excl;
      }
    }
  }
  // static pieces of long rows, spread over the waves (wave gw owns pieces
  // gw, gw + nwaves, ...), 64 tested per step
  for (int64_t hb = gw; hb < a.push.nsplit; hb += 64 * nwaves) {
    const int64_t h = hb + (int64_t)ln * nwaves;
    int u = -1, b = 0, e = 0;
    if (h < a.push.nsplit) {
      u = a.push.split[2 * h];
      b = a.push.split[2 * h + 1];
      if (bit_of(a.act, u)) e = min(b + kPushSplit, rp[u + 1]);
      else u = -1;
    }
    uint64_t act = __ballot(u >= 0);
    while (act) {
      const int kk = __ffsll((unsigned long long)act) - 1;
      act &= act - 1;
      const int pu = __shfl(u, kk), pb = __shfl(b, kk), pe = __shfl(e, kk);
      for (int jj = 0; jj < a.kt; ++jj) {
        const int j = j0 + jj;
        if (j >= a.W) break;
        const uint64_t fu = a.F[(int64_t)pu * a.W + j];
        if (fu == 0ull) continue;
        for (int base = pb; base < pe; base += 64) {
          const int pos = base + ln;
          int64_t tv = -1;
          uint64_t nb = 0ull;
          if (pos < pe) {
            tv = ci[pos];
            nb = claim_bits(a, tv, j, fu, edges_acc);
            act_acc += __popcll(nb);
          }
          write_levels(a, tv, j, nb, s_alive);
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ms_level(MsbfsArgs a) {
  __shared__ int s_mark[kWavesPerBlock][64];
  __shared__ int64_t s_act, s_edges;
  __shared__ int64_t s_red[kWavesPerBlock][2];
  __shared__ unsigned long long s_alive[kMsMaxWordsPerPass];
  const bool leader = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  if (threadIdx.x < kMsMaxWordsPerPass) s_alive[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    int64_t c = 0, e = 0;
    for (int t = 0; t < kCntStripes; ++t) {
      c += a.cnt_cur[2 * t];
      e += a.cnt_cur[2 * t + 1];
    }
    s_act = c;
    s_edges = e;
    if (leader) {
      for (int i = 0; i < 2 * kCntStripes; ++i) a.cnt_clr[i] = 0;
      if (a.alive_clr)
        for (int j = 0; j < a.W; ++j) a.alive_clr[j] = 0ull;
      if (c > 0) {
        a.ctrl->nlev = a.d + 1;
        if (a.stats && a.d < kStatsCap) {
          a.stats[a.d * kStatFields + 0] = c;
          a.stats[a.d * kStatFields + 1] = e;
          a.stats[a.d * kStatFields + 2] = ms_decide(a, c, e);
        }
      }
    }
  }
  __syncthreads();
  // clear the frontier block two levels ahead: only rows its active bitmap
  // marks can be non-zero; tile 0 clears all words of those rows, then the
  // bitmap word (the same thread reads and clears it, no other tile reads it)
  if (blockIdx.y == 0) {
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < a.nw;
         w += (int64_t)gridDim.x * kBlock) {
      uint64_t aw = a.actc[w];
      if (aw == 0ull) continue;
      while (aw) {
        const int b = __ffsll((unsigned long long)aw) - 1;
        aw &= aw - 1;
        uint64_t *row = a.Fc + (w * 64 + b) * a.W;
        for (int j = 0; j < a.W; ++j) row[j] = 0ull;
      }
      a.actc[w] = 0ull;
    }
  }
  if (s_act == 0) return;
  const int dir = ms_decide(a, s_act, s_edges);
  int64_t act_acc = 0, edges_acc = 0;
  if (dir == GRB_DIR_PUSH) ms_push(a, s_mark[threadIdx.x >> 6], act_acc, edges_acc, s_alive);
  else ms_pull(a, s_mark[threadIdx.x >> 6], act_acc, edges_acc, s_alive);
  act_acc = wave_sum64(act_acc);
  const int64_t ed = wave_sum64(edges_acc);
  if ((threadIdx.x & 63) == 0) {
    s_red[threadIdx.x >> 6][0] = act_acc;
    s_red[threadIdx.x >> 6][1] = ed;
  }
  __syncthreads();
  if (a.alive_nxt && threadIdx.x < kMsMaxWordsPerPass) {
    const int j = blockIdx.y * a.kt + threadIdx.x;
    const unsigned long long x = s_alive[threadIdx.x];
    if (x && j < a.W) atomicOr(&a.alive_nxt[j], x);
  }
  if (threadIdx.x == 0) {
    int64_t c = 0, e = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      c += s_red[i][0];
      e += s_red[i][1];
    }
    if (c) {
      const int t = (blockIdx.x + blockIdx.y * 7) % kCntStripes;
      atomicAdd((unsigned long long *)&a.cnt_nxt[2 * t], (unsigned long long)c);
      atomicAdd((unsigned long long *)&a.cnt_nxt[2 * t + 1], (unsigned long long)e);
    }
  }
}

// levels = -1, blocks zeroed, sources set
__global__ void k_ms_start(MsbfsArgs a, const int32_t *sources, uint64_t *F1, uint64_t *F2,
                           uint64_t *act1, uint64_t *act2) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t nk = a.n * (int64_t)a.k;
  for (int64_t i = gt; i < nk; i += nt) a.levels[i] = -1;
  const int64_t nb = a.n * (int64_t)a.W;
  for (int64_t i = gt; i < nb; i += nt) {
    a.V[i] = ~qmask(a, (int)(i % a.W));  // queries beyond k count as visited
    a.F[i] = 0ull;
    F1[i] = 0ull;
    F2[i] = 0ull;
  }
  for (int64_t i = gt; i < a.nw; i += nt) {
    a.act[i] = 0ull;
    act1[i] = 0ull;
    act2[i] = 0ull;
  }
  if (gt == 0) {
    for (int i = 0; i < 6 * kCntStripes; ++i) a.cnt_base[i] = 0;
    a.ctrl->nlev = 0;
    a.ctrl->error = 0;
  }
}

// Session start: every query idle, i.e. all of V set (an idle query has
// visited everything, so it never claims); frontier blocks, active
// bitmaps, counters and the three "has a frontier bit" arrays cleared.  The
// level block is not touched: a query's levels are valid where its V bit is.
__global__ void k_ms_session_init(MsbfsArgs a, uint64_t *F1, uint64_t *F2, uint64_t *act1,
                                  uint64_t *act2, unsigned long long *alive3) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  const int64_t nb = a.n * (int64_t)a.W;
  for (int64_t i = gt; i < nb; i += nt) {
    a.V[i] = ~0ull;
    a.F[i] = 0ull;
    F1[i] = 0ull;
    F2[i] = 0ull;
  }
  for (int64_t i = gt; i < a.nw; i += nt) {
    a.act[i] = 0ull;
    act1[i] = 0ull;
    act2[i] = 0ull;
  }
  for (int64_t i = gt; i < 3 * (int64_t)a.W; i += nt) alive3[i] = 0ull;
  if (gt == 0) {
    for (int i = 0; i < 6 * kCntStripes; ++i) a.cnt_base[i] = 0;
    a.ctrl->nlev = 0;
    a.ctrl->error = 0;
  }
}

// Joining queries: their bits cleared in every vertex's V word (clr[j]
// holds the joining queries of word j)
__global__ void k_ms_session_clear(MsbfsArgs a, const uint64_t *clr) {
  const int64_t nb = a.n * (int64_t)a.W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = clr[i % a.W];
    if (m) a.V[i] &= ~m;
  }
}

// ... then each starts at its source at the current level a.d (lanes and
// sources checked on the host)
__global__ void k_ms_session_sources(MsbfsArgs a, const int32_t *lanes, const int32_t *sources,
                                     int32_t count, int32_t *start,
                                     unsigned long long *alive_cur) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t q = lanes[i], s = sources[i];
  if (q < 0 || q >= a.k || s < 0 || s >= a.n) return;
  const int j = (int)(q >> 6);
  const uint64_t bit = 1ull << (q & 63);
  atomicOr((unsigned long long *)&a.V[s * a.W + j], (unsigned long long)bit);
  const uint64_t pf = atomicOr((unsigned long long *)&a.F[s * a.W + j], (unsigned long long)bit);
  atomicOr((unsigned long long *)&a.act[s >> 6], 1ull << (s & 63));
  a.levels[s * a.k + q] = 0;
  start[q] = a.d;
  atomicOr(&alive_cur[j], (unsigned long long)bit);
  atomicAdd((unsigned long long *)&a.cnt_cur[0], 1ull);
  if (pf == 0ull)
    atomicAdd((unsigned long long *)&a.cnt_cur[1],
              (unsigned long long)(a.push.rp[s + 1] - a.push.rp[s]));
}

// out[i * n + v]: level of query lanes[i] at v, -1 where it has not visited v
__global__ void k_ms_session_extract(MsbfsArgs a, const int32_t *lanes, int32_t count,
                                     int32_t *out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    for (int i = 0; i < count; ++i) {
      const int64_t q = lanes[i];
      if (q < 0 || q >= a.k) continue;
      const bool seen = (a.V[v * a.W + (q >> 6)] >> (q & 63)) & 1ull;
      out[(int64_t)i * a.n + v] = seen ? a.levels[v * a.k + q] : -1;
    }
  }
}

__global__ void k_ms_sources(MsbfsArgs a, const int32_t *sources) {
  // one thread per query: serial over nothing, so duplicates are fine
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.k) return;
  const int64_t s = sources[q];
  if (s < 0 || s >= a.n) {  // reported by the driver; nothing is written for it
    atomicOr(&a.ctrl->error, 1);
    return;
  }
  const int j = (int)(q >> 6);
  const uint64_t bit = 1ull << (q & 63);
  atomicOr((unsigned long long *)&a.V[s * a.W + j], (unsigned long long)bit);
  const uint64_t pf = atomicOr((unsigned long long *)&a.F[s * a.W + j], (unsigned long long)bit);
  atomicOr((unsigned long long *)&a.act[s >> 6], 1ull << (s & 63));
  a.levels[s * a.k + q] = 0;
  atomicAdd((unsigned long long *)&a.cnt_cur[0], 1ull);
  if (pf == 0ull)
    atomicAdd((unsigned long long *)&a.cnt_cur[1],
              (unsigned long long)(a.push.rp[s + 1] - a.push.rp[s]));
}

}  // namespace

void launch_msbfs_start(const MsbfsArgs &a, const int32_t *sources, uint64_t *F1, uint64_t *F2,
                        uint64_t *act1, uint64_t *act2, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_ms_start, dim3(2048), dim3(256), 0, s, a, sources, F1, F2, act1, act2);
  const int g = (int)((a.k + 255) / 256);
  hipLaunchKernelGGL(k_ms_sources, dim3(g < 1 ? 1 : g), dim3(256), 0, s, a, sources);
}

void launch_msbfs_session_init(const MsbfsArgs &a, uint64_t *F1, uint64_t *F2, uint64_t *act1,
                               uint64_t *act2, unsigned long long *alive3, void *stream) {
  hipLaunchKernelGGL(k_ms_session_init, dim3(2048), dim3(256), 0, (hipStream_t)stream, a, F1, F2,
                     act1, act2, alive3);
}

void launch_msbfs_session_join(const MsbfsArgs &a, const int32_t *lanes, const int32_t *sources,
                               int32_t count, const uint64_t *clr, int32_t *start,
                               unsigned long long *alive_cur, void *stream) {
  if (count <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_ms_session_clear, dim3(2048), dim3(256), 0, s, a, clr);
  hipLaunchKernelGGL(k_ms_session_sources, dim3((count + 255) / 256), dim3(256), 0, s, a, lanes,
                     sources, count, start, alive_cur);
}

void launch_msbfs_session_extract(const MsbfsArgs &a, const int32_t *lanes, int32_t count,
                                  int32_t *out, void *stream) {
  if (count <= 0 || a.n <= 0) return;
  int64_t g = (a.n + 255) / 256;
  g = g > 4096 ? 4096 : g;
  hipLaunchKernelGGL(k_ms_session_extract, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, a,
                     lanes, count, out);
}

void launch_msbfs_level(const MsbfsArgs &a, int grid_x, void *stream) {
  const int tiles = (a.W + a.kt - 1) / a.kt;
  hipLaunchKernelGGL(k_ms_level, dim3(grid_x, tiles), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
