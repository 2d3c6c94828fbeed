// HIP kernels for gfx950 (CDNA4, wave64): frontier compaction, push
// (SpMSpV) and pull (masked SpMV) expansion for SSSP, and small utility
// kernels.  BFS lives in grb_bfs.hip, PageRank in grb_spmv.hip and the
// generic masked products in grb_mxv.hip.
//
// Design notes (prior art in the paper: Sections 4-6; the kernels below are
// written for this hardware, not translated):
// * Frontiers are kept both as a presence bitmap (one uint64 word per 64
//   vertices: exactly one wave64 ballot) and as a sorted vertex list with an
//   exclusive prefix of degrees.  The compaction kernel builds the list from
//   the bitmap in one pass with a decoupled look-back scan.
// * Push walks the list with merge-path tiles over (entries + edges), so a
//   hub's edges are spread over many workgroups; the mask test is fused into
//   the scatter (bitmap atomicOr, atomicMin for parents / distances).
// * Pull gives each wave one bitmap word of candidate rows and walks their
//   adjacency as one concatenated stream, 64 edges per step (a wave-level
//   load-balanced search): a row drops out as soon as it finds a frontier
//   neighbour (early exit of the Boolean semiring).  Rows longer than
//   kHeavyDeg are split into fixed pieces processed by any wave.
// * The push/pull decision is made on the device from the compaction's
//   counts, so a whole BFS level runs without a host round trip.
#include <hip/hip_runtime.h>

#include "grb_internal.h"
#include "grb_device.h"

namespace grb {
namespace {

// ---------------------------------------------------------------------------
// compaction: bitmap -> sorted list, degree prefix, merge-path tile starts
// ---------------------------------------------------------------------------

constexpr uint64_t kFlagAgg = 1, kFlagPre = 2;

__device__ __forceinline__ uint64_t pack_status(uint64_t flag, int64_t c, int64_t d) {
  return (flag << 62) | ((uint64_t)c << 31) | (uint64_t)d;
}
__device__ __forceinline__ int64_t status_cnt(uint64_t s) { return (int64_t)((s >> 31) & 0x7fffffffull); }
__device__ __forceinline__ int64_t status_deg(uint64_t s) { return (int64_t)(s & 0x7fffffffull); }

// Each workgroup (16 waves) compacts 256 bitmap words; its position in the
// output comes from a decoupled look-back over the workgroups before it
// (tickets, not blockIdx, order the workgroups, so every workgroup a
// look-back waits on is already running).  The status word packs
// flag (2 bits) | count (31 bits) | degree sum (31 bits).
template <int MODE>
__global__ __launch_bounds__(kCompactThreads) void k_compact(CompactArgs a) {
  constexpr int NWV = kCompactThreads / 64;  // waves per workgroup
  constexpr int WPW = kCompactWords / NWV;   // words per wave
  __shared__ int s_cnt[kCompactWords];
  __shared__ int s_deg[kCompactWords];
  __shared__ int s_blk;
  __shared__ int s_base_c, s_base_d;
  const int tid = threadIdx.x, wid = tid >> 6, ln = tid & 63;
  // once a frontier is empty every later one is: nothing to compact
  if (a.skip_if_empty && a.ctrl->count == 0) return;
  if (tid == 0) s_blk = atomicAdd(&a.ctrl->ticket, 1);
  __syncthreads();
  const int blk = s_blk;
  const int64_t w0 = (int64_t)blk * kCompactWords + wid * WPW;
  if (tid == 0) a.status_next[blk] = 0ull;

#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int64_t w = w0 + k;
    const uint64_t word = w < a.nw ? a.nb[w] : 0ull;
    int deg = 0;
    if ((word >> ln) & 1ull) {
      const int64_t v = w * 64 + ln;
      if (a.rp) deg = a.rp[v + 1] - a.rp[v];
    }
    const int ds = wave_sum(deg);
    if (ln == 0) {
      s_cnt[wid * WPW + k] = __popcll(word);
      s_deg[wid * WPW + k] = ds;
      if (a.clear && w < a.nw) a.clear[w] = 0ull;
    }
  }
  __syncthreads();

  if (wid == 0) {
    // block-wide exclusive scan: lane l covers words 4l .. 4l+3
    int c[4], d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c[i] = s_cnt[4 * ln + i];
      d[i] = s_deg[4 * ln + i];
    }
    const int cl = c[0] + c[1] + c[2] + c[3], dl = d[0] + d[1] + d[2] + d[3];
    const int ci = wave_incl_scan(cl), di = wave_incl_scan(dl);
    const int ctot = __shfl(ci, 63), dtot = __shfl(di, 63);
    int ce = ci - cl, de = di - dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s_cnt[4 * ln + i] = ce;
      s_deg[4 * ln + i] = de;
      ce += c[i];
      de += d[i];
    }
    int64_t ec = 0, ed = 0;
    if (blk > 0) {
      if (ln == 0) store_relaxed_u64(&a.status_cur[blk], pack_status(kFlagAgg, ctot, dtot));
      int jhi = blk - 1;
      for (;;) {  // window of 128 predecessors, nearest first
        const int j1 = jhi - ln, j2 = jhi - 64 - ln;
        uint64_t s1 = pack_status(kFlagPre, 0, 0), s2 = s1;
        if (j1 >= 0) {
          do { s1 = load_relaxed_u64(&a.status_cur[j1]); } while ((s1 >> 62) == 0);
        }
        if (j2 >= 0) {
          do { s2 = load_relaxed_u64(&a.status_cur[j2]); } while ((s2 >> 62) == 0);
        }
        const uint64_t p1 = __ballot((s1 >> 62) == kFlagPre);
        const uint64_t p2 = __ballot((s2 >> 62) == kFlagPre);
        const int f1 = p1 ? (__ffsll((unsigned long long)p1) - 1) : 64;
        ec += wave_sum64(ln <= f1 ? status_cnt(s1) : 0);
        ed += wave_sum64(ln <= f1 ? status_deg(s1) : 0);
        if (p1) break;
        const int f2 = p2 ? (__ffsll((unsigned long long)p2) - 1) : 64;
        ec += wave_sum64(ln <= f2 ? status_cnt(s2) : 0);
        ed += wave_sum64(ln <= f2 ? status_deg(s2) : 0);
        if (p2) break;
        jhi -= 128;
      }
    }
    if (ln == 0) {
      store_relaxed_u64(&a.status_cur[blk], pack_status(kFlagPre, ec + ctot, ed + dtot));
      s_base_c = (int)ec;
      s_base_d = (int)ed;
      if (blk == (int)gridDim.x - 1) {
        const int64_t cnt = ec + ctot, sd = ed + dtot;
        a.ctrl->count = (int)cnt;
        a.ctrl->sumdeg = (int)sd;
        const int64_t nt = (cnt + sd + kPushTile - 1) / kPushTile;
        a.ctrl->ntiles = (int)nt;
        if (a.tiles && cnt > 0) a.tiles[nt] = (int)(cnt - 1);
        if (MODE != kCompactPlain && cnt > 0) a.ctrl->nlev = a.lev + 1;
        a.ctrl->ticket = 0;
      }
    }
  }
  __syncthreads();

  const int bc = s_base_c, bd = s_base_d;
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int64_t w = w0 + k;
    const uint64_t word = w < a.nw ? a.nb[w] : 0ull;
    if (word == 0ull) continue;
    const bool bit = (word >> ln) & 1ull;
    const int rank = __popcll(word & mask_below(ln));
    const int64_t v = w * 64 + ln;
    int deg = 0, rs = 0;
    if (bit && a.rp) {  // second read of the same row extents: a cache hit
      rs = a.rp[v];
      deg = a.rp[v + 1] - rs;
    }
    const int dinc = wave_incl_scan(deg);
    const int idx = bc + s_cnt[wid * WPW + k] + rank;
    const int dex = bd + s_deg[wid * WPW + k] + dinc - deg;
    if (bit) {
      if (a.list) a.list[idx] = (int)v;
      if (a.degpre) a.degpre[idx] = dex;
      if (a.rowstart) a.rowstart[idx] = rs;
      if (a.tiles) {
        const int64_t s0 = (int64_t)dex + idx, s1 = s0 + deg;
        for (int64_t t = (s0 + kPushTile - 1) / kPushTile; t * kPushTile <= s1; ++t)
          a.tiles[t] = idx;
      }
      if (MODE == kCompactBfs) a.levels[v] = a.lev;
      if (MODE == kCompactSssp) {
        const float dv = a.dist[v];
        a.fval[v] = dv;
        a.lval[idx] = dv;
      }
    }
    if (MODE == kCompactBfs && ln == 0) a.visited[w] |= word;
  }
}

// ---------------------------------------------------------------------------
// direction decision (Table 5 / Section 4.4.1 of the paper)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int decide_dir(const TravArgs &a, int count, int sumdeg) {
  if (a.forced) return a.forced;
  if (!a.can_pull) return GRB_DIR_PUSH;
  if (!a.can_push) return GRB_DIR_PULL;
  const bool pull = a.rule == GRB_SWITCH_EXACT ? (int64_t)a.denom * sumdeg > a.nnz
                                               : (int64_t)a.denom * count > a.n;
  return pull ? GRB_DIR_PULL : GRB_DIR_PUSH;
}

__device__ __forceinline__ void record_stats(const TravArgs &a, int count, int sumdeg, int dir) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctrl->dir = dir;
    if (a.stats && a.d < kStatsCap) {
      a.stats[a.d * kStatFields + 0] = count;
      a.stats[a.d * kStatFields + 1] = sumdeg;
      a.stats[a.d * kStatFields + 2] = dir;
    }
  }
}

// Stages the list entries of merge-path tile t into LDS; returns the number
// of staged entries and the tile's edge range [e0, e1).
struct PushStage {
  int deg[kPushTile + 1];  // exclusive degree prefix
  int u[kPushTile + 1];    // vertex
  int rs[kPushTile + 1];   // row start in the push CSR
  float val[kPushTile + 1];
};

template <bool VAL>
__device__ __forceinline__ int stage_tile(PushStage &st, const TravArgs &a, int t, int sumdeg,
                                          int64_t &e0, int64_t &e1) {
  const int i0 = a.tiles[t], i1 = a.tiles[t + 1];
  const int ne = i1 - i0 + 1;
  for (int k = threadIdx.x; k < ne; k += kBlock) {
    const int u = a.list[i0 + k];
    st.u[k] = u;
    st.deg[k] = a.degpre[i0 + k];
    st.rs[k] = a.rowstart[i0 + k];
    if (VAL) st.val[k] = a.lval[i0 + k];
  }
  e0 = (int64_t)t * kPushTile - i0;
  e1 = (int64_t)(t + 1) * kPushTile - i1;
  if (e1 > sumdeg) e1 = sumdeg;
  __syncthreads();
  return ne;
}

// index of the staged entry holding edge e: largest k with deg[k] <= e
__device__ __forceinline__ int find_entry(const PushStage &st, int ne, int64_t e) {
  int lo = 0, hi = ne - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st.deg[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void set_bit_guarded(uint64_t *bm, int64_t v) {
  const uint64_t b = 1ull << (v & 63);
  if (!(bm[v >> 6] & b)) atomicOr((unsigned long long *)&bm[v >> 6], (unsigned long long)b);
}

// ---------------------------------------------------------------------------
// SSSP (Bellman-Ford over min-plus with an improved-vertex frontier)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_sssp_init(TravArgs a, int32_t source, uint64_t *iso,
                                                      uint64_t *fa, uint64_t *fb, uint64_t *status,
                                                      int64_t nstatus) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const int64_t v = w * 64 + ln;
    bool isov = true;
    if (v < a.n) {
      isov = a.can_pull ? (a.pull.rp[v + 1] == a.pull.rp[v]) : false;
      a.dist[v] = (v == source) ? 0.0f : __int_as_float(0x7f800000);
    }
    const uint64_t isom = __ballot(isov);
    if (ln == 0) {
      iso[w] = isom;
      fa[w] = 0ull;
      fb[w] = (w == (source >> 6)) ? (1ull << (source & 63)) : 0ull;
    }
  }
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t i = gt; i < nstatus; i += (int64_t)gridDim.x * kBlock) status[i] = 0ull;
  if (gt == 0) {
    Ctrl c = {};
    *a.ctrl = c;
  }
}

__device__ void sssp_push(const TravArgs &a, PushStage &st, int sumdeg) {
  const int ntiles = a.ctrl->ntiles;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int64_t e0, e1;
    const int ne = stage_tile<true>(st, a, t, sumdeg, e0, e1);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
      const int k = find_entry(st, ne, e);
      const int64_t pos = st.rs[k] + (e - st.deg[k]);
      const int v = a.push.ci[pos];
      const float nd = st.val[k] + a.wpush[pos];
      if (nd < a.dist[v]) {
        const int old = atomicMin((int *)&a.dist[v], __float_as_int(nd));
        if (nd < __int_as_float(old)) set_bit_guarded(a.fnxt, v);
      }
    }
    __syncthreads();
  }
}

__device__ void sssp_pull(const TravArgs &a, int *mark) {
  const int ln = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t *rp = a.pull.rp, *ci = a.pull.ci;
  const float inf = __int_as_float(0x7f800000);
  for (int64_t w = gw; w < a.nw; w += nwaves) {
    const uint64_t cand = ~a.visited[w];  // non-isolated vertices
    if (cand == 0ull) continue;
    const int64_t v = w * 64 + ln;
    bool act = (cand >> ln) & 1ull;
    int cur = 0, end = 0;
    if (act) {
      cur = rp[v];
      end = rp[v + 1];
      if (end - cur > kHeavyDeg) act = false;
    }
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
      const bool valid = ln < total;
      float x = inf;
      if (valid) {
        const int pos = rcur + (ln - rexcl);
        const int c = ci[pos];
        if (bit_of(a.fcur, c)) x = a.fval[c] + a.wpull[pos];
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
        if (bit_of(a.fcur, c)) best = fminf(best, a.fval[c] + a.wpull[pos]);
      }
    }
    best = wave_min(best);
    if (ln == 0 && best < a.dist[r]) {
      const int old = atomicMin((int *)&a.dist[r], __float_as_int(best));
      if (best < __int_as_float(old)) set_bit_guarded(a.fnxt, r);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sssp_expand(TravArgs a) {
  __shared__ PushStage st;
  __shared__ int s_mark[kWavesPerBlock][64];
  const int count = a.ctrl->count;
  if (count == 0) return;
  const int sumdeg = a.ctrl->sumdeg;
  const int dir = decide_dir(a, count, sumdeg);
  record_stats(a, count, sumdeg, dir);
  if (dir == GRB_DIR_PUSH) sssp_push(a, st, sumdeg);
  else sssp_pull(a, s_mark[threadIdx.x >> 6]);
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------

__global__ void k_fill_u64(uint64_t *p, int64_t count, uint64_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_pattern(unsigned char *p, int64_t count, int elem, uint64_t pattern) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (elem == 1) p[i] = (unsigned char)pattern;
    else if (elem == 4) ((uint32_t *)p)[i] = (uint32_t)pattern;
    else ((uint64_t *)p)[i] = pattern;
  }
}

__global__ __launch_bounds__(1024) void k_popcount(const uint64_t *bm, int64_t nw, int64_t *out) {
  __shared__ int64_t s[16];
  int64_t acc = 0;
  for (int64_t i = threadIdx.x; i < nw; i += 1024) acc += __popcll(bm[i]);
  acc = wave_sum64(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < 16; ++i) t += s[i];
    *out = t;
  }
}

__global__ void k_vector_scatter(uint64_t *bitmap, unsigned char *values, int elem, int64_t n,
                                 const int32_t *idx, const unsigned char *vals, int64_t count,
                                 uint64_t one) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx[k];
    if (i < 0 || i >= n) continue;
    atomicOr((unsigned long long *)&bitmap[i >> 6], 1ull << (i & 63));
    if (elem == 1) values[i] = vals ? vals[k] : (unsigned char)one;
    else if (elem == 4) ((uint32_t *)values)[i] = vals ? ((const uint32_t *)vals)[k] : (uint32_t)one;
    else ((uint64_t *)values)[i] = vals ? ((const uint64_t *)vals)[k] : one;
  }
}

inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int compact_blocks(int64_t nw) {
  int64_t b = (nw + kCompactWords - 1) / kCompactWords;
  return (int)(b < 1 ? 1 : b);
}

void launch_compact(int mode, const CompactArgs &a, void *stream) {
  const int g = compact_blocks(a.nw);
  hipStream_t s = (hipStream_t)stream;
  const dim3 blk(kCompactThreads);
  if (mode == kCompactBfs) hipLaunchKernelGGL(k_compact<kCompactBfs>, dim3(g), blk, 0, s, a);
  else if (mode == kCompactSssp) hipLaunchKernelGGL(k_compact<kCompactSssp>, dim3(g), blk, 0, s, a);
  else hipLaunchKernelGGL(k_compact<kCompactPlain>, dim3(g), blk, 0, s, a);
}

void launch_sssp_init(const TravArgs &a, int32_t source, uint64_t *iso, uint64_t *fa,
                      uint64_t *fb, uint64_t *status, int64_t nstatus, void *stream) {
  const int g = grid_for(a.nw, kWavesPerBlock, 4096);
  hipLaunchKernelGGL(k_sssp_init, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, a, source, iso,
                     fa, fb, status, nstatus);
}

void launch_sssp_expand(const TravArgs &a, void *stream) {
  hipLaunchKernelGGL(k_sssp_expand, dim3(kExpandGrid), dim3(kBlock), 0, (hipStream_t)stream, a);
}

void launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, void *stream) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0,
                     (hipStream_t)stream, p, count, value);
}

void launch_fill_bytes_pattern(void *p, int64_t count, int elem_size, const void *value,
                               void *stream) {
  if (count <= 0) return;
  uint64_t pat = 0;
  __builtin_memcpy(&pat, value, (size_t)elem_size);
  hipLaunchKernelGGL(k_fill_pattern, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0,
                     (hipStream_t)stream, (unsigned char *)p, count, elem_size, pat);
}

void launch_popcount(const uint64_t *bm, int64_t nw, int64_t *out, void *stream) {
  hipLaunchKernelGGL(k_popcount, dim3(1), dim3(1024), 0, (hipStream_t)stream, bm, nw, out);
}

void launch_vector_build(uint64_t *bitmap, void *values, int elem_size, int64_t n,
                         const int32_t *idx, const void *vals, int64_t count, uint64_t one,
                         void *stream) {
  launch_fill_u64(bitmap, words_of(n), 0ull, stream);
  if (count <= 0) return;
  hipLaunchKernelGGL(k_vector_scatter, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0,
                     (hipStream_t)stream, bitmap, (unsigned char *)values, elem_size, n, idx,
                     (const unsigned char *)vals, count, one);
}

}  // namespace grb
