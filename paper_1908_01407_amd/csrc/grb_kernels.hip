// HIP kernels for gfx950 (CDNA4, wave64): frontier compaction (bitmap ->
// sorted list with degree prefix and merge-path tile starts) used by the
// generic masked products, and small utility kernels.  BFS lives in
// grb_bfs.hip, SSSP in grb_sssp.hip, batched BFS in grb_msbfs.hip,
// PageRank in grb_spmv.hip and the generic products in grb_mxv.hip.
//
// Design notes (prior art in the paper: Sections 4-6; the kernels below are
// written for this hardware, not translated):
// * Frontiers are kept both as a presence bitmap (one uint64 word per 64
//   vertices: exactly one wave64 ballot) and as a sorted vertex list with an
//   exclusive prefix of degrees.  The compaction kernel builds the list from
//   the bitmap in one pass with a decoupled look-back scan.
// * The list feeds push kernels that walk it with merge-path tiles over
//   (entries + edges), so a hub's edges spread over many workgroups.
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
// output comes from the blocks' sums when an earlier kernel left them
// (blk_part), else from a decoupled look-back over the workgroups before it
// (tickets, not blockIdx, order the workgroups, so every workgroup a
// look-back waits on is already running).  The status word packs
// flag (2 bits) | count (31 bits) | degree sum (31 bits).
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
  // a generic product that pulls needs no list
  if (a.gated && gate_dir(a.gate) != GRB_DIR_PUSH) return;
  // with the blocks' sums given, a block's offset needs no other block to
  // run first (workgroup id = block); otherwise tickets order the look-back
  if (tid == 0) s_blk = a.blk_part ? (int)blockIdx.x : atomicAdd(&a.ctrl->ticket, 1);
  __syncthreads();
  const int blk = s_blk;
  const int64_t w0 = (int64_t)blk * kCompactWords + wid * WPW;
  if (tid == 0 && !a.blk_part) a.status_next[blk] = 0ull;

  // bits at positions >= nbits (a bitmap's padding) never enter the list
  const int64_t nbits = a.nbits > 0 ? a.nbits : a.nw * 64;
  const int64_t wlast = (nbits - 1) >> 6;
  const uint64_t mlast = mask_below((int)(nbits - wlast * 64));
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int64_t w = w0 + k;
    const uint64_t word = w < a.nw ? (a.nb[w] & (w == wlast ? mlast : ~0ull)) : 0ull;
    int deg = 0;
    if ((word >> ln) & 1ull) {
      const int64_t v = w * 64 + ln;
      if (a.rp) deg = a.rp[v + 1] - a.rp[v];
    }
    const int ds = word ? wave_sum(deg) : 0;  // the word is the same in every lane
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
    const int ctot = lane_last(ci), dtot = lane_last(di);
    int ce = ci - cl, de = di - dl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s_cnt[4 * ln + i] = ce;
      s_deg[4 * ln + i] = de;
      ce += c[i];
      de += d[i];
    }
    int64_t ec = 0, ed = 0;
    if (a.blk_part) {  // the sums of the blocks before this one
      for (int j = ln; j < blk; j += 64) {
        ec += a.blk_part[2 * j];
        ed += a.blk_part[2 * j + 1];
      }
      ec = wave_sum64(ec);
      ed = wave_sum64(ed);
    } else if (blk > 0) {
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
      if (!a.blk_part)
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
        if (a.count_out) *a.count_out = (int)cnt;
        a.ctrl->ticket = 0;
      }
    }
  }
  __syncthreads();

  const int bc = s_base_c, bd = s_base_d;
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int64_t w = w0 + k;
    const uint64_t word = w < a.nw ? (a.nb[w] & (w == wlast ? mlast : ~0ull)) : 0ull;
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
    }
  }
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------

// first two column ids of every row, -1 where the row is shorter
__global__ void k_first_two(const int32_t *rp, const int32_t *ci, int64_t nrows, int2 *out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int b = rp[r], e = rp[r + 1];
    out[r] = make_int2(e > b ? ci[b] : -1, e > b + 1 ? ci[b + 1] : -1);
  }
}

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
    if (!values) continue;
    if (elem == 1) values[i] = vals ? vals[k] : (unsigned char)one;
    else if (elem == 4) ((uint32_t *)values)[i] = vals ? ((const uint32_t *)vals)[k] : (uint32_t)one;
    else ((uint64_t *)values)[i] = vals ? ((const uint64_t *)vals)[k] : one;
  }
}

// first position k in [lo, hi) with list[k] >= key (hi if none), found by
// the wave together: each round probes 64 evenly spaced positions.  Needs
// all 64 lanes; the list must be sorted for the answer to mean anything,
// but every probe stays inside [lo, hi) in any case.
__device__ int64_t wave_lower_bound(const int32_t *list, int64_t lo, int64_t hi, int64_t key) {
  const int ln = threadIdx.x & 63;
  while (hi - lo > 64) {
    // probe f is the first of p_l = lo + l * step at or past the answer (a
    // probe at or past hi counts as past it); the answer is in (p_{f-1}, p_f]
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t p = lo + ln * step;
    const bool ge = p >= hi || (int64_t)list[p] >= key;
    const uint64_t b = __ballot(ge);
    const int f = b ? __ffsll((unsigned long long)b) - 1 : 64;
    const int64_t nlo = f == 0 ? lo : lo + (int64_t)(f - 1) * step + 1;
    const int64_t nhi = f == 64 ? hi : lo + (int64_t)f * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
    if (lo >= hi) return lo;
  }
  const int64_t p = lo + ln;
  const uint64_t b = __ballot(p < hi && (int64_t)list[p] >= key);
  return b ? lo + (__ffsll((unsigned long long)b) - 1) : hi;
}

// Sorted list -> presence bitmap: each wave owns 64 consecutive words, finds
// the list entries that fall in them, ORs their bits in LDS and writes all
// 64 words (zeros included, so the bitmap needs no clearing first).  With
// `gated`, returns unless the product pulls.
__global__ __launch_bounds__(kBlock) void k_list_to_bitmap(const int32_t *list, const int32_t *cnt,
                                                           int64_t cap, int64_t nw, uint64_t *bm,
                                                           DirGate gate, bool gated) {
  __shared__ unsigned long long s_w[kWavesPerBlock][64];
  if (gated && gate_dir(gate) != GRB_DIR_PULL) return;
  const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t c = *cnt;
  c = c < 0 ? 0 : (c > cap ? cap : c);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w0 = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * 64; w0 < nw; w0 += nwaves * 64) {
    s_w[wv][ln] = 0ull;
    wave_lds_sync();
    const int64_t lo = wave_lower_bound(list, 0, c, w0 * 64);
    const int64_t hi = wave_lower_bound(list, lo, c, (w0 + 64) * 64);
    for (int64_t k = lo + ln; k < hi; k += 64) {
      const int64_t id = list[k];
      const int64_t off = (id >> 6) - w0;
      if (off >= 0 && off < 64) atomicOr(&s_w[wv][off], 1ull << (id & 63));
    }
    wave_lds_sync();
    if (w0 + ln < nw) bm[w0 + ln] = s_w[wv][ln];
    wave_lds_sync();
  }
}

// Presence bitmap -> sorted list and count in one workgroup (a setup-time
// conversion that needs no workspace): 1024 words per round, a block scan of
// their popcounts places each word's indices.
__global__ __launch_bounds__(1024) void k_bitmap_to_list_small(const uint64_t *bm, int64_t n,
                                                               int32_t *list, int32_t *cnt) {
  const int64_t nw = (n + 63) / 64;
  __shared__ int s_wave[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < nw; w0 += 1024) {
    const int64_t w = w0 + tid;
    uint64_t word = w < nw ? bm[w] : 0ull;
    if (w == nw - 1 && (n & 63)) word &= mask_below((int)(n & 63));  // padding bits
    const int c = __popcll(word);
    const int incl = wave_incl_scan(c);
    if (ln == 63) s_wave[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < 16; ++k) {
      const int x = s_wave[k];
      if (k < wv) before += x;
      total += x;
    }
    int pos = s_base + before + incl - c;
    for (uint64_t x = word; x; x &= x - 1) list[pos++] = (int32_t)(w * 64 + __ffsll((unsigned long long)x) - 1);
    __syncthreads();
    if (tid == 0) s_base += total;
    __syncthreads();
  }
  if (tid == 0) *cnt = s_base;
}

__global__ void k_iota(int32_t *list, int64_t n, int32_t *cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    list[i] = (int32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) *cnt = (int32_t)n;
}

__global__ void k_gather_values(const unsigned char *values, int elem, const int32_t *list,
                                const int32_t *cnt, int64_t cap, unsigned char *out) {
  int64_t c = *cnt;
  c = c < 0 ? 0 : (c > cap ? cap : c);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < c;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = list[k];
    if (i < 0 || i >= cap) continue;
    if (elem == 1) out[k] = values[i];
    else if (elem == 4) ((uint32_t *)out)[k] = ((const uint32_t *)values)[i];
    else ((uint64_t *)out)[k] = ((const uint64_t *)values)[i];
  }
}

__global__ void k_any_negative(const void *values, int vtype, int64_t n, int32_t *flag) {
  bool neg = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (vtype == GRB_FP32) neg |= !(((const float *)values)[i] >= 0.0f);
    else neg |= !(((const double *)values)[i] >= 0.0);
  }
  if (__ballot(neg) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
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

void launch_compact(const CompactArgs &a, void *stream) {
  const int g = compact_blocks(a.nw);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_compact, dim3(g), dim3(kCompactThreads), 0, s, a);
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

void launch_first_two(const int32_t *rp, const int32_t *ci, int64_t nrows, int2 *out,
                      void *stream) {
  if (nrows <= 0) return;
  int64_t g = (nrows + 255) / 256;
  g = g > 8192 ? 8192 : g;
  hipLaunchKernelGGL(k_first_two, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, rp, ci,
                     nrows, out);
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

void launch_list_to_bitmap(const int32_t *list, const int32_t *cnt, int64_t n, uint64_t *bm,
                           void *stream, const DirGate *gate) {
  const int64_t nw = words_of(n);
  if (nw <= 0) return;
  const int g = grid_for(nw, 64 * kWavesPerBlock, 4096);
  hipLaunchKernelGGL(k_list_to_bitmap, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, list, cnt,
                     n, nw, bm, gate ? *gate : DirGate(), gate != nullptr);
}

void launch_bitmap_to_list_small(const uint64_t *bm, int64_t n, int32_t *list, int32_t *cnt,
                                 void *stream) {
  hipLaunchKernelGGL(k_bitmap_to_list_small, dim3(1), dim3(1024), 0, (hipStream_t)stream, bm, n,
                     list, cnt);
}

void launch_any_negative(const void *values, int vtype, int64_t n, int32_t *flag, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_pattern, dim3(1), dim3(64), 0, s, (unsigned char *)flag, (int64_t)1, 4,
                     (uint64_t)0);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_any_negative, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, values,
                     vtype, n, flag);
}

void launch_iota(int32_t *list, int64_t n, int32_t *cnt, void *stream) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0,
                     (hipStream_t)stream, list, n, cnt);
}

void launch_gather_values(const void *values, int elem_size, const int32_t *list,
                          const int32_t *cnt, int64_t cap, void *out, void *stream) {
  hipLaunchKernelGGL(k_gather_values, dim3(grid_for(cap, kBlock, 4096)), dim3(kBlock), 0,
                     (hipStream_t)stream, (const unsigned char *)values, elem_size, list, cnt,
                     cap, (unsigned char *)out);
}

}  // namespace grb
