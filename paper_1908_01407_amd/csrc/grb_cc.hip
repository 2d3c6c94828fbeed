// Connected components (Section 7.4 of the paper: the FastSV form of
// Shiloach-Vishkin, hooking and shortcutting in linear algebra).  Vectors
// f (parent), gf (grandparent), mngf (smallest grandparent seen among the
// neighbours); every label is a vertex id and only ever decreases, so the
// fixed point labels each component with its smallest id.  Per iteration:
//   mngf = min(mngf, A (min, second) gf)      the generic product, pull
//   f[f_old[u]] = min(., mngf[u])             stochastic hooking (scatter)
//   f[u] = min(f[u], mngf[u])                 aggressive hooking
//   f[u] = min(f[u], gf[u])                   shortcutting
//   gf[u] = f[f[u]]; count the u whose gf changed
// until an iteration changes no grandparent.  The product is grb_mxv; the
// element-wise steps are the kernels below, one grid-stride pass each.
#include <hip/hip_runtime.h>

#include "grb_device.h"
#include "grb_internal.h"

namespace grb {
namespace {

__global__ void k_cc_init(CcArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a.f[i] = (int32_t)i;
    a.f_old[i] = (int32_t)i;
    a.gf[i] = (int32_t)i;
    a.mngf[i] = (int32_t)i;
  }
  // presence bitmaps of gf and mngf: every index present, padding bits zero
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nw;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rem = a.n - w * 64;
    const uint64_t bits = rem >= 64 ? ~0ull : mask_below((int)rem);
    a.gf_bm[w] = bits;
    a.mngf_bm[w] = bits;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kStatsCap; i += blockDim.x) a.changed[i] = 0;
}

// hooking: the smallest neighbour grandparent hooks the old parent (scatter,
// atomic minimum: several vertices may share a parent) and the vertex itself.
// Labels only decrease, so a target already at or below m never needs the
// atomic; after the first iteration most vertices share a handful of roots,
// and the read keeps millions of atomics off those few words.
__global__ void k_cc_hook(CcArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = a.mngf[i];
    const int32_t p = a.f_old[i];
    if (m < a.f[p]) atomicMin(&a.f[p], m);
    if (m < a.f[i]) atomicMin(&a.f[i], m);
  }
}

__global__ void k_cc_shortcut(CcArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = a.gf[i];
    if (g < a.f[i]) a.f[i] = g;
  }
}

// gf = f[f]; the vertices whose grandparent changed are counted for this
// iteration; f_old = f for the next hooking
__global__ void k_cc_grand(CcArgs a, int32_t it) {
  int cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t fi = a.f[i];
    const int32_t g = a.f[fi];
    if (g != a.gf[i]) ++cnt;
    a.gf[i] = g;
    a.f_old[i] = fi;
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long *)&a.changed[it],
                                                (unsigned long long)cnt);
}

__global__ void k_cc_out(CcArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x)
    a.labels[i] = a.gf[i];
}

int grid_of(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

void launch_cc_init(const CcArgs &a, void *stream) {
  hipLaunchKernelGGL(k_cc_init, dim3(grid_of(std::max<int64_t>(a.n, kStatsCap))), dim3(kBlock), 0,
                     (hipStream_t)stream, a);
}

void launch_cc_step(const CcArgs &a, int32_t it, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int g = grid_of(a.n);
  hipLaunchKernelGGL(k_cc_hook, dim3(g), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_cc_shortcut, dim3(g), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_cc_grand, dim3(g), dim3(kBlock), 0, s, a, it);
}

void launch_cc_out(const CcArgs &a, void *stream) {
  hipLaunchKernelGGL(k_cc_out, dim3(grid_of(a.n)), dim3(kBlock), 0, (hipStream_t)stream, a);
}

}  // namespace grb
