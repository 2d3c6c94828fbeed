// BFS entry point for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation): the same
// direction-optimised BFS as grb_bfs, with its workspace in a file-scope
// device array instead of a caller buffer.
//
// The array holds the BFS workspace of graphs up to 2^24 vertices (visited
// and three frontier bitmaps of n / 8 bytes each, the control block, level
// records and the device-side level loop's queues): 9 MiB, held on every
// GPU the library runs on
// until the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) on the first call there;
// in host code the array's own name is not a device address.  Every call on
// one GPU uses that GPU's array: calls that overlap on one GPU race (one
// stream at a time).  The BFS start kernel rewrites every word of the
// workspace it reads, so nothing carries over from a previous call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "grb_internal.h"

namespace grb {
namespace {

constexpr int64_t kNoAllocMaxVertices = (int64_t)1 << 24;
constexpr size_t kNoAllocBytes = (size_t)9 << 20;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The device address of this device's array (looked up on first use).
grb_info scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GRB_PANIC;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GRB_PANIC;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GRB_SUCCESS;
}

}  // namespace
}  // namespace grb

extern "C" grb_info grb_bfs_noalloc(int32_t *levels, int32_t *parents, grb_matrix A,
                                    int32_t source, const grb_descriptor *d, void *stream) {
  using namespace grb;
  if (!A || !A->prepared) return GRB_UNINITIALIZED_OBJECT;
  size_t need = 0;
  grb_info info = grb_workspace_size(GRB_OP_BFS, A, 0, &need);
  if (info != GRB_SUCCESS) return info;
  if (A->nrows > kNoAllocMaxVertices || need > kNoAllocBytes) return GRB_INSUFFICIENT_SPACE;
  grb_descriptor desc;
  if (d) desc = *d;
  else grb_descriptor_init(&desc);
  desc.flags &= ~GRB_PROFILE;  // timing events would be created on demand
  void *ws = nullptr;
  if ((info = scratch_address(&ws)) != GRB_SUCCESS) return info;
  NoAllocScope guard;  // read-backs without a pinned staging buffer
  return grb_bfs(levels, parents, A, source, &desc, ws, kNoAllocBytes, stream);
}
