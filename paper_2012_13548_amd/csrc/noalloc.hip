// g5_bfs_batch_noalloc: the batched traversal with its workspace in a fixed
// device array of the library, for callers that cannot allocate device memory.
//
// `scratch` holds the seen masks and three frontier mask buffers of at most
// G5_NOALLOC_MAX_N vertices, then the level counters.  Each GPU the library
// runs on holds its own copy until the process ends.  On the host, the
// array's name is a stand-in symbol, not a device address: host code reaches
// the array only through the pointer hipGetSymbolAddress returns for the
// current device, looked up once per device and kept.  Calls on one GPU share
// the array, so calls that overlap on one GPU race; every part that must
// start at zero is cleared by each call.
#include <mutex>
#include <string>

#include "g5_internal.h"

namespace g5 {
namespace {

constexpr int64_t kNoAllocMaxN = G5_NOALLOC_MAX_N;
constexpr size_t kMaskBytes = 4 * (size_t)kNoAllocMaxN * sizeof(uint64_t);
constexpr size_t kCtlBytes = 4096;  // at least batch_ctl_bytes(), checked at run time
constexpr size_t kScratchBytes = kMaskBytes + kCtlBytes;

static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (the current device).
g5_status scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("g5_bfs_batch_noalloc: device index out of range");
    return G5_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error(std::string("g5_bfs_batch_noalloc: address of the fixed workspace: ") +
                hipGetErrorString(e));
      return G5_EDEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return G5_OK;
}

}  // namespace

g5_status bfs_batch_noalloc_impl(const g5_csr *g, const int64_t *roots, int k, int32_t *parents,
                                 int8_t *levels, hipStream_t s) {
  if (g->n > kNoAllocMaxN) {
    set_error("g5_bfs_batch_noalloc: the graph has " + std::to_string(g->n) +
              " vertices; the fixed workspace holds at most " + std::to_string(kNoAllocMaxN));
    return G5_EINVAL;
  }
  if (batch_ctl_bytes() > kCtlBytes) {
    set_error("g5_bfs_batch_noalloc: level counters larger than their fixed slot");
    return G5_EDEVICE;
  }
  int dev = 0;
  G5_HIP(hipGetDevice(&dev));
  if (dev != g->device) {
    set_error("g5_bfs_batch_noalloc: the graph's device is not the current device");
    return G5_EINVAL;
  }
  void *base = nullptr;
  {
    const g5_status st = scratch_ptr(dev, &base);
    if (st != G5_OK) return st;
  }
  uint64_t *masks = static_cast<uint64_t *>(base);
  void *ctl = static_cast<char *>(base) + kMaskBytes;
  return batch_in_workspace(g, masks, ctl, roots, k, parents, levels, s);
}

}  // namespace g5
