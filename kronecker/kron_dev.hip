// Device build of the seeded Kronecker input generator (definition in
// kron_core.h).  Bit-identical to the host build; used to produce large
// inputs directly in HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kron_core.h"

__global__ void kron_edges_kernel(kron_params p, int relabel, int64_t m,
                                  int64_t *__restrict__ out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    uint64_t r, c;
    kron_raw_tuple(&p, (uint64_t)i, &r, &c);
    if (relabel) {
      r = kron_relabel(&p, r);
      c = kron_relabel(&p, c);
    }
    longlong2 t;
    t.x = (long long)r;
    t.y = (long long)c;
    reinterpret_cast<longlong2 *>(out)[i] = t;
  }
}

__global__ void kron_nonisolated_kernel(const int64_t *__restrict__ edges, int64_t m,
                                        int64_t n, uint8_t *__restrict__ mask,
                                        int *__restrict__ bad) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    longlong2 t = reinterpret_cast<const longlong2 *>(edges)[i];
    if (t.x < 0 || t.x >= n || t.y < 0 || t.y >= n) {
      *bad = 1;
      continue;
    }
    if (t.x == t.y) continue;
    mask[t.x] = 1;
    mask[t.y] = 1;
  }
}

__global__ void kron_weights_kernel(uint64_t base, int64_t m, uint8_t *__restrict__ out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    out[i] = kron_weight(base, (uint64_t)i);
}

static int grid_for(int64_t m) {
  int64_t g = (m + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

extern "C" {

// Writes the m = ef * 2^scale tuples of (scale, seed) to the device buffer
// out[m][2] on stream.  Returns 0, -1 on a bad argument, -3 on a HIP error.
int kron_edges_device(int scale, uint64_t seed, int relabel, int64_t m, int64_t *out,
                      void *stream) {
  if (scale < 1 || scale > KRON_MAX_SCALE || m < 0 || (m > 0 && !out)) return -1;
  if (m == 0) return 0;
  kron_params p = kron_make_params(scale, seed);
  hipLaunchKernelGGL(kron_edges_kernel, dim3(grid_for(m)), dim3(256), 0,
                     (hipStream_t)stream, p, relabel, m, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Writes the weights of tuples [0, m) of (seed) to the device buffer out[m].
int kron_weights_device(uint64_t seed, int64_t m, uint8_t *out, void *stream) {
  if (m < 0 || (m > 0 && !out)) return -1;
  if (m == 0) return 0;
  hipLaunchKernelGGL(kron_weights_kernel, dim3(grid_for(m)), dim3(256), 0, (hipStream_t)stream,
                     kron_weight_base(seed), m, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// mask[v] = 1 for endpoints of non-loop tuples (device buffers).  *bad is set
// to 1 (device int, caller-cleared) if an id is outside [0, n).
int kron_nonisolated_device(const int64_t *edges, int64_t m, int64_t n, uint8_t *mask,
                            int *bad, void *stream) {
  if (m < 0 || n < 1 || !mask || !bad) return -1;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemsetAsync(mask, 0, (size_t)n, s) != hipSuccess) return -3;
  if (m == 0) return 0;
  hipLaunchKernelGGL(kron_nonisolated_kernel, dim3(grid_for(m)), dim3(256), 0, s, edges,
                     m, n, mask, bad);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
}
