// Measurement helper: the work a level of a finished traversal had to do,
// from its level array alone (the level array is unique, so these counts do
// not depend on how the traversal ran).  They define the algorithmic bytes of
// a top-down step (the paper's parallel BFS loops of Section 2.3.2: read the
// frontier queue, each frontier vertex's row offsets and row, write the
// claimed vertices' level, parent and queue entry) and of a bottom-up step
// (each unvisited vertex with a row reads its row offsets and its row in order
// up to the first frontier neighbour; the visited and next-frontier bitmaps
// are read and written once; each claimed vertex gets a level and a parent).
//
// One thread per vertex; rows longer than a wavefront are scanned by the
// whole wavefront, 64 entries per step, stopping at the first frontier entry.
#include <algorithm>

#include "g5_internal.h"

namespace g5 {
namespace {

constexpr int kWorkBlock = 256;

enum WorkOut : int { W_Q = 0, W_MF = 1, W_CLAIMED = 2, W_UNVIS = 3, W_SCANNED = 4, W_N = 5 };

__global__ __launch_bounds__(kWorkBlock) void k_level_work(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ level, int64_t n, int32_t lvl, bool bottom_up,
    unsigned long long *__restrict__ out) {
  __shared__ unsigned long long s_red[kWorkBlock / kWave];
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * kWorkBlock;
  unsigned long long q = 0, mf = 0, claimed = 0, unvis = 0, scanned = 0;
  // the loop bound is rounded up to whole wavefronts so every lane takes part
  // in the wave-wide row scans
  const int64_t span = ((n + kWave - 1) / kWave) * kWave;
  for (int64_t v = (int64_t)blockIdx.x * kWorkBlock + threadIdx.x; v < span; v += stride) {
    int32_t lv = -2;
    int64_t b = 0, e = 0;
    if (v < n) {
      lv = level[v];
      b = rp[v];
      e = rp[v + 1];
    }
    const int64_t d = e - b;
    if (lv == lvl) {
      ++q;
      mf += (unsigned long long)d;
    }
    if (v < n && lv == lvl + 1) ++claimed;
    const bool cand = bottom_up && v < n && d > 0 && (lv == -1 || lv > lvl);
    if (cand) ++unvis;
    // short rows: this lane alone
    if (cand && d <= kWave) {
      int64_t k = b;
      while (k < e && level[ci[k]] != lvl) ++k;
      scanned += (unsigned long long)(k < e ? k - b + 1 : d);
    }
    // long rows: the whole wavefront, one row at a time
    uint64_t rem = __ballot(cand && d > kWave);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      int64_t hit = -1;
      for (int64_t c = kb; c < ke; c += kWave) {
        const int64_t k = c + lane;
        const uint64_t m = __ballot(k < ke && level[ci[k]] == lvl);
        if (m) {
          hit = c + __ffsll((unsigned long long)m) - 1;
          break;
        }
      }
      if (lane == L) scanned += (unsigned long long)(hit >= 0 ? hit - kb + 1 : ke - kb);
    }
  }
  const unsigned long long vals[W_N] = {q, mf, claimed, unvis, scanned};
#pragma unroll
  for (int i = 0; i < W_N; ++i) {
    const unsigned long long t = block_sum<kWorkBlock, unsigned long long>(vals[i], s_red);
    if (threadIdx.x == 0 && t) atomicAdd(out + i, t);
  }
}

__global__ void k_work_zero(unsigned long long *out) {
  if (threadIdx.x < W_N) out[threadIdx.x] = 0;
}

}  // namespace

g5_status level_work_impl(const g5_csr *g, const int32_t *level, int32_t lvl, bool bottom_up,
                          int64_t *out, hipStream_t s) {
  unsigned long long *d = nullptr;
  G5_HIP(hipMalloc((void **)&d, W_N * sizeof(unsigned long long)));
  hipLaunchKernelGGL(k_work_zero, dim3(1), dim3(64), 0, s, d);
  const int64_t blocks = std::min<int64_t>((g->n + kWorkBlock - 1) / kWorkBlock,
                                           (int64_t)g->num_cu * 16);
  hipLaunchKernelGGL(k_level_work, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(kWorkBlock),
                     0, s, (const int64_t *)g->row_ptr, (const int32_t *)g->col_idx, level, g->n,
                     lvl, bottom_up, d);
  hipError_t e = hipGetLastError();
  unsigned long long h[W_N] = {};
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) {
    set_error(std::string("g5_level_work: ") + hipGetErrorString(e));
    return G5_EDEVICE;
  }
  for (int i = 0; i < W_N; ++i) out[i] = (int64_t)h[i];
  return G5_OK;
}

}  // namespace g5
