// Internal declarations of the g5 library: the graph object, error state and
// wave-level device helpers for gfx950 (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "g5.h"

namespace g5 {

constexpr int kWave = 64;
// Rows longer than kHubDeg ("hubs") are listed by Kernel 1 and split into
// kHubChunk-edge work items by the batched traversal.
constexpr int kHubDeg = 4096;
constexpr int kHubChunk = 1024;
// Hint targets given a compact per-level frontier bitmap (2^18 bits = 32 KiB,
// staged in LDS by the bottom-up step).
constexpr int64_t kHotMax = 1 << 18;
// Hint word flag: the hint target is the vertex's only neighbour.
constexpr int32_t kHintOnly = 1 << 30;
// Zeroed col_idx entries past nnz, so fixed-width row reads stay in bounds.
constexpr int64_t kColPad = 16;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

#define G5_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ::g5::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return e_ == hipErrorOutOfMemory ? G5_ENOMEM : G5_EDEVICE;                      \
    }                                                                                 \
  } while (0)

#define G5_LAUNCH_CHECK()                                                             \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess) {                                                           \
      ::g5::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));       \
      return G5_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

// ---------------------------------------------------------------- workspaces
// Device state of one single-root traversal; reused across calls.
struct BfsWork {
  int64_t n = 0, words = 0;
  uint64_t *vis = nullptr;    // visited bitmap (isolated vertices pre-set)
  uint8_t *lev8 = nullptr;    // levels as bytes while they fit (0xff = not reached)
  uint64_t *front = nullptr;  // frontier bitmap (bottom-up input)
  uint64_t *next = nullptr;   // next-frontier bitmap (bottom-up output)
  uint32_t *sum = nullptr;    // frontier summary staged in LDS by bottom-up steps
  int64_t sum_words = 0;      // its 32-bit words
  int sum_gs = 0;             // log2 of the vertices per summary bit
  uint64_t *fh = nullptr;     // frontier bits of the hot hint targets (bottom-up input)
  int32_t *q[2] = {nullptr, nullptr};  // frontier queues
  uint32_t *qoff[2] = {nullptr, nullptr};  // per queue entry: the index of its first edge
                                           // in the queue's edge list
  uint64_t *ctr = nullptr;    // device counters (Ctr in bfs.hip)
  uint64_t *host_pub = nullptr;   // pinned, mapped: counters published by kernels + seq
  uint64_t *host_pub_dev = nullptr;  // its device address
  uint64_t seq = 0;           // last sequence number published
  std::vector<hipEvent_t> ev; // step timing: 2 per timed step launch of a call
  ~BfsWork();
};

// Device state of one batched traversal.
struct BatchWork {
  int64_t n = 0;
  uint64_t *seen = nullptr;            // per-vertex mask of roots that reached it
  uint64_t *buf[3] = {nullptr, nullptr, nullptr};  // frontier masks, rotated per level
  void *ctl = nullptr;                 // level counters (MsCtl in msbfs.hip)
  void *host_ctl = nullptr;            // pinned mirror
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};  // level-loop graph (without / with parents)
  int gblocks[2] = {0, 0};             // the grid each was built for
  ~BatchWork();
};

// Device state of one shortest-path computation (sssp.hip); reused across calls.
struct SsspWork {
  uint64_t *pend = nullptr;   // far set: vertices improved at or above the threshold
  unsigned long long *dp = nullptr;  // per vertex: distance << 32 | predecessor
  uint32_t *stamp = nullptr;  // per vertex: the stamp of the last queue it joined
  int32_t *q[2] = {nullptr, nullptr};  // current and next queue
  uint32_t *qo[2] = {nullptr, nullptr}; // per entry: its first edge in the queue's edge list
  uint64_t *ctr = nullptr;    // device counters (SCtr in sssp.hip)
  uint32_t epoch = 0;         // last queue stamp handed out (only grows)
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~SsspWork();
};

// Defaults picked per graph from the autotuned table (tuned_table.inc).
struct Tuning {
  int scale;              // log2 n the entry was tuned at
  double alpha, beta;     // single-root direction switch
  int lane_scan;          // bottom-up lane scan width
  int bu_blocks_per_cu;   // bottom-up grid
  int vertices_per_lane;  // bottom-up unvisited vertices per lane at once
  int packed;             // bottom-up packed row scan
  int lds_kb;             // LDS budget of the staged frontier per workgroup
  double lds_density;     // stage the frontier in LDS below this summary density
  double batch_alpha;     // batched direction switch
  int batch_blocks_per_cu;
  double gamma;           // single-root switch also when m_f > gamma * unvisited vertices
};
Tuning pick_tuning(int scale);

}  // namespace g5

struct g5_csr {
  int64_t n = 0, nnz = 0, words = 0;
  int sb = 1;                  // bits of a vertex id in a sort key
  int device = 0;
  int num_cu = 256;
  int64_t lds_bytes = 65536;   // LDS a workgroup may use on this device
  int64_t nonisolated = 0;     // vertices of degree >= 1
  int64_t *row_ptr = nullptr;  // device [n+1]
  int32_t *col_idx = nullptr;  // device [nnz]
  uint8_t *wt = nullptr;       // device [nnz]: edge weights (weighted graphs only)
  uint64_t *iso = nullptr;     // device [words]: bit set = degree 0 (or padding)
  uint32_t *rp32 = nullptr;    // device [n+1]: row_ptr as 32-bit offsets
  int32_t *hint = nullptr;     // device [n]: highest-degree neighbour, -1 if none, or
                               // INT32_MIN | i when that neighbour is hot[i]; | kHintOnly
                               // when it is the only neighbour
  int32_t *hint_id = nullptr;  // device [n]: highest-degree neighbour id, -1 if none
  int32_t *hint_c = nullptr;   // device [nonisolated]: hint of the vertices of degree >= 1,
                               // in vertex order (the dense-frontier bottom-up step reads these)
  uint64_t *chunk_ni = nullptr;  // device [(words + 63) / 64]: vertices of degree >= 1 before
                                 // each chunk of 64 bitmap words (4,096 vertices)
  int32_t *hot = nullptr;      // device [num_hot]: hint targets with a compact frontier bit
  int64_t num_hot = 0;         // at most kHotMax
  g5::Tuning tune{};           // defaults for this graph's scale
  int64_t num_hubs = 0;        // vertices with degree > kHubDeg
  int64_t hub_chunks = 0;      // their rows in kHubChunk-edge pieces
  int32_t *hub_list = nullptr; // device [num_hubs]
  uint64_t *hub_off = nullptr; // device [num_hubs+1]: first chunk of each hub
  mutable std::mutex mu;
  mutable std::vector<g5::BfsWork *> bfs_pool;
  mutable std::vector<g5::BatchWork *> batch_pool;
  mutable std::vector<g5::SsspWork *> sssp_pool;
};

namespace g5 {

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  int l = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const T o = __shfl_xor(v, d, kWave);
    v = o < v ? o : v;
  }
  return v;
}

// x of lane l, for a lane index that is the same in every lane (a constant or
// derived from a ballot): a scalar read, not a cross-lane permute through LDS.
__device__ __forceinline__ uint32_t lane_u32(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ int64_t lane_i64(int64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Exclusive prefix sum over a block of NT threads; `s` is LDS scratch of
// NT/64 entries.  Returns the exclusive prefix; `total` gets the block sum.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *s, T &total) {
  constexpr int NW = NT / kWave;
  int l = __lane_id();
  int w = threadIdx.x / kWave;
  T v = wave_incl_scan(x);
  if (l == kWave - 1) s[w] = v;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    T t = s[i];
    if (i < w) base += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + v - x;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T x, T *s) {
  T tot;
  block_excl_scan<NT, T>(x, s, tot);
  return tot;
}

// ---------------------------------------------------------------- host entry points
g5_status build_csr_impl(const int64_t *edges, const uint8_t *weights, bool weighted, int64_t m,
                         int64_t n, hipStream_t s, g5_csr **out);
g5_status bfs_impl(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level,
                   hipStream_t s, const g5_bfs_params &p, g5_bfs_stats *stats);
g5_status bfs_batch_impl(const g5_csr *g, const int64_t *roots, int k, int32_t *parents,
                         int8_t *levels, hipStream_t s, const g5_batch_params &p,
                         g5_batch_stats *stats);
// A stepped batch (default parameters, no statistics) on a workspace the
// caller provides: masks = device uint64 [4n] (seen and three frontier
// buffers), ctl = device memory of batch_ctl_bytes() bytes.  Every part that
// must start at zero is cleared by the call; nothing is allocated.
size_t batch_ctl_bytes();
g5_status batch_in_workspace(const g5_csr *g, uint64_t *masks, void *ctl, const int64_t *roots,
                             int k, int32_t *parents, int8_t *levels, hipStream_t s);
g5_status bfs_batch_noalloc_impl(const g5_csr *g, const int64_t *roots, int k, int32_t *parents,
                                 int8_t *levels, hipStream_t s);
g5_status sssp_impl(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, hipStream_t s,
                    const g5_sssp_params &p, g5_sssp_stats *stats);
g5_status level_work_impl(const g5_csr *g, const int32_t *level, int32_t lvl, bool bottom_up,
                          int64_t *out, hipStream_t s);

}  // namespace g5
