// Kernel 3 of the paper (Section 2.4): single-source shortest paths over the
// weighted graph, as the parallel delta-stepping that its future-work section
// names (Meyer and Sanders, "Delta-stepping: a parallelizable shortest path
// algorithm", J. Algorithms 2003), in the near/far form suited to GPUs
// (Davidson, Baxter, Garland and Owens, IPDPS 2014).
//
//   threshold T   vertices with dist < T form the current buckets; T advances
//                 by delta once nothing below it is left to relax
//   relax         every vertex of the current queue relaxes all its edges:
//                 nd = dist[u] + w, atomic minimum into dist[v]; an improved v
//                 goes to the next queue if nd < T (once per queue, by a stamp
//                 per vertex), else its "pending" bit is set (the far set)
//   scan          when the queue runs dry: pending vertices with dist < T
//                 form the next queue; with none, T jumps to the bucket of the
//                 smallest pending distance; with no pending vertex, done
//   predecessors  one pass at the end: prev[v] = the smallest-id neighbour u
//                 with dist[u] + w(u, v) = dist[v] (so prev is deterministic)
//
// Rows longer than kHubDeg are relaxed in kHubChunk-edge pieces spread over
// all wavefronts (the hub list of Kernel 1); the main loop skips them.
#include <algorithm>

#include "g5_internal.h"

namespace g5 {
namespace {

constexpr int kBlock = 256;
constexpr int kLaneRow = 32;  // rows up to this length are relaxed by one lane
constexpr uint32_t kInf = 0xffffffffu;
// Bucket width when the caller gives none: weights lie in [1, 255] for the
// seeded graphs, with tens of edges per vertex.
constexpr uint32_t kDefaultDelta = 32;

enum SCtr : int {
  S_QLEN0 = 0,  // length of queue 0
  S_QLEN1 = 1,  // length of queue 1
  S_PEND = 2,   // pending vertices left after a scan
  S_MIN = 3,    // smallest distance among them (kInf if none)
  S_ERR = 4,    // a distance exceeded kInf - 1
  S_RELAX = 5,  // queue entries relaxed (statistics)
  S_N = 8
};

// Pushes v (one lane each) onto a queue: one atomic per wavefront.
__device__ __forceinline__ void push_wave(bool want, int32_t v, int32_t *q,
                                          unsigned long long *len) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(len, (unsigned long long)__popcll(m));
  base = __shfl(base, leader, kWave);
  if (want) q[base + __popcll(m & lanemask_lt())] = v;
}

struct RelaxArgs {
  const int64_t *rp;
  const int32_t *ci;
  const uint8_t *wt;
  uint32_t *dist;
  uint64_t *pend;
  uint32_t *stamp;
  int32_t *qn;
  unsigned long long *ctr;
  int nxt;
  uint64_t T;
  uint32_t epoch;  // stamp of the next queue
};

// Relaxes edge (u, v) of weight w from distance du; returns true when v must
// join the next queue (improved below T and not yet in it).
__device__ __forceinline__ bool relax(const RelaxArgs &a, uint32_t du, int32_t v, uint32_t w) {
  const uint64_t nd = (uint64_t)du + w;
  if (nd >= (uint64_t)a.dist[v]) return false;
  if (nd >= (uint64_t)kInf) {
    atomicOr(a.ctr + S_ERR, 1ull);
    return false;
  }
  const uint32_t old = atomicMin(a.dist + v, (uint32_t)nd);
  if (nd >= old) return false;
  if (nd < a.T) return atomicExch(a.stamp + v, a.epoch) != a.epoch;
  const uint64_t bit = 1ull << (v & 63);
  if (!(a.pend[v >> 6] & bit)) atomicOr((unsigned long long *)(a.pend + (v >> 6)), bit);
  return false;
}

// Start: dist = infinity except the source (0); no pending vertex; queue 0 =
// {src} with the stamp of the first queue; counters zeroed.
__global__ void k_sssp_init(uint32_t *__restrict__ dist, int64_t n, int64_t src,
                            uint64_t *__restrict__ pend, int64_t words, int32_t *__restrict__ q0,
                            uint32_t *__restrict__ stamp, uint32_t epoch,
                            unsigned long long *__restrict__ ctr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < n; i += stride) dist[i] = i == src ? 0u : kInf;
  for (int64_t i = t; i < words; i += stride) pend[i] = 0;
  if (t == 0) {
    for (int i = 0; i < S_N; ++i) ctr[i] = 0;
    ctr[S_QLEN0] = 1;
    ctr[S_MIN] = kInf;
    q0[0] = (int32_t)src;
    stamp[src] = epoch;
  }
}

// One relaxation round over queue `cur` (its length in ctr); fills queue nxt.
__global__ __launch_bounds__(kBlock) void k_sssp_relax(const int32_t *__restrict__ q, int cur,
                                                       RelaxArgs a) {
  const int lane = __lane_id();
  const int64_t qlen = (int64_t)a.ctr[S_QLEN0 + cur];
  const int64_t gw = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) / kWave;
  unsigned long long *nlen = a.ctr + S_QLEN0 + a.nxt;
  for (int64_t base = gw * kWave; base < qlen; base += nw * kWave) {
    const int64_t i = base + lane;
    int32_t u = -1;
    int64_t b = 0, e = 0;
    uint32_t du = kInf;
    if (i < qlen) {
      u = q[i];
      b = a.rp[u];
      e = a.rp[u + 1];
      du = a.dist[u];
      // u is relaxed now: it leaves the far set if it was there
      const uint64_t bit = 1ull << (u & 63);
      if (a.pend[u >> 6] & bit) atomicAnd((unsigned long long *)(a.pend + (u >> 6)), ~bit);
    }
    const int64_t d = e - b;
    // short rows: one lane each; the queue pushes stay wave-uniform
    int64_t k = b;
    const bool mine = u >= 0 && d <= kLaneRow;
    while (__ballot(mine && k < e)) {
      bool push = false;
      int32_t v = 0;
      if (mine && k < e) {
        v = a.ci[k];
        push = relax(a, du, v, a.wt[k]);
        ++k;
      }
      push_wave(push, v, a.qn, nlen);
    }
    // longer rows (not hubs): the whole wavefront, one row at a time
    uint64_t rem = __ballot(u >= 0 && d > kLaneRow && d <= kHubDeg);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      const uint32_t dL = __shfl(du, L, kWave);
      for (int64_t c = kb; c < ke; c += kWave) {
        const int64_t kk = c + lane;
        bool push = false;
        int32_t v = 0;
        if (kk < ke) {
          v = a.ci[kk];
          push = relax(a, dL, v, a.wt[kk]);
        }
        push_wave(push, v, a.qn, nlen);
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.ctr + S_RELAX, (unsigned long long)qlen);
}

// Hub rows of the current queue (stamp = cur_epoch) in kHubChunk-edge pieces.
__global__ __launch_bounds__(kBlock) void k_sssp_relax_hubs(const int32_t *__restrict__ hub_list,
                                                            const uint64_t *__restrict__ hub_off,
                                                            int64_t num_hubs, int64_t chunks,
                                                            uint32_t cur_epoch, RelaxArgs a) {
  const int lane = __lane_id();
  const int64_t gw = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) / kWave;
  unsigned long long *nlen = a.ctr + S_QLEN0 + a.nxt;
  for (int64_t c = gw; c < chunks; c += nw) {
    int64_t lo = 0, hi = num_hubs;  // hub owning chunk c: largest i with hub_off[i] <= c
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (hub_off[mid] <= (uint64_t)c)
        lo = mid;
      else
        hi = mid;
    }
    const int32_t h = hub_list[lo];
    if (a.stamp[h] != cur_epoch) continue;
    const uint32_t dh = a.dist[h];
    const int64_t kb = a.rp[h] + (int64_t)((uint64_t)c - hub_off[lo]) * kHubChunk;
    const int64_t ke = std::min<int64_t>(kb + kHubChunk, a.rp[h + 1]);
    for (int64_t k0 = kb; k0 < ke; k0 += kWave) {
      const int64_t k = k0 + lane;
      bool push = false;
      int32_t v = 0;
      if (k < ke) {
        v = a.ci[k];
        push = relax(a, dh, v, a.wt[k]);
      }
      push_wave(push, v, a.qn, nlen);
    }
  }
}

// Pending vertices with dist < T leave the far set for queue nxt (stamp =
// epoch); the rest are counted and their smallest distance taken.
__global__ __launch_bounds__(kBlock) void k_sssp_scan(const uint32_t *__restrict__ dist,
                                                      uint64_t *__restrict__ pend, int64_t words,
                                                      uint64_t T, int32_t *__restrict__ qn,
                                                      int nxt, uint32_t *__restrict__ stamp,
                                                      uint32_t epoch,
                                                      unsigned long long *__restrict__ ctr) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t span = ((words + kWave - 1) / kWave) * kWave;  // whole wavefronts
  unsigned long long left = 0;
  uint32_t dmin = kInf;
  for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < span; w += stride) {
    uint64_t m = w < words ? pend[w] : 0;
    uint64_t take = 0;
    // one vertex of the word per step; every lane steps until all words are done
    uint64_t rest = m;
    while (__ballot(rest != 0)) {
      bool push = false;
      int32_t v = 0;
      if (rest) {
        const int b = __ffsll((unsigned long long)rest) - 1;
        rest &= rest - 1;
        v = (int32_t)(w * kWave + b);
        const uint32_t dv = dist[v];
        if ((uint64_t)dv < T) {
          take |= 1ull << b;
          stamp[v] = epoch;
          push = true;
        } else {
          ++left;
          dmin = std::min(dmin, dv);
        }
      }
      push_wave(push, v, qn, ctr + S_QLEN0 + nxt);
    }
    if (take) pend[w] = m & ~take;
  }
  __shared__ unsigned long long s_red[kBlock / kWave];
  const unsigned long long tl = block_sum<kBlock, unsigned long long>(left, s_red);
  uint32_t bm = dmin;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) bm = std::min(bm, (uint32_t)__shfl_xor(bm, d, kWave));
  if (threadIdx.x == 0 && tl) atomicAdd(ctr + S_PEND, tl);
  if (__lane_id() == 0 && bm != kInf) atomicMin(ctr + S_MIN, (unsigned long long)bm);
}

// prev[v] = src for the source, -1 where dist is infinite, else the
// smallest-id neighbour u with dist[u] + w(u, v) = dist[v] (rows ascending:
// the first such entry).
__global__ __launch_bounds__(kBlock) void k_sssp_prev(const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const uint8_t *__restrict__ wt,
                                                      const uint32_t *__restrict__ dist, int64_t n,
                                                      int64_t src, int32_t *__restrict__ prev,
                                                      unsigned long long *__restrict__ ctr) {
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t span = ((n + kWave - 1) / kWave) * kWave;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < span; v += stride) {
    uint32_t dv = kInf;
    int64_t b = 0, e = 0;
    if (v < n) {
      dv = dist[v];
      if (dv != kInf && v != src) {
        b = rp[v];
        e = rp[v + 1];
      }
    }
    int32_t p = (v < n && dv != kInf && v == src) ? (int32_t)src : -1;
    const bool lane_row = e - b <= kLaneRow;
    if (lane_row)
      for (int64_t k = b; k < e; ++k) {
        const uint32_t du = dist[ci[k]];
        if (du != kInf && (uint64_t)du + wt[k] == (uint64_t)dv) {
          p = ci[k];
          break;
        }
      }
    uint64_t rem = __ballot(!lane_row);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      const uint32_t dL = __shfl(dv, L, kWave);
      int32_t found = -1;
      for (int64_t c = kb; c < ke && found < 0; c += kWave) {
        const int64_t k = c + lane;
        bool hit = false;
        if (k < ke) {
          const uint32_t du = dist[ci[k]];
          hit = du != kInf && (uint64_t)du + wt[k] == (uint64_t)dL;
        }
        const uint64_t m = __ballot(hit);
        if (m) found = __shfl(ci[std::min<int64_t>(c + __ffsll((unsigned long long)m) - 1, ke - 1)],
                              0, kWave);
      }
      if (lane == L) p = found;
    }
    if (v < n) {
      if (dv != kInf && p < 0) atomicOr(ctr + S_ERR, 2ull);  // no tight neighbour
      prev[v] = p;
    }
  }
}

// Clears the next queue's length (and, before a scan, the pending count and
// minimum).
__global__ void k_reset_ctr(unsigned long long *ctr, int nxt, bool scan) {
  if (threadIdx.x == 0) {
    ctr[S_QLEN0 + nxt] = 0;
    if (scan) {
      ctr[S_PEND] = 0;
      ctr[S_MIN] = kInf;
    }
  }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t len, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = v;
}

int grid_blocks(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

SsspWork::~SsspWork() {
  if (pend) (void)hipFree(pend);
  if (stamp) (void)hipFree(stamp);
  for (auto *p : q)
    if (p) (void)hipFree(p);
  if (ctr) (void)hipFree(ctr);
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
}

namespace {
g5_status alloc_sssp(const g5_csr *g, SsspWork **out) {
  SsspWork *w = new SsspWork();
  hipError_t e = hipSuccess;
  auto A = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  A((void **)&w->pend, g->words * 8);
  A((void **)&w->stamp, g->n * 4);
  A((void **)&w->q[0], g->n * 4);
  A((void **)&w->q[1], g->n * 4);
  A((void **)&w->ctr, S_N * 8);
  if (e == hipSuccess) e = hipMemset(w->stamp, 0, g->n * 4);
  if (e != hipSuccess) {
    set_error(std::string("g5_sssp workspace: ") + hipGetErrorString(e));
    delete w;
    return e == hipErrorOutOfMemory ? G5_ENOMEM : G5_EDEVICE;
  }
  *out = w;
  return G5_OK;
}

struct SsspLease {
  const g5_csr *g;
  SsspWork *w = nullptr;
  ~SsspLease() {
    if (w) {
      std::lock_guard<std::mutex> lk(g->mu);
      g->sssp_pool.push_back(w);
    }
  }
};
}  // namespace

g5_status sssp_impl(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, hipStream_t s,
                    const g5_sssp_params &p, g5_sssp_stats *stats) {
  if (!g->wt) {
    set_error("g5_sssp: the graph has no weights (build it with g5_build_csr_w)");
    return G5_EINVAL;
  }
  SsspLease lease{g};
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->sssp_pool.empty()) {
      lease.w = g->sssp_pool.back();
      g->sssp_pool.pop_back();
    }
  }
  if (!lease.w) {
    g5_status st = alloc_sssp(g, &lease.w);
    if (st != G5_OK) return st;
  }
  SsspWork &w = *lease.w;
  const bool timed = stats && (p.flags & G5_FLAG_TIME_STEPS);
  if (timed && !w.ev[0]) {
    G5_HIP(hipEventCreate(&w.ev[0]));
    G5_HIP(hipEventCreate(&w.ev[1]));
  }
  // stamps only grow, so the queues of earlier calls never match; restart
  // them (a fill kernel, not a memset) well before the counter wraps
  if (w.epoch > 0xf0000000u) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(g->n, 256, g->num_cu * 16)), dim3(256), 0, s,
                       w.stamp, g->n, 0u);
    w.epoch = 0;
  }
  const int64_t n = g->n, W = g->words;
  const int ncu = g->num_cu;
  const uint64_t delta = p.delta > 0 ? (uint64_t)p.delta : (uint64_t)kDefaultDelta;
  const int grid = ncu * 8;
  unsigned long long *ctr = (unsigned long long *)w.ctr;
  if (timed) G5_HIP(hipEventRecord(w.ev[0], s));
  uint32_t ep = ++w.epoch;
  hipLaunchKernelGGL(k_sssp_init, dim3(grid_blocks(std::max(n, W), 256, ncu * 16)), dim3(256), 0,
                     s, dist, n, src, w.pend, W, w.q[0], w.stamp, ep, ctr);
  G5_LAUNCH_CHECK();
  uint64_t T = delta;
  int cur = 0;
  int64_t rounds = 0, scans = 0, buckets = 1;
  unsigned long long hc[S_N] = {};
  unsigned long long qlen = 1;
  bool last_scan = false;
  RelaxArgs a;
  a.rp = g->row_ptr;
  a.ci = g->col_idx;
  a.wt = g->wt;
  a.dist = dist;
  a.pend = w.pend;
  a.stamp = w.stamp;
  a.ctr = ctr;
  while (true) {
    const int nxt = cur ^ 1;
    if (qlen > 0) {
      // relax the current queue into the other one
      a.qn = w.q[nxt];
      a.nxt = nxt;
      a.T = T;
      const uint32_t cur_ep = ep;
      a.epoch = ep = ++w.epoch;
      hipLaunchKernelGGL(k_reset_ctr, dim3(1), dim3(64), 0, s, ctr, nxt, false);
      hipLaunchKernelGGL(k_sssp_relax, dim3(grid_blocks((int64_t)qlen, kBlock, grid)),
                         dim3(kBlock), 0, s, (const int32_t *)w.q[cur], cur, a);
      if (g->hub_chunks > 0)
        hipLaunchKernelGGL(k_sssp_relax_hubs,
                           dim3(grid_blocks(g->hub_chunks, kBlock / kWave, grid)), dim3(kBlock),
                           0, s, (const int32_t *)g->hub_list, (const uint64_t *)g->hub_off,
                           g->num_hubs, g->hub_chunks, cur_ep, a);
      G5_LAUNCH_CHECK();
      ++rounds;
      last_scan = false;
    } else {
      // the queue ran dry: pending vertices below T form the next one
      ep = ++w.epoch;
      hipLaunchKernelGGL(k_reset_ctr, dim3(1), dim3(64), 0, s, ctr, nxt, true);
      hipLaunchKernelGGL(k_sssp_scan, dim3(grid_blocks(W, kBlock, ncu * 16)), dim3(kBlock), 0, s,
                         (const uint32_t *)dist, w.pend, W, T, w.q[nxt], nxt, w.stamp, ep, ctr);
      G5_LAUNCH_CHECK();
      ++scans;
      last_scan = true;
    }
    cur = nxt;
    G5_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
    G5_HIP(hipStreamSynchronize(s));
    if (hc[S_ERR]) {
      set_error("g5_sssp: a distance exceeds 2^32 - 2");
      return G5_ERANGE;
    }
    qlen = hc[S_QLEN0 + cur];
    if (qlen > 0 || !last_scan) continue;
    // a scan found nothing below T: done without pending vertices, else T
    // moves to the end of the bucket of the smallest pending distance
    if (hc[S_PEND] == 0) break;
    T = (hc[S_MIN] / delta + 1) * delta;
    ++buckets;
  }
  hipLaunchKernelGGL(k_sssp_prev, dim3(grid_blocks(n, kBlock, ncu * 16)), dim3(kBlock), 0, s,
                     g->row_ptr, g->col_idx, g->wt, (const uint32_t *)dist, n, src, prev, ctr);
  G5_LAUNCH_CHECK();
  if (timed) G5_HIP(hipEventRecord(w.ev[1], s));
  G5_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
  G5_HIP(hipStreamSynchronize(s));
  if (hc[S_ERR]) {
    set_error("g5_sssp: a reached vertex has no tight neighbour (inconsistent distances)");
    return G5_EDEVICE;
  }
  if (stats) {
    *stats = g5_sssp_stats{};
    stats->rounds = rounds;
    stats->scans = scans;
    stats->buckets = buckets;
    stats->relaxed = (int64_t)hc[S_RELAX];
    stats->delta = (int64_t)delta;
    if (timed) {
      float ms = 0;
      G5_HIP(hipEventElapsedTime(&ms, w.ev[0], w.ev[1]));
      stats->ms = ms;
    }
  }
  return G5_OK;
}

}  // namespace g5
