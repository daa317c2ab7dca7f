// Kernel 3 of the paper (Section 2.4): single-source shortest paths over the
// weighted graph, as the parallel delta-stepping that its future-work section
// names (Meyer and Sanders, "Delta-stepping: a parallelizable shortest path
// algorithm", J. Algorithms 2003), in the near/far form suited to GPUs
// (Davidson, Baxter, Garland and Owens, IPDPS 2014).
//
//   threshold T   vertices with dist < T form the current buckets; T advances
//                 by delta once nothing below it is left to relax
//   relax         every vertex of the current queue relaxes all its edges:
//                 nd = dist[u] + w; a 64-bit atomic minimum of (nd << 32 | u)
//                 into v's word keeps its distance and, among the relaxations
//                 that reach it, the smallest-id predecessor; a v whose
//                 distance improved goes to the next queue if nd < T (once per
//                 queue, by a stamp per vertex), else its "pending" bit is set
//                 (the far set)
//   scan          when the queue runs dry: pending vertices with dist < T
//                 form the next queue; with none, T jumps to the bucket of the
//                 smallest pending distance; with no pending vertex, done
//   predecessors  every neighbour u on a shortest path to v relaxes v with
//                 its final distance at some round, so the packed minimum ends
//                 as (dist[v], the smallest such u): prev is deterministic; one
//                 streaming pass writes dist and prev
//
// Relaxations are edge-balanced: every queue entry carries the index of its
// first edge in the queue's edge list (assigned when it was appended, from one
// packed atomic per wavefront), and each workgroup takes 1,024-edge tiles of
// that list in turn, so hub rows are split across workgroups and short rows
// are packed together.  A round whose queue holds a large share of the
// graph's edges pulls instead: every vertex takes the best relaxation over its
// neighbours in the queue (known by their stamp) and keeps it if it beats its
// own word, so the distances need no atomics (a hub's row is read in pieces
// that combine by atomic minimum).
#include <algorithm>

#include "g5_internal.h"

namespace g5 {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int kTile = kBlock * kItems;  // edges per relaxation tile
constexpr uint32_t kInf = 0xffffffffu;
// Bucket width when the caller gives none: weights lie in [1, 255] for the
// seeded graphs, with tens of edges per vertex (a sweep at scale 22 over
// 4..2^20: 16 and 32 within 4 %, 8 and 64 10-20 % slower).
constexpr uint32_t kDefaultDelta = 32;
// A relaxation round pulls when its queue's rows hold at least nnz /
// kDefaultPullDiv edges.
constexpr int kDefaultPullDiv = 4;

enum SCtr : int {
  S_QP0 = 0,    // queue 0: entries << 32 | edges (appended to by one atomic per wavefront)
  S_QP1 = 1,    // queue 1: the same
  S_PEND = 2,   // pending vertices left after a scan
  S_MIN = 3,    // smallest distance among them (kInf if none)
  S_ERR = 4,    // 1: a distance exceeded kInf - 1; 4: a tile met more entries than edges
  S_RELAX = 5,  // queue entries relaxed (statistics)
  S_EDGES = 6,  // edges relaxed (statistics)
  S_DONE = 7,   // 1: no queue and no pending vertex left (read by the host)
  S_ROUNDS = 8,   // relaxation steps (statistics)
  S_SCANS = 9,    // scan steps (statistics)
  S_BUCKETS = 10, // thresholds used (statistics)
  S_EPOCH = 11,   // last queue stamp handed out (read back by the host)
  S_TICK0 = 12,   // step tickets, by step parity (S_TICK0 + (j & 1))
  S_PULLS = 14,   // relaxation rounds done by pulling (statistics)
  S_ST0 = 16,     // step state, by step parity: S_ST0 + (j & 1) * kStSlots + ST_*
  S_N = 32
};
// Per-step state.  Step j reads the slots of parity j & 1, which only step
// j - 1 (finished before j starts) and step j + 1 (which starts after j ends)
// write, so a workgroup of step j that starts late still sees its step's state.
enum StSlot : int { ST_QP = 0, ST_CUR = 1, ST_T = 2, ST_EP = 3, ST_DONE = 4 };
constexpr int kStSlots = 8;

// The counters and step states are written by one workgroup and read by the
// workgroups of later steps, which may run on another XCD whose L2 holds an
// older copy of the line: every access is a device-scope atomic.
__device__ __forceinline__ unsigned long long s_ld(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void s_st(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends v (one lane each) to a queue with its first-edge index: a wave
// prefix sum of the degrees and one atomic on the queue's packed counter
// (entries << 32 | edges) per wavefront.  Called by every lane of the wave.
__device__ __forceinline__ void push_wave(bool want, int32_t v, const int64_t *__restrict__ rp,
                                          int32_t *__restrict__ q, uint32_t *__restrict__ qo,
                                          unsigned long long *pack) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  const int lane = __lane_id();
  const uint32_t deg = want ? (uint32_t)(rp[v + 1] - rp[v]) : 0u;
  const uint32_t inc = wave_incl_scan(deg);
  const uint32_t tot = __shfl(inc, kWave - 1, kWave);
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader)
    base = atomicAdd(pack, ((unsigned long long)__popcll(m) << 32) | (unsigned long long)tot);
  base = __shfl(base, leader, kWave);
  if (want) {
    const uint64_t pos = (base >> 32) + (uint64_t)__popcll(m & lanemask_lt());
    q[pos] = v;
    qo[pos] = (uint32_t)base + inc - deg;
  }
}

struct RelaxArgs {
  const int64_t *rp;
  const int32_t *ci;
  const uint8_t *wt;
  unsigned long long *dp;  // per vertex: dist << 32 | predecessor
  uint64_t *pend;
  uint32_t *stamp;
  int32_t *qn;   // next queue
  uint32_t *qon; // its first-edge indices
  unsigned long long *ctr;
  int nxt;
  uint64_t T;
  uint32_t epoch;  // stamp of the next queue
  int64_t n;
  const int32_t *hubs;      // rows longer than kHubDeg (from Kernel 1) and the
  const uint64_t *hub_off;  // first kHubChunk-edge piece of each
  int64_t num_hubs, hub_chunks;
  uint64_t pull_edges;  // a round whose queue has at least this many edges pulls (0: never)
};

// Relaxes edge (u, v) of weight w from distance du; returns true when v must
// join the next queue (its distance improved below T and it is not yet in it).
// A relaxation that reaches v's distance with a smaller-id u only updates the
// predecessor.
__device__ __forceinline__ bool relax(const RelaxArgs &a, uint32_t du, int32_t u, int32_t v,
                                      uint32_t w) {
  const uint64_t nd = (uint64_t)du + w;
  if (nd >= (uint64_t)kInf) {
    atomicOr(a.ctr + S_ERR, 1ull);
    return false;
  }
  const unsigned long long cand = (nd << 32) | (uint32_t)u;
  if (cand >= a.dp[v]) return false;
  const unsigned long long old = atomicMin(a.dp + v, cand);
  if (nd >= (old >> 32)) return false;  // not closer (at most a smaller predecessor)
  if (nd < a.T) return atomicExch(a.stamp + v, a.epoch) != a.epoch;
  const uint64_t bit = 1ull << (v & 63);
  if (!(a.pend[v >> 6] & bit)) atomicOr((unsigned long long *)(a.pend + (v >> 6)), bit);
  return false;
}

// Start: distance infinity (and no predecessor) except the source (0, itself);
// no pending vertex; queue 0 = {src} with the stamp of the first queue;
// counters zeroed.
__global__ void k_sssp_init(unsigned long long *__restrict__ dp, int64_t n, int64_t src,
                            uint64_t *__restrict__ pend, int64_t words, int32_t *__restrict__ q0,
                            uint32_t *__restrict__ qo0, const int64_t *__restrict__ rp,
                            uint32_t *__restrict__ stamp, uint32_t epoch, uint64_t delta,
                            unsigned long long *__restrict__ ctr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < n; i += stride)
    dp[i] = i == src ? (unsigned long long)src : ((unsigned long long)kInf << 32) | 0xffffffffull;
  for (int64_t i = t; i < words; i += stride) pend[i] = 0;
  if (t == 0) {
    for (int i = 0; i < S_N; ++i) s_st(ctr + i, 0ull);
    unsigned long long *st = ctr + S_ST0;  // step 0's state: queue 0 = {src}
    s_st(st + ST_QP, (1ull << 32) | (unsigned long long)(rp[src + 1] - rp[src]));
    s_st(st + ST_CUR, 0ull);
    s_st(st + ST_T, delta);
    s_st(st + ST_EP, (unsigned long long)epoch + 1);
    s_st(ctr + S_MIN, kInf);
    s_st(ctr + S_BUCKETS, 1ull);
    s_st(ctr + S_EPOCH, (unsigned long long)epoch + 1);
    q0[0] = (int32_t)src;
    qo0[0] = 0;
    stamp[src] = epoch;
  }
}

// Edge index of queue entry i in the queue's edge list (non-decreasing in i;
// the total past the last entry).
struct QueueOffsets {
  const uint32_t *qo;
  int64_t qlen;
  uint32_t total;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    return i >= qlen ? total : qo[i];
  }
};

// Largest i in [0, len) with off(i) <= e (off non-decreasing, off(0) = 0 <= e):
// a kBlock-way search, one probe per thread per round.
template <class Off>
__device__ int64_t tile_search(const Off &off, int64_t len, uint32_t e) {
  int64_t lo = 0, hi = len;
  while (true) {
    const int64_t span = hi - lo;
    if (span <= kBlock) {
      const int64_t p = lo + threadIdx.x;
      const int c = __syncthreads_count(p < hi && off(p) <= e);
      return lo + c - 1;
    }
    const int64_t p = lo + (span * (int64_t)threadIdx.x) / kBlock;
    const int c = __syncthreads_count(off(p) <= e);
    const int64_t nlo = lo + (span * (int64_t)(c - 1)) / kBlock;
    const int64_t nhi = (c < kBlock) ? lo + (span * (int64_t)c) / kBlock : hi;
    lo = nlo;
    hi = nhi;
  }
}

// One relaxation round over a queue (qlen entries, total edges): every queue
// vertex leaves the far set, then 1,024-edge tiles of the queue's edge list
// are relaxed by workgroups 0 .. active - 1 in turn; improved vertices below T
// fill queue nxt.
__device__ void relax_round(const int32_t *__restrict__ q, const uint32_t *__restrict__ qo,
                            int64_t qlen, uint32_t total, uint32_t active, const RelaxArgs &a) {
  __shared__ uint32_t s_off[kTile + 1];
  __shared__ int64_t s_base[kTile];
  __shared__ uint32_t s_du[kTile];
  __shared__ int32_t s_u[kTile];
  unsigned long long *npack = a.ctr + S_QP0 + a.nxt;
  // the queue's vertices are relaxed now: they leave the far set (no relaxation
  // of this round can put them back, their distances lie below T)
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < qlen;
       i += (int64_t)active * kBlock) {
    const int32_t u = q[i];
    const uint64_t bit = 1ull << (u & 63);
    if (a.pend[u >> 6] & bit) atomicAnd((unsigned long long *)(a.pend + (u >> 6)), ~bit);
  }
  const QueueOffsets off{qo, qlen, total};
  for (uint64_t tile = blockIdx.x; tile * kTile < total; tile += active) {
    const uint32_t e0 = (uint32_t)(tile * kTile);
    const uint32_t e1 = (uint32_t)std::min<uint64_t>((uint64_t)e0 + kTile, total);
    const int64_t i0 = tile_search(off, qlen, e0);
    const int64_t i1 = tile_search(off, qlen, e1 - 1);
    const int S = (int)(i1 - i0 + 1);
    if (S > kTile) {  // only degree-0 entries could do this, and none are queued
      if (threadIdx.x == 0) atomicOr(a.ctr + S_ERR, 4ull);
      break;
    }
    for (int k = threadIdx.x; k < S; k += kBlock) {
      const uint32_t o = off(i0 + k);
      const int32_t u = q[i0 + k];
      s_off[k] = o;
      s_base[k] = a.rp[u] - (int64_t)o;
      s_du[k] = (uint32_t)(a.dp[u] >> 32);
      s_u[k] = u;
    }
    if (threadIdx.x == 0) s_off[S] = off(i1 + 1);
    __syncthreads();
    int klo = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t e = e0 + j * kBlock + threadIdx.x;
      bool push = false;
      int32_t v = 0;
      if (e < e1) {
        int lo = klo, hi = S;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[mid] <= e)
            lo = mid;
          else
            hi = mid;
        }
        klo = lo;
        const int64_t k = s_base[lo] + (int64_t)e;
        v = a.ci[k];
        push = relax(a, s_du[lo], s_u[lo], v, a.wt[k]);
      }
      push_wave(push, v, a.rp, a.qn, a.qon, npack);
    }
    __syncthreads();  // the shared arrays are reused by the next tile
  }
}

// The packed relaxation (dist[u] + w) << 32 | u of row entry k (edge (u, v) of
// weight w) if u lies in the current queue (stamp == cur), else ~0.
__device__ __forceinline__ unsigned long long pull_entry(const RelaxArgs &a, int64_t k,
                                                         uint32_t cur) {
  const int32_t u = a.ci[k];
  if (a.stamp[u] != cur) return ~0ull;
  const uint64_t du = a.dp[u] >> 32;
  const uint64_t nd = du + a.wt[k];
  if (nd >= (uint64_t)kInf) {  // du < kInf: u is in the queue
    atomicOr(a.ctr + S_ERR, 1ull);
    return ~0ull;
  }
  return (nd << 32) | (uint32_t)u;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) x |= __shfl_xor(x, d, kWave);
  return x;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const unsigned long long o = __shfl_xor(x, d, kWave);
    x = o < x ? o : x;
  }
  return x;
}

// Keeps v's pulled word `best` if it beats `old` (v's word before): v joins
// the next queue when its distance improved below T, else the far set.
// Returns whether v is to be appended (the caller appends by wavefront).
__device__ __forceinline__ bool pull_keep(const RelaxArgs &a, int64_t v,
                                          unsigned long long best, unsigned long long old,
                                          uint64_t &far) {
  if ((best >> 32) >= (old >> 32)) return false;  // at most a smaller predecessor
  if ((best >> 32) < a.T) return atomicExch(a.stamp + v, a.epoch) != a.epoch;
  far |= 1ull << (v & 63);
  return false;
}

// One relaxation round by pulling (queue stamp cur): rows of up to kPullLane
// entries are read by their lane, longer rows up to kHubDeg by the whole
// wavefront, hub rows in kHubChunk-edge pieces spread over the wavefronts.
// The queue's vertices leave the far set first, as in relax_round.  Every
// relaxation of the round is at least `lower` (the start of the current
// bucket, weights being non-negative), so a vertex whose distance is below it
// cannot change, not even its predecessor, and its row is not read.
constexpr int kPullLane = 32;

__device__ void pull_round(const int32_t *__restrict__ q, int64_t qlen, uint32_t active,
                           const RelaxArgs &a, uint32_t cur, uint64_t lower) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < qlen;
       i += (int64_t)active * kBlock) {
    const int32_t u = q[i];
    const uint64_t bit = 1ull << (u & 63);
    if (a.pend[u >> 6] & bit) atomicAnd((unsigned long long *)(a.pend + (u >> 6)), ~bit);
  }
  const int lane = __lane_id();
  const int64_t gw = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)active * kBlock) / kWave;
  const int64_t W = (a.n + kWave - 1) / kWave;
  unsigned long long *npack = a.ctr + S_QP0 + a.nxt;
  for (int64_t w = gw; w < W; w += nw) {
    const int64_t v = w * kWave + lane;
    int64_t b = 0, e = 0;
    unsigned long long mine = 0;
    if (v < a.n) mine = a.dp[v];
    if (v < a.n && (mine >> 32) >= lower) {
      b = a.rp[v];
      e = a.rp[v + 1];
    }
    const int64_t d = e - b;
    unsigned long long best = ~0ull;
    if (d <= kPullLane)
      for (int64_t k = b; k < e; ++k) {
        const unsigned long long c = pull_entry(a, k, cur);
        best = c < best ? c : best;
      }
    uint64_t rem = __ballot(d > kPullLane && d <= kHubDeg);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      unsigned long long m = ~0ull;
      for (int64_t k = kb + lane; k < ke; k += kWave) {
        const unsigned long long c = pull_entry(a, k, cur);
        m = c < m ? c : m;
      }
      m = wave_min_u64(m);
      if (lane == L) best = m;
    }
    bool want = false;
    uint64_t far = 0;
    if (v < a.n && d <= kHubDeg && best != ~0ull && best < mine) {
      // v's word has no other writer in this round; the atomic keeps it so
      const unsigned long long old = atomicMin(a.dp + v, best);
      if (best < old) want = pull_keep(a, v, best, old, far);
    }
    // the far-set bits of the wavefront's vertices share one word
    far = wave_or_u64(far);
    if (far && lane == 0) atomicOr((unsigned long long *)(a.pend + w), far);
    push_wave(want, (int32_t)v, a.rp, a.qn, a.qon, npack);
  }
  for (int64_t c = gw; c < a.hub_chunks; c += nw) {
    int64_t lo = 0, hi = a.num_hubs;  // the hub of piece c: the last i with hub_off[i] <= c
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)a.hub_off[mid] <= c)
        lo = mid;
      else
        hi = mid;
    }
    const int32_t h = a.hubs[lo];
    if ((a.dp[h] >> 32) < lower) continue;  // wave-uniform
    const int64_t kb = a.rp[h] + (c - (int64_t)a.hub_off[lo]) * kHubChunk;
    const int64_t ke = std::min<int64_t>(kb + kHubChunk, a.rp[h + 1]);
    unsigned long long m = ~0ull;
    for (int64_t k = kb + lane; k < ke; k += kWave) {
      const unsigned long long cnd = pull_entry(a, k, cur);
      m = cnd < m ? cnd : m;
    }
    m = wave_min_u64(m);
    bool want = false;
    uint64_t far = 0;
    if (lane == 0 && m != ~0ull) {
      const unsigned long long old = atomicMin(a.dp + h, m);
      if (m < old) want = pull_keep(a, h, m, old, far);
    }
    if (far) atomicOr((unsigned long long *)(a.pend + (h >> 6)), far);
    push_wave(want, h, a.rp, a.qn, a.qon, npack);
  }
  // every wavefront's appends have returned before thread 0 takes the
  // workgroup's ticket (the last workgroup reads the next queue's counter)
  __syncthreads();
}

// Pending vertices with dist < T leave the far set for queue nxt (stamp =
// epoch); the rest are counted and their smallest distance taken.
__device__ void scan_pending(const unsigned long long *__restrict__ dp,
                             const int64_t *__restrict__ rp,
                             uint64_t *__restrict__ pend, int64_t words, uint64_t T,
                             int32_t *__restrict__ qn, uint32_t *__restrict__ qon, int nxt,
                             uint32_t *__restrict__ stamp, uint32_t epoch,
                             unsigned long long *__restrict__ ctr, uint32_t active) {
  const int64_t stride = (int64_t)active * kBlock;
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
        const uint32_t dv = (uint32_t)(dp[v] >> 32);
        if ((uint64_t)dv < T) {
          take |= 1ull << b;
          stamp[v] = epoch;
          push = true;
        } else {
          ++left;
          dmin = std::min(dmin, dv);
        }
      }
      push_wave(push, v, rp, qn, qon, ctr + S_QP0 + nxt);
    }
    if (take) pend[w] = m & ~take;
  }
  __shared__ unsigned long long s_red[kBlock / kWave];
  __shared__ uint32_t s_min[kBlock / kWave];
  const unsigned long long tl = block_sum<kBlock, unsigned long long>(left, s_red);
  uint32_t bm = dmin;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) bm = std::min(bm, (uint32_t)__shfl_xor(bm, d, kWave));
  if (__lane_id() == 0) s_min[threadIdx.x / kWave] = bm;
  __syncthreads();
  // thread 0 adds the block's counts, and has their results back before it
  // takes the workgroup's ticket (the last workgroup reads them)
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / kWave; ++i) bm = std::min(bm, s_min[i]);
    if (tl) s_red[0] = atomicAdd(ctr + S_PEND, tl);
    if (bm != kInf) s_red[1] = atomicMin(ctr + S_MIN, (unsigned long long)bm);
  }
}

// Step j of the traversal; the host queues steps in groups without waiting.
// It relaxes its queue if that holds entries, else it scans the far set below
// the threshold; its last workgroup (a ticket) writes step j + 1's state:
// the queues flip, the threshold moves to the end of the bucket of the
// smallest pending distance after a scan found nothing below it, or the end
// is marked.  Steps queued past the end do nothing.
__global__ __launch_bounds__(kBlock) void k_sssp_step(RelaxArgs a, int64_t j, int32_t *q0,
                                                      int32_t *q1, uint32_t *qo0, uint32_t *qo1,
                                                      int64_t words, uint64_t delta) {
  __shared__ int s_last;
  unsigned long long *ctr = a.ctr;
  unsigned long long *st = ctr + S_ST0 + (int)(j & 1) * kStSlots;
  if (s_ld(st + ST_DONE)) return;
  const unsigned long long qp = s_ld(st + ST_QP);
  const int cur = (int)s_ld(st + ST_CUR);
  const int nxt = cur ^ 1;
  const int64_t qlen = (int64_t)(qp >> 32);
  const uint32_t total = (uint32_t)qp;
  a.T = s_ld(st + ST_T);
  a.epoch = (uint32_t)s_ld(st + ST_EP);
  a.nxt = nxt;
  a.qn = nxt ? q1 : q0;
  a.qon = nxt ? qo1 : qo0;
  // workgroups with work take part (and a ticket): same-address atomics serialise
  const bool pull = qlen > 0 && a.pull_edges > 0 && (uint64_t)total >= a.pull_edges;
  const uint64_t need =
      pull ? ((uint64_t)a.n + kBlock - 1) / kBlock
      : qlen > 0 ? std::max<uint64_t>(((uint64_t)total + kTile - 1) / kTile,
                                      ((uint64_t)qlen + kBlock - 1) / kBlock)
                 : ((uint64_t)words + kBlock - 1) / kBlock;
  const uint32_t active = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(gridDim.x, need));
  if (blockIdx.x >= active) return;
  if (pull)
    pull_round(cur ? q1 : q0, qlen, active, a, a.epoch - 1,  // the queue's stamp
               a.T > delta ? a.T - delta : 0);
  else if (qlen > 0)
    relax_round(cur ? q1 : q0, cur ? qo1 : qo0, qlen, total, active, a);
  else
    scan_pending(a.dp, a.rp, a.pend, words, a.T, a.qn, a.qon, nxt, a.stamp, a.epoch, ctr,
                 active);
  unsigned long long *tick = ctr + S_TICK0 + (int)(j & 1);
  if (threadIdx.x == 0) s_last = atomicAdd(tick, 1ull) + 1 == active;
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  // every workgroup's pushes and counts returned before its ticket
  const unsigned long long np = atomicAdd(ctr + S_QP0 + nxt, 0ull);
  unsigned long long *ns = ctr + S_ST0 + (int)((j + 1) & 1) * kStSlots;
  unsigned long long T = a.T, done = 0;
  if (qlen > 0) {
    s_st(ctr + S_ROUNDS, s_ld(ctr + S_ROUNDS) + 1);
    s_st(ctr + S_RELAX, s_ld(ctr + S_RELAX) + (unsigned long long)qlen);
    s_st(ctr + S_EDGES, s_ld(ctr + S_EDGES) + (unsigned long long)total);
    if (pull) s_st(ctr + S_PULLS, s_ld(ctr + S_PULLS) + 1);
  } else {
    s_st(ctr + S_SCANS, s_ld(ctr + S_SCANS) + 1);
    if ((np >> 32) == 0) {
      // nothing below T: done without pending vertices, else the next scan
      // uses the end of the bucket of the smallest pending distance
      const unsigned long long left = atomicAdd(ctr + S_PEND, 0ull);
      const unsigned long long mn = atomicAdd(ctr + S_MIN, 0ull);
      if (left == 0) {
        done = 1;
      } else {
        T = (mn / delta + 1) * delta;
        s_st(ctr + S_BUCKETS, s_ld(ctr + S_BUCKETS) + 1);
      }
    }
    atomicExch(ctr + S_PEND, 0ull);
    atomicExch(ctr + S_MIN, (unsigned long long)kInf);
  }
  s_st(ns + ST_QP, np);
  s_st(ns + ST_CUR, (unsigned long long)nxt);
  s_st(ns + ST_T, T);
  s_st(ns + ST_EP, (unsigned long long)a.epoch + 1);
  s_st(ns + ST_DONE, done);
  s_st(ctr + S_EPOCH, (unsigned long long)a.epoch + 1);
  if (done) {
    // both parities: every later step finds the end, whichever state it reads
    // (every workgroup of this step has passed its check of st already)
    s_st(st + ST_DONE, 1ull);
    s_st(ctr + S_DONE, 1ull);
  }
  atomicExch(ctr + S_QP0 + cur, 0ull);  // the consumed queue is step j + 1's output
  atomicExch(tick, 0ull);
}

// dist[v] and prev[v] from v's packed word: infinity and -1 where unreached,
// the source its own predecessor.
__global__ void k_sssp_unpack(const unsigned long long *__restrict__ dp, int64_t n, int64_t src,
                              uint32_t *__restrict__ dist, int32_t *__restrict__ prev) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const unsigned long long x = dp[v];
    const uint32_t d = (uint32_t)(x >> 32);
    dist[v] = d;
    prev[v] = d == kInf ? -1 : (v == src ? (int32_t)src : (int32_t)(uint32_t)x);
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
  if (dp) (void)hipFree(dp);
  if (stamp) (void)hipFree(stamp);
  for (auto *p : q)
    if (p) (void)hipFree(p);
  for (auto *p : qo)
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
  A((void **)&w->dp, g->n * 8);
  A((void **)&w->stamp, g->n * 4);
  A((void **)&w->q[0], g->n * 4);
  A((void **)&w->q[1], g->n * 4);
  A((void **)&w->qo[0], g->n * 4);
  A((void **)&w->qo[1], g->n * 4);
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
                     s, w.dp, n, src, w.pend, W, w.q[0], w.qo[0], g->row_ptr, w.stamp, ep, delta,
                     ctr);
  G5_LAUNCH_CHECK();
  RelaxArgs a{};
  a.rp = g->row_ptr;
  a.ci = g->col_idx;
  a.wt = g->wt;
  a.dp = w.dp;
  a.pend = w.pend;
  a.stamp = w.stamp;
  a.ctr = ctr;
  a.n = n;
  a.hubs = g->hub_list;
  a.hub_off = g->hub_off;
  a.num_hubs = g->num_hubs;
  a.hub_chunks = g->hub_chunks;
  // rounds whose queue holds at least nnz / pull_div edges pull
  const int pull_div = p.pull_div != 0 ? p.pull_div : kDefaultPullDiv;
  a.pull_edges = pull_div > 0 ? std::max<uint64_t>(1, (uint64_t)g->nnz / (uint64_t)pull_div) : 0;
  // steps are queued in groups; the host reads the counters once per group
  unsigned long long hc[S_N] = {};
  int64_t steps = 0;
  for (int group = 8;; group = 16) {
    for (int i = 0; i < group; ++i, ++steps)
      hipLaunchKernelGGL(k_sssp_step, dim3(grid), dim3(kBlock), 0, s, a, steps, w.q[0], w.q[1],
                         w.qo[0], w.qo[1], W, delta);
    G5_LAUNCH_CHECK();
    G5_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
    G5_HIP(hipStreamSynchronize(s));
    if (hc[S_ERR]) {
      set_error(hc[S_ERR] & 1 ? "g5_sssp: a distance exceeds 2^32 - 2"
                              : "g5_sssp: a relaxation tile met more queue entries than edges");
      return (hc[S_ERR] & 1) ? G5_ERANGE : G5_EDEVICE;
    }
    if (hc[S_DONE]) break;
  }
  w.epoch = (uint32_t)hc[S_EPOCH];
  hipLaunchKernelGGL(k_sssp_unpack, dim3(grid_blocks(n, 256, ncu * 16)), dim3(256), 0, s,
                     (const unsigned long long *)w.dp, n, src, dist, prev);
  G5_LAUNCH_CHECK();
  if (timed) G5_HIP(hipEventRecord(w.ev[1], s));
  G5_HIP(hipStreamSynchronize(s));
  if (stats) {
    *stats = g5_sssp_stats{};
    stats->rounds = (int64_t)hc[S_ROUNDS];
    stats->scans = (int64_t)hc[S_SCANS];
    stats->buckets = (int64_t)hc[S_BUCKETS];
    stats->relaxed = (int64_t)hc[S_RELAX];
    stats->edges = (int64_t)hc[S_EDGES];
    stats->pulls = (int64_t)hc[S_PULLS];
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
