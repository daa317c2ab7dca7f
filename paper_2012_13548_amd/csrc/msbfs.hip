// Batched breadth-first search from up to 64 roots in one persistent launch.
//
// Each vertex carries 64-bit masks (bit b = roots[b]): seen (roots that have
// reached it) and frontier (roots whose level-l frontier contains it), as in
// multi-source BFS (Then et al., "The More the Merrier", VLDB 2014).  One pass
// over the graph per level serves every root.  Levels stay synchronous
// (Section 2.3.2 of the paper): a grid-wide barrier separates levels inside a
// cooperative launch.
//
//   top-down  for u with frontier[u] != 0 and each neighbour v:
//             new = frontier[u] & ~seen[v]; the atomic OR of new into next[v]
//             returns the bits this edge won, and each won bit b gives
//             level[b][v] = l+1, parent[b][v] = u
//   bottom-up for v with seen[v] != all: OR frontier[u] & missing over its row
//             (stop early once every missing bit is found); the first
//             neighbour providing bit b is parent[b][v]
//   hubs      rows longer than kHubDeg are split into kHubChunk-edge pieces
//             spread over all wavefronts (list built by Kernel 1)
//
// Frontier masks rotate through three buffers: at level l buffer l%3 is read,
// (l+1)%3 receives the next frontier and (l+2)%3 (the previous frontier) is
// cleared for level l+1.  Level counters rotate the same way.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cstring>

#include "g5_internal.h"

namespace cg = cooperative_groups;

namespace g5 {
namespace {

constexpr int kBlock = 256;
constexpr int kLaneRow = 32;  // rows up to this length are scanned by one lane
// A lane's row goes in batches of kRowBatch entries: their neighbour ids, then
// the masks they index, loaded together, so a batch costs two dependent loads
// rather than two per entry.
constexpr int kRowBatch = 8;
constexpr int kStatLevels = G5_MAX_STAT_LEVELS;

struct Slot {
  unsigned long long nf;   // vertices with a nonzero frontier mask
  unsigned long long mf;   // their degree sum
  unsigned long long dec;  // degree sum of vertices that became fully seen
  unsigned long long pad;
};

struct MsCtl;

struct MsArgs {
  const int64_t *rp;
  const int32_t *ci;
  int64_t n;
  uint64_t full;
  uint64_t *seen;
  uint64_t *buf0, *buf1, *buf2;
  int8_t *levels;
  int32_t *parents;
  const int32_t *hub_list;
  const uint64_t *hub_off;
  int64_t num_hubs;
  int64_t hub_chunks;
  const int32_t *hint;  // per vertex: its highest-degree neighbour (-1: none), from Kernel 1
  MsCtl *ctl;
  double alpha;
  int direction;
  int max_level;
};

struct MsCtl {
  Slot slot[3];
  unsigned long long mu0;  // degree sum of vertices not yet seen by every root
  unsigned long long err;
  unsigned long long nlevels;
  unsigned long long mu_lv[2];  // stepped mode: m_u at the start of level l, by parity
  unsigned long long lbase;     // graph replays: the first level of the next replay
  unsigned long long pad;
  MsArgs args;                  // graph replays: the arguments of this batch
  int64_t frontier[kStatLevels];
  int32_t dir[kStatLevels];
};

// The roots of a batch, passed by value to the seeding kernel (no copy of
// them to device memory is needed).
struct Roots64 {
  int64_t r[64];
};

__device__ __forceinline__ unsigned long long ld_agent(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) x |= __shfl_xor(x, d, kWave);
  return x;
}

// Hub owning work item c: largest i with hub_off[i] <= c.
__device__ __forceinline__ int64_t hub_of(const MsArgs &a, uint64_t c) {
  int64_t lo = 0, hi = a.num_hubs;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (a.hub_off[mid] <= c)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

struct Acc {
  uint64_t nf = 0, mf = 0, dec = 0;
};

// Records the bits `won` of vertex v (already OR-ed into next[v], which held
// `old`): seen, levels, parents and the frontier counters.
template <bool PAR>
__device__ __forceinline__ void commit_atomic(const MsArgs &a, int64_t v, uint64_t won,
                                              uint64_t old, int32_t par, int8_t lvl,
                                              Acc &acc) {
  uint64_t ps = atomicOr((unsigned long long *)&a.seen[v], (unsigned long long)won);
  int64_t d = -1;
  if (old == 0) {
    d = a.rp[v + 1] - a.rp[v];
    acc.nf += 1;
    acc.mf += (uint64_t)d;
  }
  if ((ps | won) == a.full && ps != a.full) {
    if (d < 0) d = a.rp[v + 1] - a.rp[v];
    acc.dec += (uint64_t)d;
  }
  while (won) {
    const int b = __ffsll((unsigned long long)won) - 1;
    won &= won - 1;
    a.levels[(int64_t)b * a.n + v] = lvl;
    if (PAR) a.parents[(int64_t)b * a.n + v] = par;
  }
}

template <bool PAR>
__device__ __forceinline__ void td_edge(const MsArgs &a, uint64_t *next, int32_t u, uint64_t fu,
                                        int32_t v, int8_t lvl, Acc &acc) {
  const uint64_t nw = fu & ~a.seen[v];
  if (!nw) return;
  const uint64_t old = atomicOr((unsigned long long *)&next[v], (unsigned long long)nw);
  const uint64_t won = nw & ~old;
  if (won) commit_atomic<PAR>(a, v, won, old, u, lvl, acc);
}

template <bool PAR>
__device__ void td_phase(const MsArgs &a, const uint64_t *front, uint64_t *next, int8_t lvl,
                         int64_t gw, int64_t nw, Acc &acc) {
  const int lane = __lane_id();
  const int64_t W = (a.n + kWave - 1) / kWave;
  for (int64_t w = gw; w < W; w += nw) {
    const int64_t u = w * kWave + lane;
    const uint64_t f = (u < a.n) ? front[u] : 0;
    if (__ballot(f != 0) == 0) continue;
    int64_t b = 0, e = 0;
    if (f) {
      b = a.rp[u];
      e = a.rp[u + 1];
    }
    const int64_t d = e - b;
    if (f && d <= kLaneRow)
      for (int64_t k0 = b; k0 < e; k0 += kRowBatch) {
        int32_t vv[kRowBatch];
        uint64_t nw[kRowBatch], old[kRowBatch];
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) vv[t] = k0 + t < e ? a.ci[k0 + t] : -1;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) nw[t] = vv[t] >= 0 ? f & ~a.seen[vv[t]] : 0ull;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t)
          old[t] = nw[t] ? atomicOr((unsigned long long *)&next[vv[t]], (unsigned long long)nw[t])
                         : ~0ull;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) {
          const uint64_t won = nw[t] & ~old[t];
          if (won) commit_atomic<PAR>(a, vv[t], won, old[t], (int32_t)u, lvl, acc);
        }
      }
    uint64_t rem = __ballot(f && d > kLaneRow && d <= kHubDeg);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      const uint64_t fL = __shfl(f, L, kWave);
      const int32_t uL = (int32_t)(w * kWave + L);
      for (int64_t k = kb + lane; k < ke; k += kWave) td_edge<PAR>(a, next, uL, fL, a.ci[k], lvl, acc);
    }
  }
  for (int64_t c = gw; c < a.hub_chunks; c += nw) {
    const int64_t i = hub_of(a, (uint64_t)c);
    const int32_t h = a.hub_list[i];
    const uint64_t fh = front[h];
    if (!fh) continue;
    const int64_t kb = a.rp[h] + (int64_t)((uint64_t)c - a.hub_off[i]) * kHubChunk;
    const int64_t ke = std::min<int64_t>(kb + kHubChunk, a.rp[h + 1]);
    for (int64_t k = kb + lane; k < ke; k += kWave) td_edge<PAR>(a, next, h, fh, a.ci[k], lvl, acc);
  }
}

// Parents of the bits `found` of vertex v from one 64-edge step: lane with the
// lowest index providing bit b (its neighbour u) is parent[b][v].
template <bool PAR>
__device__ __forceinline__ void step_parents(const MsArgs &a, int64_t v, uint64_t found,
                                             uint64_t g, int32_t u) {
  if (!PAR) return;
  const int lane = __lane_id();
  while (found) {
    const int b = __ffsll((unsigned long long)found) - 1;
    found &= found - 1;
    const int pl = __ffsll((unsigned long long)__ballot((g >> b) & 1)) - 1;
    const int32_t pu = __shfl(u, pl, kWave);
    if (lane == 0) a.parents[(int64_t)b * a.n + v] = pu;
  }
}

template <bool PAR>
__device__ void bu_phase(const MsArgs &a, const uint64_t *front, uint64_t *next, int8_t lvl,
                         int64_t gw, int64_t nw, Acc &acc) {
  const int lane = __lane_id();
  const int64_t W = (a.n + kWave - 1) / kWave;
  for (int64_t w = gw; w < W; w += nw) {
    const int64_t v = w * kWave + lane;
    const uint64_t s = (v < a.n) ? a.seen[v] : a.full;
    int64_t b = 0, e = 0;
    if (s != a.full) {
      b = a.rp[v];
      e = a.rp[v + 1];
    }
    const int64_t d = e - b;
    const bool act = s != a.full && d > 0 && d <= kHubDeg;  // hubs: chunk loop below
    if (__ballot(act) == 0) continue;
    const uint64_t missing = a.full & ~s;
    uint64_t got = 0;
    // the highest-degree neighbour first: a hub in many roots' frontiers often
    // provides every missing bit at once, and the row is not read
    if (act && a.hint) {
      const int32_t h = a.hint[v];
      if (h >= 0) {
        got = front[h] & missing;
        if (PAR) {
          uint64_t x = got;
          while (x) {
            const int bb = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            a.parents[(int64_t)bb * a.n + v] = h;
          }
        }
      }
    }
    if (act && d <= kLaneRow && got != missing) {
      // entries in row order, so the first provider of a bit is its parent; a
      // batch past the point where every missing bit is found contributes nothing
      for (int64_t k0 = b; k0 < e && got != missing; k0 += kRowBatch) {
        int32_t uu[kRowBatch];
        uint64_t fu[kRowBatch];
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) uu[t] = k0 + t < e ? a.ci[k0 + t] : -1;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) fu[t] = uu[t] >= 0 ? front[uu[t]] : 0ull;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) {
          const uint64_t g = fu[t] & missing & ~got;
          if (g) {
            got |= g;
            if (PAR) {
              uint64_t x = g;
              while (x) {
                const int bb = __ffsll((unsigned long long)x) - 1;
                x &= x - 1;
                a.parents[(int64_t)bb * a.n + v] = uu[t];
              }
            }
          }
        }
      }
    }
    uint64_t rem = __ballot(act && d > kLaneRow && got != missing);
    while (rem) {
      const int L = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int64_t kb = __shfl(b, L, kWave), ke = __shfl(e, L, kWave);
      const uint64_t mL = __shfl(missing, L, kWave);
      const int64_t vL = w * kWave + L;
      uint64_t gotL = __shfl(got, L, kWave);  // the hint's bits
      for (int64_t c = kb; c < ke; c += kWave) {
        const int64_t k = c + lane;
        int32_t u = -1;
        uint64_t g = 0;
        if (k < ke) {
          u = a.ci[k];
          g = front[u] & mL;
        }
        const uint64_t fresh = wave_or(g) & ~gotL;
        if (fresh) {
          step_parents<PAR>(a, vL, fresh, g, u);
          gotL |= fresh;
          if (gotL == mL) break;
        }
      }
      if (lane == L) got = gotL;
    }
    if (got) {
      next[v] = got;
      a.seen[v] = s | got;
      acc.nf += 1;
      acc.mf += (uint64_t)d;
      if ((s | got) == a.full) acc.dec += (uint64_t)d;
    }
    uint64_t any = wave_or(got);
    while (any) {  // one coalesced byte row per root
      const int bb = __ffsll((unsigned long long)any) - 1;
      any &= any - 1;
      if ((got >> bb) & 1) a.levels[(int64_t)bb * a.n + v] = lvl;
    }
  }
  for (int64_t c = gw; c < a.hub_chunks; c += nw) {
    const int64_t i = hub_of(a, (uint64_t)c);
    const int32_t h = a.hub_list[i];
    const uint64_t sh = a.seen[h];
    if (sh == a.full) continue;
    const uint64_t mh = a.full & ~sh;
    const int64_t kb = a.rp[h] + (int64_t)((uint64_t)c - a.hub_off[i]) * kHubChunk;
    const int64_t ke = std::min<int64_t>(kb + kHubChunk, a.rp[h + 1]);
    uint64_t gotc = 0;
    for (int64_t cc = kb; cc < ke; cc += kWave) {
      const int64_t k = cc + lane;
      int32_t u = -1;
      uint64_t g = 0;
      if (k < ke) {
        u = a.ci[k];
        g = front[u] & mh;
      }
      const uint64_t fresh = wave_or(g) & ~gotc;
      if (!fresh) continue;
      gotc |= fresh;
      uint64_t old = 0;
      if (lane == 0) old = atomicOr((unsigned long long *)&next[h], (unsigned long long)fresh);
      old = __shfl(old, 0, kWave);
      const uint64_t won = fresh & ~old;
      if (won) {
        step_parents<PAR>(a, h, won, g, u);
        if (lane == 0) commit_atomic<false>(a, h, won, old, -1, lvl, acc);
      }
      if (gotc == mh) break;
    }
  }
}

// One level l: expands buffer l%3 into (l+1)%3 top-down or bottom-up, clears
// (l+2)%3, and adds the next frontier's counters into slot (l+1)%3.
template <bool PAR>
__device__ void level_body(const MsArgs &a, int l, bool td, uint64_t nf, uint64_t *s_red) {
  MsCtl *ctl = a.ctl;
  const int64_t gtid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t gthreads = (int64_t)gridDim.x * kBlock;
  const int64_t gw = gtid / kWave, nw = gthreads / kWave;
  Slot *nxt = &ctl->slot[(l + 1) % 3], *old = &ctl->slot[(l + 2) % 3];
  if (gtid == 0) {
    atomicExch(&old->nf, 0ull);
    atomicExch(&old->mf, 0ull);
    atomicExch(&old->dec, 0ull);
    ctl->nlevels = (unsigned long long)(l + 1);
    if (l < kStatLevels) {
      ctl->dir[l] = td ? 1 : 2;
      ctl->frontier[l] = (int64_t)nf;
    }
  }
  uint64_t *bufs[3] = {a.buf0, a.buf1, a.buf2};
  const uint64_t *front = bufs[l % 3];
  uint64_t *next = bufs[(l + 1) % 3];
  uint64_t *clr = bufs[(l + 2) % 3];
  for (int64_t v = gtid; v < a.n; v += gthreads) clr[v] = 0;
  Acc acc;
  if (td)
    td_phase<PAR>(a, front, next, (int8_t)(l + 1), gw, nw, acc);
  else
    bu_phase<PAR>(a, front, next, (int8_t)(l + 1), gw, nw, acc);
  const uint64_t tnf = block_sum<kBlock, uint64_t>(acc.nf, s_red);
  const uint64_t tmf = block_sum<kBlock, uint64_t>(acc.mf, s_red);
  const uint64_t tdec = block_sum<kBlock, uint64_t>(acc.dec, s_red);
  if (threadIdx.x == 0) {
    if (tnf) atomicAdd(&nxt->nf, (unsigned long long)tnf);
    if (tmf) atomicAdd(&nxt->mf, (unsigned long long)tmf);
    if (tdec) atomicAdd(&nxt->dec, (unsigned long long)tdec);
  }
}

__device__ __forceinline__ bool choose_td(const MsArgs &a, uint64_t mf, uint64_t mu) {
  return a.direction == G5_DIR_TOPDOWN ||
         (a.direction == G5_DIR_AUTO && (double)mf <= (double)mu / a.alpha);
}

// Every level in one cooperative launch, a grid barrier after each level.
template <bool PAR>
__global__ __launch_bounds__(kBlock) void k_msbfs(MsArgs a) {
  cg::grid_group grid = cg::this_grid();
  if (!grid.is_valid()) return;  // only a cooperative launch may run this kernel
  __shared__ uint64_t s_red[kBlock / kWave];
  MsCtl *ctl = a.ctl;
  const int64_t gtid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint64_t mu = ld_agent(&ctl->mu0);  // the seeding kernel left the root level's counters
  for (int l = 0;; ++l) {
    Slot *cur = &ctl->slot[l % 3], *nxt = &ctl->slot[(l + 1) % 3];
    const uint64_t nf = ld_agent(&cur->nf), mf = ld_agent(&cur->mf);
    if (nf == 0) break;
    level_body<PAR>(a, l, choose_td(a, mf, mu), nf, s_red);
    grid.sync();
    mu -= ld_agent(&nxt->dec);
    if (l + 1 > a.max_level && ld_agent(&nxt->nf) != 0) {
      // a vertex lies deeper than int8 can hold (its level byte wrapped)
      if (gtid == 0) atomicExch(&ctl->err, 1ull);
      break;
    }
  }
}

// Stepped mode: the same level as a plain launch (the kernel boundary is the
// level barrier), so batches can share the device with other work.

// Level l takes its own direction decision from the counters the previous
// level left (every workgroup computes the same one), so the host can queue
// levels ahead: a level whose frontier is empty (the traversal ended earlier)
// does nothing, and one deeper than int8 levels allow flags the error.  m_u at
// the start of level l is kept by parity: m_u(l) = m_u(l - 1) - the degree sum
// of vertices that level l - 1 made fully seen.
template <bool PAR>
__global__ __launch_bounds__(kBlock) void k_ms_level(MsArgs a, int l) {
  __shared__ uint64_t s_red[kBlock / kWave];
  MsCtl *ctl = a.ctl;
  Slot *cur = &ctl->slot[l % 3];
  const uint64_t nf = ld_agent(&cur->nf), mf = ld_agent(&cur->mf);
  if (nf == 0) return;
  if (l > a.max_level) {  // a vertex lies deeper than int8 can hold
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(&ctl->err, 1ull);
    return;
  }
  const uint64_t mu =
      l == 0 ? ld_agent(&ctl->mu0) : ld_agent(&ctl->mu_lv[(l - 1) & 1]) - ld_agent(&cur->dec);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(&ctl->mu_lv[l & 1], mu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  level_body<PAR>(a, l, choose_td(a, mf, mu), nf, s_red);
}

// Graph replays: the same level as k_ms_level, with the arguments and the
// level number read from ctl (level = ctl->lbase + j), so one instantiated
// graph of kGraphLevels level nodes and a final k_ms_advance serves every
// group of levels of every batch that uses this workspace.
template <bool PAR>
__global__ __launch_bounds__(kBlock) void k_ms_level_g(MsCtl *ctl, int j) {
  const MsArgs a = ctl->args;
  const int l = (int)ld_agent(&ctl->lbase) + j;
  __shared__ uint64_t s_red[kBlock / kWave];
  Slot *cur = &ctl->slot[l % 3];
  const uint64_t nf = ld_agent(&cur->nf), mf = ld_agent(&cur->mf);
  if (nf == 0) return;
  if (l > a.max_level) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(&ctl->err, 1ull);
    return;
  }
  const uint64_t mu =
      l == 0 ? ld_agent(&ctl->mu0) : ld_agent(&ctl->mu_lv[(l - 1) & 1]) - ld_agent(&cur->dec);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(&ctl->mu_lv[l & 1], mu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  level_body<PAR>(a, l, choose_td(a, mf, mu), nf, s_red);
}

// Moves the level base of graph replays on by the levels one replay runs.
__global__ void k_ms_advance(MsCtl *ctl, int levels) {
  if (threadIdx.x == 0)
    __hip_atomic_store(&ctl->lbase, ld_agent(&ctl->lbase) + (unsigned long long)levels,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fill_i8(int8_t *__restrict__ p, int64_t len, bool vec) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t n16 = vec ? len / 16 : 0;
  int4 m1 = make_int4(-1, -1, -1, -1);
  for (int64_t i = t; i < n16; i += stride) reinterpret_cast<int4 *>(p)[i] = m1;
  for (int64_t i = n16 * 16 + t; i < len; i += stride) p[i] = -1;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t len, bool vec) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t n4 = vec ? len / 4 : 0;
  int4 m1 = make_int4(-1, -1, -1, -1);
  for (int64_t i = t; i < n4; i += stride) reinterpret_cast<int4 *>(p)[i] = m1;
  for (int64_t i = n4 * 4 + t; i < len; i += stride) p[i] = -1;
}

__global__ void k_zero_words(uint64_t *__restrict__ p, int64_t len) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

// Seeds the roots (seen and frontier bits, level 0, parent = itself) and the
// root level's counters in the zeroed ctl: n_f = the distinct roots, m_f their
// degree sum, and m_u (degree sum of the vertices not yet seen by every root)
// = nnz minus the degree of a vertex every root has seen, which happens only
// when all roots are one vertex.  One thread per root.
__global__ void k_ms_seed(Roots64 roots_v, int k, int64_t n, uint64_t *seen, uint64_t *front,
                          int8_t *levels, int32_t *parents, const int64_t *__restrict__ rp,
                          MsCtl *ctl, MsArgs args) {
  const int64_t *roots = roots_v.r;
  int b = threadIdx.x;
  if (b == 0) {
    ctl->args = args;
    __hip_atomic_store(&ctl->lbase, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (b >= k) return;
  int64_t v = roots[b];
  atomicOr((unsigned long long *)&seen[v], 1ull << b);
  atomicOr((unsigned long long *)&front[v], 1ull << b);
  levels[(int64_t)b * n + v] = 0;
  if (parents) parents[(int64_t)b * n + v] = (int32_t)v;
  const int64_t d = rp[v + 1] - rp[v];
  bool first = true;  // the first of equal roots counts the vertex
  for (int c = 0; c < b; ++c)
    if (roots[c] == v) {
      first = false;
      break;
    }
  if (first) {
    atomicAdd(&ctl->slot[0].nf, 1ull);
    atomicAdd(&ctl->slot[0].mf, (unsigned long long)d);
  }
  if (b == 0) {
    bool all = true;
    for (int c = 1; c < k; ++c)
      if (roots[c] != v) {
        all = false;
        break;
      }
    __hip_atomic_store(&ctl->mu0, (unsigned long long)(rp[n] - (all ? d : 0)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

BatchWork::~BatchWork() {
  for (auto &x : gexec)
    if (x) (void)hipGraphExecDestroy(x);
  if (seen) (void)hipFree(seen);
  for (auto *b : buf)
    if (b) (void)hipFree(b);
  if (ctl) (void)hipFree(ctl);
  if (host_ctl) (void)hipHostFree(host_ctl);
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
}

namespace {
g5_status alloc_batch(const g5_csr *g, BatchWork **out) {
  BatchWork *w = new BatchWork();
  w->n = g->n;
  hipError_t e = hipSuccess;
  auto A = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  A((void **)&w->seen, g->n * 8);
  for (auto &b : w->buf) A((void **)&b, g->n * 8);
  A(&w->ctl, sizeof(MsCtl));
  if (e == hipSuccess) e = hipHostMalloc(&w->host_ctl, sizeof(MsCtl), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error(std::string("g5_bfs_batch workspace: ") + hipGetErrorString(e));
    delete w;
    return e == hipErrorOutOfMemory ? G5_ENOMEM : G5_EDEVICE;
  }
  *out = w;
  return G5_OK;
}

struct BatchLease {
  const g5_csr *g;
  BatchWork *w = nullptr;
  ~BatchLease() {
    if (w) {
      std::lock_guard<std::mutex> lk(g->mu);
      g->batch_pool.push_back(w);
    }
  }
};

// Device workspace of one batch (a pooled BatchWork, or the library's fixed
// scratch array) and the host buffer the level counters are read into.
struct BatchSpace {
  uint64_t *seen;
  uint64_t *buf[3];
  MsCtl *ctl;
  MsCtl *host_ctl;
  hipEvent_t ev[2];
};

// Output fills, zeroed masks and counters, the roots seeded; fills `a`.
g5_status batch_start(const g5_csr *g, const BatchSpace &ws, const int64_t *roots, int k,
                      int32_t *parents, int8_t *levels, hipStream_t s, const g5_batch_params &p,
                      MsArgs &a) {
  const int64_t n = g->n;
  const int fg = g->num_cu * 16;
  hipLaunchKernelGGL(k_fill_i8, dim3(grid_for((int64_t)k * n / 16, 256, fg)), dim3(256), 0, s,
                     levels, (int64_t)k * n, ((uintptr_t)levels & 15) == 0);
  if (parents)
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)k * n / 4, 256, fg)), dim3(256), 0, s,
                       parents, (int64_t)k * n, ((uintptr_t)parents & 15) == 0);
  hipLaunchKernelGGL(k_zero_words, dim3(grid_for(n, 256, fg)), dim3(256), 0, s, ws.seen, n);
  // buf[2] is cleared by level 0 before level 1 fills it
  for (int i = 0; i < 2; ++i)
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(n, 256, fg)), dim3(256), 0, s, ws.buf[i], n);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (uint64_t *)ws.ctl,
                     (int64_t)(sizeof(MsCtl) / 8));
  a.rp = g->row_ptr;
  a.ci = g->col_idx;
  a.n = n;
  a.full = (k == 64) ? ~0ull : ((1ull << k) - 1);
  a.seen = ws.seen;
  a.buf0 = ws.buf[0];
  a.buf1 = ws.buf[1];
  a.buf2 = ws.buf[2];
  a.levels = levels;
  a.parents = parents;
  a.hub_list = g->hub_list;
  a.hub_off = g->hub_off;
  a.num_hubs = g->num_hubs;
  a.hub_chunks = g->hub_chunks;
  a.hint = (p.flags & G5_FLAG_NO_HINT) ? nullptr : g->hint_id;
  a.ctl = ws.ctl;
  a.alpha = p.alpha > 0 ? p.alpha : g->tune.batch_alpha;
  a.direction = p.direction;
  a.max_level = 127;
  Roots64 rv{};
  for (int i = 0; i < k; ++i) rv.r[i] = roots[i];
  hipLaunchKernelGGL(k_ms_seed, dim3(1), dim3(64), 0, s, rv, k, n, ws.seen, ws.buf[0], levels,
                     parents, g->row_ptr, ws.ctl, a);
  G5_LAUNCH_CHECK();
  return G5_OK;
}

g5_status read_ctl(const BatchSpace &ws, hipStream_t s) {
  G5_HIP(hipMemcpyAsync(ws.host_ctl, ws.ctl, sizeof(MsCtl), hipMemcpyDeviceToHost, s));
  G5_HIP(hipStreamSynchronize(s));
  return G5_OK;
}

// After `queued` levels ran (or exited at once past the end): done when fewer
// levels ran than were queued (one found its frontier empty), or the frontier
// of the next level is empty (its slot was cleared by level queued - 2 and
// filled by level queued - 1, both of which ran).
bool batch_done(const MsCtl *hc, int queued) {
  return (int)hc->nlevels < queued || hc->slot[queued % 3].nf == 0;
}

g5_status batch_finish(const BatchSpace &ws, const MsArgs &a, int blocks, bool timed,
                       g5_batch_stats *stats) {
  const MsCtl *hc = ws.host_ctl;
  if (stats) {
    *stats = g5_batch_stats{};
    stats->nlevels = (int32_t)hc->nlevels;
    for (int i = 0; i < std::min<int>((int)hc->nlevels, kStatLevels); ++i) {
      stats->dir[i] = hc->dir[i];
      stats->frontier[i] = hc->frontier[i];
    }
    stats->grid_blocks = blocks;
    stats->alpha = a.alpha;
    if (timed) {
      float ms = 0;
      G5_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]));
      stats->launch_ms = ms;
    }
  }
  if (hc->err) {
    set_error("g5_bfs_batch: a level exceeds 127 (int8 levels); use g5_bfs for this root set");
    return G5_ERANGE;
  }
  return G5_OK;
}

// Stepped batch: one launch per level, each taking its own direction
// decision on the device.  The host queues levels in groups (8, then 4 at a
// time) and reads the counters once per group instead of once per level; the
// levels queued past the end do nothing.
g5_status batch_stepped(const g5_csr *g, const BatchSpace &ws, const MsArgs &a, hipStream_t s,
                        bool timed, g5_batch_stats *stats, int bpc) {
  const int blocks = g->num_cu * bpc;
  if (timed) G5_HIP(hipEventRecord(ws.ev[0], s));
  int l = 0;  // levels queued
  for (int group = 8;; group = 4) {
    for (int j = 0; j < group; ++j, ++l) {
      if (a.parents)
        hipLaunchKernelGGL(k_ms_level<true>, dim3(blocks), dim3(kBlock), 0, s, a, l);
      else
        hipLaunchKernelGGL(k_ms_level<false>, dim3(blocks), dim3(kBlock), 0, s, a, l);
    }
    G5_LAUNCH_CHECK();
    g5_status st = read_ctl(ws, s);
    if (st != G5_OK) return st;
    if (ws.host_ctl->err || batch_done(ws.host_ctl, l)) break;
  }
  if (timed) {
    G5_HIP(hipEventRecord(ws.ev[1], s));
    G5_HIP(hipStreamSynchronize(s));
  }
  return batch_finish(ws, a, blocks, timed, stats);
}

// The graph of one replay: kGraphLevels level kernels (k_ms_level_g, level =
// ctl->lbase + j) and k_ms_advance, in a chain of kernel nodes (no memset or
// copy nodes).  Built once per workspace, parents mode and grid; the batch's
// arguments travel in ctl (written by the seeding kernel).
constexpr int kGraphLevels = 8;

g5_status graph_exec(BatchWork &w, bool par, int blocks, hipGraphExec_t *out) {
  const int i = par ? 1 : 0;
  if (w.gexec[i] && w.gblocks[i] == blocks) {
    *out = w.gexec[i];
    return G5_OK;
  }
  if (w.gexec[i]) {
    G5_HIP(hipGraphExecDestroy(w.gexec[i]));
    w.gexec[i] = nullptr;
  }
  hipGraph_t graph = nullptr;
  G5_HIP(hipGraphCreate(&graph, 0));
  MsCtl *ctl = (MsCtl *)w.ctl;
  hipGraphNode_t prev = nullptr;
  int js[kGraphLevels];
  hipError_t e = hipSuccess;
  for (int j = 0; j <= kGraphLevels && e == hipSuccess; ++j) {
    hipKernelNodeParams kp{};
    void *args_level[2];
    void *args_adv[2];
    int adv = kGraphLevels;
    if (j < kGraphLevels) {
      js[j] = j;
      args_level[0] = &ctl;
      args_level[1] = &js[j];
      kp.func = par ? (void *)&k_ms_level_g<true> : (void *)&k_ms_level_g<false>;
      kp.gridDim = dim3(blocks);
      kp.blockDim = dim3(kBlock);
      kp.kernelParams = args_level;
    } else {
      args_adv[0] = &ctl;
      args_adv[1] = &adv;
      kp.func = (void *)&k_ms_advance;
      kp.gridDim = dim3(1);
      kp.blockDim = dim3(64);
      kp.kernelParams = args_adv;
    }
    kp.sharedMemBytes = 0;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    set_error(std::string("g5_bfs_batch: graph: ") + hipGetErrorString(e));
    return G5_EDEVICE;
  }
  w.gexec[i] = exec;
  w.gblocks[i] = blocks;
  *out = exec;
  return G5_OK;
}

// Graph batch: the level loop as replays of one instantiated graph of
// kGraphLevels levels; the host reads the counters after each replay.
g5_status batch_graph(const g5_csr *g, BatchWork &w, const BatchSpace &ws, const MsArgs &a,
                      hipStream_t s, bool timed, g5_batch_stats *stats, int bpc) {
  const int blocks = g->num_cu * bpc;
  hipGraphExec_t exec = nullptr;
  {
    g5_status st = graph_exec(w, a.parents != nullptr, blocks, &exec);
    if (st != G5_OK) return st;
  }
  if (timed) G5_HIP(hipEventRecord(ws.ev[0], s));
  for (int l = kGraphLevels;; l += kGraphLevels) {
    G5_HIP(hipGraphLaunch(exec, s));
    g5_status st = read_ctl(ws, s);
    if (st != G5_OK) return st;
    if (ws.host_ctl->err || batch_done(ws.host_ctl, l)) break;
  }
  if (timed) {
    G5_HIP(hipEventRecord(ws.ev[1], s));
    G5_HIP(hipStreamSynchronize(s));
  }
  return batch_finish(ws, a, blocks, timed, stats);
}

// Every level in one cooperative launch.
g5_status batch_persistent(const g5_csr *g, const BatchSpace &ws, MsArgs a, hipStream_t s,
                           bool timed, g5_batch_stats *stats, int bpc) {
  const void *fn = a.parents ? reinterpret_cast<const void *>(&k_msbfs<true>)
                             : reinterpret_cast<const void *>(&k_msbfs<false>);
  int per_cu = 0;
  G5_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0));
  if (per_cu < 1) {
    set_error("g5_bfs_batch: the persistent kernel does not fit on a compute unit");
    return G5_EDEVICE;
  }
  const int blocks = g->num_cu * std::min(per_cu, bpc);
  void *args[] = {&a};
  if (timed) G5_HIP(hipEventRecord(ws.ev[0], s));
  G5_HIP(hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kBlock), args, 0, s));
  if (timed) G5_HIP(hipEventRecord(ws.ev[1], s));
  g5_status st = read_ctl(ws, s);
  if (st != G5_OK) return st;
  return batch_finish(ws, a, blocks, timed, stats);
}

}  // namespace

g5_status bfs_batch_impl(const g5_csr *g, const int64_t *roots, int k, int32_t *parents,
                         int8_t *levels, hipStream_t s, const g5_batch_params &p,
                         g5_batch_stats *stats) {
  BatchLease lease{g};
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->batch_pool.empty()) {
      lease.w = g->batch_pool.back();
      g->batch_pool.pop_back();
    }
  }
  if (!lease.w) {
    g5_status st = alloc_batch(g, &lease.w);
    if (st != G5_OK) return st;
  }
  BatchWork &w = *lease.w;
  const bool timed = stats && (p.flags & G5_FLAG_TIME_STEPS);
  if (timed && !w.ev[0]) {
    for (auto &e : w.ev) G5_HIP(hipEventCreate(&e));
  }
  const BatchSpace ws{w.seen, {w.buf[0], w.buf[1], w.buf[2]}, (MsCtl *)w.ctl,
                      (MsCtl *)w.host_ctl, {w.ev[0], w.ev[1]}};
  MsArgs a;
  {
    g5_status st = batch_start(g, ws, roots, k, parents, levels, s, p, a);
    if (st != G5_OK) return st;
  }
  const int bpc = p.blocks_per_cu > 0 ? p.blocks_per_cu : g->tune.batch_blocks_per_cu;
  if (p.flags & G5_FLAG_PERSISTENT) return batch_persistent(g, ws, a, s, timed, stats, bpc);
  if (p.flags & G5_FLAG_GRAPH) return batch_graph(g, w, ws, a, s, timed, stats, bpc);
  return batch_stepped(g, ws, a, s, timed, stats, bpc);
}

size_t batch_ctl_bytes() { return sizeof(MsCtl); }

g5_status batch_in_workspace(const g5_csr *g, uint64_t *masks, void *ctl, const int64_t *roots,
                             int k, int32_t *parents, int8_t *levels, hipStream_t s) {
  const int64_t n = g->n;
  MsCtl host{};  // the counters are read into this host buffer
  const BatchSpace ws{masks, {masks + n, masks + 2 * n, masks + 3 * n}, (MsCtl *)ctl, &host,
                      {nullptr, nullptr}};
  g5_batch_params p;
  std::memset(&p, 0, sizeof(p));
  MsArgs a;
  {
    g5_status st = batch_start(g, ws, roots, k, parents, levels, s, p, a);
    if (st != G5_OK) return st;
  }
  return batch_stepped(g, ws, a, s, false, nullptr, g->tune.batch_blocks_per_cu);
}

}  // namespace g5
