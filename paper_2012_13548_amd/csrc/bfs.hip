// Kernel 2 of the paper (Section 2.3): level-synchronous breadth-first search
// from one root, direction-optimising.
//
// Level synchronisation (Section 2.3.2): every level is a separate set of
// kernel launches, so a level's claims finish before the next level reads
// them; a vertex takes the level of the first level that reaches it.  The
// paper's parallel BFS processes a level in two phases (gather the level's
// neighbours, then update); the top-down step here does the same with one
// edge per lane after a prefix sum of frontier degrees.
//
//   top-down  (paper's parallel BFS): frontier queue Q whose entries carry
//             their first edge's index in Q's edge list -> every edge of Q gets
//             one lane (each block owns 1024 consecutive edges, so hubs are
//             split across blocks and small rows are packed together) -> claim
//             the neighbour with an atomic on the visited bitmap (or a
//             compare-and-swap on parent) -> compact winners into Q' by ballot
//             + LDS prefix; one 64-bit atomic per block adds (entries, degree
//             sum) to Q''s counter, which places the block's entries and their
//             edge indices at once, so Q' needs no separate prefix-sum pass.
//   bottom-up (Beamer, Asanovic, Patterson, SC'12): one lane per unvisited
//             vertex (a wavefront covers one 64-bit visited word); scan the
//             row until a neighbour in the frontier bitmap is found; the ballot
//             of finders is the next-frontier word, written without atomics.
//   switch    top-down -> bottom-up when m_f > m_u / alpha; back when
//             n_f < n / beta and the frontier shrinks.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>


#include "g5_internal.h"

namespace g5 {
namespace {

constexpr int kBlock = 256;
constexpr int kTdItems = 4;
constexpr int kTdTile = kBlock * kTdItems;    // edges per top-down block
// Expansion workgroups per compute unit by default: a wider window of tiles in
// flight (8, all that fit) made the large expansions of a scale-26 graph slower.
constexpr int kTdBlocksPerCu = 6;

// Device counters of one traversal (uint64 slots of BfsWork::ctr).  The last
// kernel of a level copies them, with a sequence number, to pinned host memory
// the host polls (publish), so a level costs one host wait and no copies.
enum Ctr : int {
  C_QLEN0 = 0,  // length of queue 0
  C_QLEN1 = 1,  // length of queue 1
  C_MF = 2,     // degree sum of the scanned frontier queue
  C_NNEW = 3,   // vertices found by a bottom-up step (reset after publishing)
  C_GO = 4,     // 1: the decided top-down level expands
  C_RDEG = 5,   // degree of the root
  C_ERR = 6,    // nonzero if a kernel met an impossible state
  C_SCAN = 7,   // row entries read by a bottom-up step (byte counting only)
  C_UNVIS = 8,  // unvisited non-isolated vertices it scanned (byte counting only)
  C_ROWS = 9,   // those that read their row offsets (hint missed; byte counting only)
  C_HINT = 10,  // vertices found by their hint (byte counting only)
  C_BUGO = 11,  // 1: the next level is bottom-up too (decided by the last bottom-up step)
  C_HEAVY = 12,  // 1: the decided top-down level is heavy (see TdRule)
  C_NPUB = 13,  // slots copied to the host
  C_MU = 13,    // m_u: edges of the vertices no top-down level has discovered yet
  C_LASTNF = 14,  // frontier size of the previous level
  C_NFIN = 15,  // input frontier size of the next bottom-up step
  C_UNV = 16,   // non-isolated vertices not reached yet
  C_QP0 = 17,   // queue 0: entries << 32 | degree sum (appended to by one atomic per block)
  C_QP1 = 18,   // queue 1: the same
  C_ENDL = 19,  // lvl + 1 when level lvl's queue came out empty (the traversal ended), else 0
  C_TICKET = 20,  // workgroups done in the kernel that fills a queue (the last one decides)
  C_NCTR = 21
};

// Every access to the counters is a device-scope atomic: they are written by
// one workgroup and read by the workgroups of the next kernel, which may run on
// another XCD whose L2 holds an older copy of the line.
__device__ __forceinline__ unsigned long long ctr_ld(const unsigned long long *ctr, int i) {
  return __hip_atomic_load(ctr + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ctr_st(unsigned long long *ctr, int i, unsigned long long v) {
  __hip_atomic_store(ctr + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Copies the counters to host memory.  Each 8-byte slot carries the low 16
// bits of the sequence number above a 48-bit value, so every slot is complete
// by itself and no release fence (a write-back of L2) is needed; the host waits
// until all slots show the sequence number.  All loads are issued before the
// first store so their latencies overlap.
constexpr int kPubShift = 48;
// kPubBufs host buffers of kPubSlots slots, by sequence number: with the next
// levels queued ahead, sequences k + 1 and k + 2 may be published before the
// host has read k.
constexpr int kPubSlots = 16;
constexpr int kPubBufs = 4;
__device__ void publish(const unsigned long long *ctr, unsigned long long *host,
                        unsigned long long seq) {
  unsigned long long v[C_NPUB];
#pragma unroll
  for (int i = 0; i < C_NPUB; ++i)
    v[i] = __hip_atomic_load(ctr + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long tag = (seq & 0xffffull) << kPubShift;
  unsigned long long *h = host + (seq % kPubBufs) * kPubSlots;
#pragma unroll
  for (int i = 0; i < C_NPUB; ++i)
    __hip_atomic_store(h + i, tag | (v[i] & ((1ull << kPubShift) - 1)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// Direction of a top-down level (the rule the host reads from the published
// counters): queue slot qs holds its frontier Q (qlen vertices, mf edges).
// m_u (edges of vertices no top-down level has discovered) drops by m_f except
// at the root's level; switch to bottom-up when Q grew and m_f > m_u / alpha.
// The decision is taken where the level's queue is complete (the root's at the
// start, otherwise by the last workgroup of the kernel that filled the queue),
// so an expansion queued ahead needs no kernel of its own for it: it runs when
// ctr[C_GO] = 1 (a level queued behind one that did not expand sees that
// level's 0).  Records Q for the host, marks an empty queue (the end) in
// C_ENDL, clears the counter of the queue this level fills and publishes.
struct TdRule {
  int dirmode;
  double alpha;
  double gamma;  // > 0: also switch when m_f > gamma * unvisited non-isolated vertices
  // > 0: a growing top-down level with m_f above this many edges is heavy: its
  // expansion skips the row-offset read of every vertex it claims (one random
  // line each) and writes no queue entries (only their count), and the next
  // level goes bottom-up, which uses neither (the conversion builds its
  // frontier from the byte levels).  Only before any bottom-up level, with
  // claims by OR over a pre-filled parent array.
  uint64_t heavy_edges;
};

__device__ void td_decide(unsigned long long *ctr, int qs, int32_t lvl, bool from_bu,
                          const TdRule &rule, int64_t qlen, uint64_t mf,
                          unsigned long long *host, unsigned long long seq,
                          bool after_heavy = false) {
  auto ld = [&](int i) {
    return (int64_t)__hip_atomic_load(ctr + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  int64_t mu = ld(C_MU);
  if (lvl > 0) mu -= (int64_t)mf;
  int64_t unv = ld(C_UNV);
  if (lvl > 0 && !from_bu) unv -= qlen;  // this frontier was found by a top-down level
  const bool growing = qlen > ld(C_LASTNF);
  // after a heavy level mf is unknown (0) and the level goes bottom-up
  const bool to_bu =
      rule.dirmode == G5_DIR_BOTTOMUP || after_heavy ||
      (rule.dirmode == G5_DIR_AUTO && growing &&
       ((double)mf > (double)mu / rule.alpha ||
        (rule.gamma > 0 && (double)mf > rule.gamma * (double)unv)));
  const bool go = qlen > 0 && !to_bu;
  ctr_st(ctr, C_HEAVY,
         (go && growing && rule.dirmode == G5_DIR_AUTO && rule.heavy_edges > 0 &&
          mf > rule.heavy_edges)
             ? 1ull
             : 0ull);
  ctr_st(ctr, C_MU, (unsigned long long)mu);
  ctr_st(ctr, C_UNV, (unsigned long long)unv);
  ctr_st(ctr, C_MF, mf);
  ctr_st(ctr, C_GO, go ? 1ull : 0ull);
  ctr_st(ctr, C_ENDL, qlen == 0 ? (unsigned long long)(lvl + 1) : 0ull);
  if (go) ctr_st(ctr, C_LASTNF, (unsigned long long)qlen);
  ctr_st(ctr, C_QLEN0 + qs, (unsigned long long)qlen);
  ctr_st(ctr, C_QP0 + (qs ^ 1), 0ull);
  publish(ctr, host, seq);
}

// Start of a traversal from `root`: byte levels = 0xff and parent = fill (the
// hint targets) or -1, except at the root (level 0, its own parent); visited
// bitmap = the isolated vertices and the root; counters zeroed, then queue 0 =
// {root} (edge index 0, its degree in the queue's counter), the direction
// state, and the root level's decision (published under seq).
__global__ void k_bfs_init(int64_t root, uint8_t *__restrict__ lev8,
                           int32_t *__restrict__ parent, int64_t n,
                           const int32_t *__restrict__ fill, uint64_t *__restrict__ vis,
                           const uint64_t *__restrict__ iso, int64_t words, bool vec,
                           int32_t *__restrict__ q0, uint32_t *__restrict__ qo0,
                           unsigned long long *__restrict__ ctr, const int64_t *__restrict__ rp,
                           int64_t nnz, int64_t nonisolated, TdRule rule,
                           unsigned long long *host, unsigned long long seq, bool fill_lev8) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t n4 = vec ? n / 4 : 0;
  typedef int v4i __attribute__((ext_vector_type(4)));
  const v4i m1 = {-1, -1, -1, -1};
  // streaming (non-temporal) accesses: the arrays are far larger than L2
  for (int64_t i = t; i < n4; i += stride) {
    v4i f = fill ? __builtin_nontemporal_load(reinterpret_cast<const v4i *>(fill) + i) : m1;
    if (i == (root >> 2)) f[root & 3] = (int32_t)root;
    __builtin_nontemporal_store(f, reinterpret_cast<v4i *>(parent) + i);
  }
  for (int64_t i = n4 * 4 + t; i < n; i += stride)
    parent[i] = i == root ? (int32_t)root : (fill ? fill[i] : -1);
  // A byte level is read only where the visited bitmap says the vertex was
  // reached in this traversal (stale bytes elsewhere are never used), so only
  // the root's byte is written; min-id claims test the bytes of vertices not
  // reached yet, and get 0xff everywhere (fill_lev8; lev8 is 16-byte aligned
  // and padded to a multiple of 16 bytes).
  if (fill_lev8) {
    for (int64_t i = t; i < (n + 15) / 16; i += stride) {
      v4i x = m1;
      if (i == (root >> 4)) reinterpret_cast<uint8_t *>(&x)[root & 15] = 0;
      __builtin_nontemporal_store(x, reinterpret_cast<v4i *>(lev8) + i);
    }
  } else if (t == 0) {
    lev8[root] = 0;
  }
  const int64_t rw = root >> 6;
  for (int64_t i = t; i < words; i += stride) {
    const uint64_t x = iso[i];
    vis[i] = i == rw ? x | (1ull << (root & 63)) : x;
  }
  if (t == 0) {
    for (int i = 0; i < C_NCTR; ++i) ctr_st(ctr, i, 0ull);
    const int64_t rdeg = rp[root + 1] - rp[root];  // 64-bit offsets
    q0[0] = (int32_t)root;
    qo0[0] = 0;
    ctr_st(ctr, C_QLEN0, 1ull);
    ctr_st(ctr, C_QP0, (1ull << 32) | (unsigned long long)rdeg);
    ctr_st(ctr, C_RDEG, (unsigned long long)rdeg);
    ctr_st(ctr, C_MU, (unsigned long long)(nnz - rdeg));
    ctr_st(ctr, C_UNV, (unsigned long long)(nonisolated - (rdeg > 0 ? 1 : 0)));
    td_decide(ctr, 0, 0, false, rule, 1, (uint64_t)rdeg, host, seq);
  }
}


// Levels are kept as bytes (lev8, valid where the vertex was reached) while they fit, so the
// scattered level writes of a traversal touch a quarter of the bytes; the
// int32 output is written once, by a streaming pass at the end (or, on a graph
// deeper than kByteLevels, before the first level that would not fit, after
// which kernels write int32 levels directly: lev8 == nullptr).
constexpr int32_t kByteLevels = 254;  // levels 0..254 fit a byte beside 0xff

__device__ __forceinline__ void put_level(uint8_t *lev8, int32_t *level, int32_t v,
                                          int32_t lvl) {
  if (lev8)
    lev8[v] = (uint8_t)lvl;
  else
    level[v] = lvl;
}

// Bit v: vertex v was reached in this traversal (visited and not isolated;
// the isolated bitmap also covers the padding past n), or is the root.
__device__ __forceinline__ uint64_t reached_word(const uint64_t *__restrict__ vis,
                                                 const uint64_t *__restrict__ iso, int64_t w,
                                                 int64_t root) {
  uint64_t m = vis[w] & ~iso[w];
  if ((root >> 6) == w) m |= 1ull << (root & 63);
  return m;
}

// level = lev8 widened where the vertex was reached, -1 elsewhere; 4 vertices
// per thread, grid-stride.
__device__ __forceinline__ void expand_levels(const uint8_t *__restrict__ lev8,
                                              int32_t *__restrict__ level, int64_t n, bool vec,
                                              int64_t stride, const uint64_t *__restrict__ vis,
                                              const uint64_t *__restrict__ iso, int64_t root) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n4 = vec ? n / 4 : 0;
  for (int64_t i = t; i < n4; i += stride) {
    const uint32_t x = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(lev8) + i);
    const int64_t v0 = 4 * i;
    const uint32_t r4 = (uint32_t)(reached_word(vis, iso, v0 >> 6, root) >> (v0 & 63)) & 0xfu;
    v4i o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = ((r4 >> j) & 1) ? (int)((x >> (8 * j)) & 0xffu) : -1;
    __builtin_nontemporal_store(o, reinterpret_cast<v4i *>(level) + i);
  }
  for (int64_t i = n4 * 4 + t; i < n; i += stride)
    level[i] = ((reached_word(vis, iso, i >> 6, root) >> (i & 63)) & 1) ? (int32_t)lev8[i] : -1;
}

// parent = -1 for the non-isolated vertices not visited (grid-stride over words).
__device__ __forceinline__ void unreached_words(const uint64_t *__restrict__ vis,
                                                const uint64_t *__restrict__ iso, int64_t words,
                                                int32_t *__restrict__ parent, int64_t stride) {
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    uint64_t m = ~(vis[w] | iso[w]);  // padding bits past n are set in iso
    while (m) {
      const int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      parent[w * kWave + b] = -1;
    }
  }
}

__global__ void k_zero_u64(uint64_t *__restrict__ p, int64_t len) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0;
}

// Edge index of frontier entry i in the frontier's edge list (non-decreasing
// in i; the total past the last entry).
struct FrontOffsets {
  const uint32_t *qoff;
  int64_t qlen;
  uint32_t total;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    return i >= qlen ? total : qoff[i];
  }
};

// Largest i in [0, len) with off(i) <= e (off non-decreasing, off(0) = 0 <= e):
// a 256-way search, one probe per thread per round.
template <class Off>
__device__ int64_t block_search(const Off &off, int64_t len, uint32_t e) {
  int64_t lo = 0, hi = len;
  while (true) {
    int64_t span = hi - lo;
    if (span <= kBlock) {
      int64_t p = lo + threadIdx.x;
      int c = __syncthreads_count(p < hi && off(p) <= e);
      return lo + c - 1;
    }
    int64_t p = lo + (span * (int64_t)threadIdx.x) / kBlock;
    int c = __syncthreads_count(off(p) <= e);
    int64_t nlo = lo + (span * (int64_t)(c - 1)) / kBlock;
    int64_t nhi = (c < kBlock) ? lo + (span * (int64_t)c) / kBlock : hi;
    lo = nlo;
    hi = nhi;
  }
}

// CLAIM_MIN: parent[v] is the smallest frontier neighbour (unsigned atomic
// min over every edge into a vertex unvisited at level start: its level is
// still unset or the one being written); the visited-bit OR still decides who
// appends v to the next queue.
enum Claim : int { CLAIM_OR = 0, CLAIM_CAS = 1, CLAIM_MIN = 2 };

// Top-down expansion (runs only if the level's decision set ctr[C_GO]); a
// block takes 1024-edge tiles of the frontier's edges (total ctr[C_MF]) in
// turn.  A tile's claimed vertices go to the next queue together: their
// degrees' block prefix sum, then one atomic on the queue's packed counter
// (entries << 32 | degree sum) gives the tile both its queue positions and
// its entries' edge indices.  The last block to finish (by a ticket) takes the
// next level's decision from that counter and publishes it under seq.  When
// the level's own decision found its queue empty (the traversal ended) the
// grid instead resets the parent of the unreached non-isolated vertices to -1
// if `fix` (the parent array was pre-filled with hint targets) and widens the
// byte levels into `level` when lev8 is given.

template <int CLAIM>
__global__ __launch_bounds__(kBlock) void k_td_expand(
    const int32_t *__restrict__ q, const uint32_t *__restrict__ qoff,
    unsigned long long *__restrict__ ctr, int cur,
    const uint32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    uint64_t *vis, int32_t *parent, int32_t *__restrict__ level, uint8_t *__restrict__ lev8,
    int32_t *__restrict__ qn, uint32_t *__restrict__ qon, int32_t next_level, TdRule rule,
    unsigned long long *__restrict__ host, unsigned long long seq,
    const uint64_t *__restrict__ iso, int64_t words, bool fix, int64_t n, bool vec,
    int64_t root) {
  __shared__ uint32_t s_off[kTdTile + 1];
  __shared__ int32_t s_src[kTdTile];
  __shared__ int64_t s_base[kTdTile];
  __shared__ unsigned long long s_scan[kBlock / kWave];
  __shared__ unsigned long long s_gbase;
  if (!ctr_ld(ctr, C_GO)) {
    if (ctr_ld(ctr, C_ENDL) == (unsigned long long)next_level) {
      const int64_t stride = (int64_t)gridDim.x * kBlock;
      if (fix) unreached_words(vis, iso, words, parent, stride);
      if (lev8) expand_levels(lev8, level, n, vec, stride, vis, iso, root);
    }
    return;
  }
  const int nxt = cur ^ 1;
  unsigned long long *qn_pack = ctr + C_QP0 + nxt;
  const int64_t qlen = (int64_t)ctr_ld(ctr, C_QLEN0 + cur);
  const uint32_t total = (uint32_t)ctr_ld(ctr, C_MF);
  // heavy: winners read no row offsets and get no queue entry (only counted)
  const bool heavy = ctr_ld(ctr, C_HEAVY) != 0;
  // only the blocks that own a tile take part (and take a ticket): same-address
  // atomics are serialised, so 1500 tickets cost ~20 us on a small level
  const uint64_t ntiles = ((uint64_t)total + kTdTile - 1) / kTdTile;
  const uint32_t active = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(gridDim.x, ntiles));
  if (blockIdx.x >= active) return;
  const FrontOffsets off{qoff, qlen, total};
  for (uint64_t tile = blockIdx.x; tile * kTdTile < total; tile += active) {
    const uint32_t e0 = (uint32_t)(tile * kTdTile);
    const uint32_t e1 = (uint32_t)std::min<uint64_t>((uint64_t)e0 + kTdTile, total);
    const int64_t i0 = block_search(off, qlen, e0);
    const int64_t i1 = block_search(off, qlen, e1 - 1);
    const int S = (int)(i1 - i0 + 1);
    if (S > kTdTile) {  // only degree-0 vertices could do this, and none are queued
      if (threadIdx.x == 0) atomicOr(ctr + C_ERR, 1ull);
      break;
    }
    for (int k = threadIdx.x; k < S; k += kBlock) {
      uint32_t o = off(i0 + k);
      int32_t u = q[i0 + k];
      s_off[k] = o;
      s_src[k] = u;
      s_base[k] = (int64_t)rp[u] - (int64_t)o;
    }
    if (threadIdx.x == 0) s_off[S] = off(i1 + 1);
    __syncthreads();
    int klo = 0;
    // this thread's winners; a winner's degree is loaded at once, so the loads
    // overlap the remaining edges
    int32_t wv[kTdItems];
    uint32_t wdeg[kTdItems];
    uint32_t wmask = 0;
#pragma unroll
    for (int j = 0; j < kTdItems; ++j) {
      uint32_t e = e0 + j * kBlock + threadIdx.x;
      bool won = false;
      int32_t v = 0;
      if (e < e1) {
        int lo = klo, hi = S;
        while (hi - lo > 1) {
          int mid = (lo + hi) >> 1;
          if (s_off[mid] <= e)
            lo = mid;
          else
            hi = mid;
        }
        klo = lo;
        v = ci[s_base[lo] + (int64_t)e];
        int32_t u = s_src[lo];
        uint64_t bit = 1ull << (v & 63);
        uint64_t *wp = vis + (v >> 6);
        if (CLAIM == CLAIM_MIN) {
          // (min-id mode fills the byte levels with 0xff at the start)
          const int32_t lv = lev8 ? (lev8[v] == 0xff ? -1 : (int32_t)lev8[v]) : level[v];
          if (lv < 0 || lv == next_level) {
            atomicMin((unsigned int *)(parent + v), (unsigned int)u);
            if (!(*wp & bit)) {
              won = !(atomicOr((unsigned long long *)wp, (unsigned long long)bit) & bit);
              if (won) put_level(lev8, level, v, next_level);
            }
          }
        } else if (!(*wp & bit)) {
          if (CLAIM == CLAIM_OR) {
            won = !(atomicOr((unsigned long long *)wp, (unsigned long long)bit) & bit);
            if (won) parent[v] = u;
          } else {
            won = atomicCAS(parent + v, -1, u) == -1;
            if (won) atomicOr((unsigned long long *)wp, (unsigned long long)bit);
          }
          if (won) put_level(lev8, level, v, next_level);
        }
      }
      wv[j] = v;
      wdeg[j] = 0;
      if (won) {
        wmask |= 1u << j;
        if (!heavy) {
          uint32_t be[2];
          __builtin_memcpy(be, rp + v, 8);
          wdeg[j] = be[1] - be[0];
        }
      }
    }
    // the tile's winners in thread order: one block scan of (count << 32 | degree
    // sum) and one atomic on the queue's counter give positions and edge indices
    unsigned long long mine = (unsigned long long)__popc(wmask) << 32;
#pragma unroll
    for (int j = 0; j < kTdItems; ++j) mine += wdeg[j];
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<kBlock, unsigned long long>(mine, s_scan, tot);
    const uint32_t cnt = (uint32_t)(tot >> 32);  // block-uniform
    if (cnt && heavy) {
      // the next level goes bottom-up and never reads this queue: only its
      // length.  The result is kept so the add has returned before this block's
      // ticket (the last block reads the counter after every ticket).
      if (threadIdx.x == 0) s_gbase = atomicAdd(qn_pack, tot);
    } else if (cnt) {
      // every thread has left the edge loop (the scan synchronised): stage the
      // entries at their tile positions in s_src (vertex) and s_off (edge
      // index from the tile's first), then write them out coalesced
      uint32_t p = (uint32_t)(ex >> 32), eo = (uint32_t)ex;
#pragma unroll
      for (int j = 0; j < kTdItems; ++j)
        if ((wmask >> j) & 1) {
          s_src[p] = wv[j];
          s_off[p] = eo;
          ++p;
          eo += wdeg[j];
        }
      if (threadIdx.x == 0) s_gbase = atomicAdd(qn_pack, tot);
      __syncthreads();
      const unsigned long long gb = s_gbase;
      const uint64_t pos = gb >> 32;
      for (uint32_t k = threadIdx.x; k < cnt; k += kBlock) {
        qn[pos + k] = s_src[k];
        qon[pos + k] = (uint32_t)gb + s_off[k];
      }
    }
    __syncthreads();  // the shared arrays are reused by the next tile
  }
  // No fences: a device-wide one writes back and invalidates this XCD's L2.
  // Thread 0 made the block's appends, each a returning device-scope atomic
  // waited for before the ticket is taken.  The last block reads the queue's
  // counter with a device-scope atomic (an add of 0, which the compiler emits
  // as a device-coherent load) issued after its own ticket returned, so it
  // sees every append.
  if (threadIdx.x == 0) {
    if (atomicAdd(ctr + C_TICKET, 1ull) + 1 == active) {
      const unsigned long long qp = atomicAdd(qn_pack, 0ull);
      atomicExch(ctr + C_TICKET, 0ull);
      td_decide(ctr, nxt, next_level, false, rule, (int64_t)(qp >> 32), qp & 0xffffffffull, host,
                seq, heavy);
    }
  }
}

// Frontier bitmap of level lvl (the vertices whose level is lvl), built
// without atomics from the byte levels: each thread reads 16 levels and four
// neighbouring lanes combine their 16-bit pieces into one 64-bit word.  With
// int32 levels (lev8 == nullptr, a graph deeper than the byte levels) one
// thread builds a word.  The same launch builds fh (bit r = frontier bit of
// hot[r], one wavefront per 64 hot targets), so the first bottom-up step needs
// no separate pass for it, and records the frontier size for the step.
__global__ __launch_bounds__(kBlock) void k_front_from_level(
    const uint8_t *__restrict__ lev8, const int32_t *__restrict__ level, int64_t n,
    int32_t lvl, uint64_t *__restrict__ front, int64_t words,
    unsigned long long *__restrict__ ctr, int64_t nf, const int32_t *__restrict__ hot,
    int64_t num_hot, uint64_t *__restrict__ fh, const uint64_t *__restrict__ vis,
    const uint64_t *__restrict__ iso, int64_t root) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr_st(ctr, C_NFIN, (unsigned long long)nf);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = __lane_id();
  // a byte level counts only where the vertex was reached in this traversal
  auto at = [&](int32_t v) -> bool {
    return lev8 ? lev8[v] == (uint8_t)lvl && ((reached_word(vis, iso, v >> 6, root) >> (v & 63)) & 1)
                : level[v] == lvl;
  };
  if (lev8) {
    // lev8 is padded to a multiple of 16 bytes; the padding past n is masked
    // like every vertex not reached
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const int64_t chunks = (n + 15) / 16;
    const uint32_t pat = 0x01010101u * (uint32_t)lvl;
    // the loop bound is rounded up to whole wavefronts so all lanes shuffle
    const int64_t span = ((words * 4 + kWave - 1) / kWave) * kWave;
    for (int64_t i = t; i < span; i += stride) {
      uint32_t bits = 0;
      if (i < chunks) {
        const v4u x = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(lev8) + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // byte k of y is zero exactly where byte k of x equals lvl
          const uint32_t y = x[j] ^ pat;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            bits |= (uint32_t)(((y >> (8 * k)) & 0xffu) == 0) << (4 * j + k);
        }
      }
      uint64_t wv = (uint64_t)bits << (16 * (lane & 3));
      wv |= __shfl_xor(wv, 1, kWave);
      wv |= __shfl_xor(wv, 2, kWave);
      if ((lane & 3) == 0 && (i >> 2) < words)
        front[i >> 2] = wv & reached_word(vis, iso, i >> 2, root);
    }
  } else {
    for (int64_t w = t; w < words; w += stride) {
      uint64_t m = 0;
      for (int b = 0; b < kWave; ++b) {
        const int64_t v = w * kWave + b;
        if (v < n && level[v] == lvl) m |= 1ull << b;
      }
      front[w] = m;
    }
  }
  for (int64_t i0 = t - lane; i0 < num_hot; i0 += stride) {
    const int64_t i = i0 + lane;
    const bool b = i < num_hot && at(hot[i]);
    const uint64_t m = __ballot(b);
    if (lane == 0) fh[i0 >> 6] = m;
  }
}

// Frontier membership for the bottom-up step: the frontier bitmap in HBM, or
// a summary staged in LDS (bit i set when some frontier vertex lies in
// [i << gs, (i + 1) << gs)); with gs = 0 the summary is the bitmap itself.
// pre(u): 0 = not in the frontier, 1 = in it, 2 = ask the bitmap's 32-bit word
// word(u).  Splitting the test lets a lane issue all of its bitmap loads
// before using any of them.
struct FrontGlobal {
  const uint32_t *front;  // the frontier bitmap as 32-bit words
  __device__ __forceinline__ int pre(int32_t) const { return 2; }
  __device__ __forceinline__ uint32_t word(int32_t u) const { return front[u >> 5]; }
  __device__ __forceinline__ bool test(int32_t u) const { return (word(u) >> (u & 31)) & 1; }
};

struct FrontLds {
  const uint32_t *sum;
  const uint32_t *front;
  int gs;
  __device__ __forceinline__ int pre(int32_t u) const {
    const uint32_t i = (uint32_t)u >> gs;
    if (!((sum[i >> 5] >> (i & 31)) & 1)) return 0;
    return gs == 0 ? 1 : 2;
  }
  __device__ __forceinline__ uint32_t word(int32_t u) const { return front[u >> 5]; }
  __device__ __forceinline__ bool test(int32_t u) const {
    const int p = pre(u);
    return p == 1 || (p == 2 && ((word(u) >> (u & 31)) & 1));
  }
};

// fh bit r = frontier bit of hot[r]; one wavefront per 64 targets.
__global__ __launch_bounds__(kBlock) void k_fh_build(const uint64_t *__restrict__ front,
                                                     const int32_t *__restrict__ hot,
                                                     int64_t num_hot, uint64_t *__restrict__ fh) {
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) - lane; i0 < num_hot;
       i0 += stride) {
    const int64_t i = i0 + lane;
    bool b = false;
    if (i < num_hot) {
      const int32_t t = hot[i];
      b = (front[t >> 6] >> (t & 63)) & 1;
    }
    const uint64_t m = __ballot(b);
    if (lane == 0) fh[i0 >> 6] = m;
  }
}

struct BuCount {
  uint64_t nnew = 0, nscan = 0, nunvis = 0, nrows = 0, nhint = 0;
};

// Rows a lane's own scan left unresolved are scanned by the whole wavefront,
// either packed end to end (one entry per lane per 64-entry window) or one row
// per 64-lane step.  With ACCT it counts the row entries read up to the first
// hit.
template <class Front, bool ACCT, int NW>
__device__ __forceinline__ void bu_row_rest(const Front &F, const int32_t *__restrict__ ci,
                                            bool packed, bool pending, int64_t k, int64_t e,
                                            bool &found, int32_t &par, uint32_t *s_base,
                                            int32_t *s_row, int32_t *s_first, BuCount &cnt) {
  const int lane = __lane_id();
  if (packed) {
    // Unresolved rows laid end to end, one entry per lane per 64-entry window,
    // NW windows per step whose entry loads and then frontier-word loads are
    // in flight together; a row's first hit in a step is its smallest hitting
    // position (LDS atomic min over window * 64 + lane); resolved rows stop
    // probing, and after a step that resolves rows the next step starts at the
    // next entry of a row still unresolved, so the entries resolved rows did
    // not need cost no windows (without the jump a wavefront whose other rows
    // resolve early steps over all their entries to reach its last unresolved
    // row: a bottom-up level on a small frontier of hubs took 7 ms instead of
    // 1.4).  A row resolved in one window of a step may read a few entries of
    // the next for nothing.
    constexpr int kNone = kWave * NW;
    const uint32_t len = (pending && !found) ? (uint32_t)(e - k) : 0u;
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t total = lane_u32(incl, kWave - 1);
    if (total) {
      const uint32_t pre = incl - len;
      // the wavefront's slice of the per-lane LDS arrays, in a scalar register
      const int wb = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) * kWave;
      // row entry j of the window sits at s_base + j: k - pre + j lies in
      // [0, nnz) < 2^32, so 32-bit wrap-around arithmetic gives it exactly
      s_base[wb + lane] = (uint32_t)k - pre;
      s_first[wb + lane] = kNone;
      // s_row[p] = tag << 6 | lane when that lane's row starts at position p
      // of the window with that tag (tags count windows from 1 in this call):
      // a lane reads its own slot and one ballot gives the window's row starts
      s_row[wb + lane] = 0;
      uint32_t tag = 0;
      uint64_t done = __ballot(len == 0);
      int carry = 0;
      for (uint32_t j0 = 0; j0 < total; j0 += kNone) {
        int32_t u[NW];
        int r[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t jw = j0 + (uint32_t)(w * kWave);
          ++tag;
          const bool starts = len > 0 && pre >= jw && pre < jw + kWave;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          if (starts) s_row[wb + (int)(pre - jw)] = (int32_t)((tag << 6) | (uint32_t)lane);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const uint64_t S = __ballot(((uint32_t)s_row[wb + lane] >> 6) == tag);
          const uint64_t upto = S & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1));
          r[w] = upto ? (s_row[wb + (kWave - 1 - __clzll((long long)upto))] & (kWave - 1)) : carry;
          carry = (int)lane_u32((uint32_t)r[w], kWave - 1);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const uint32_t j = jw + lane;
          u[w] = -1;
          if (j < total && !((done >> r[w]) & 1)) u[w] = ci[(uint32_t)(s_base[wb + r[w]] + j)];
        }
        int p[NW];
        uint32_t wd[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          p[w] = F.pre(u[w] < 0 ? 0 : u[w]);  // unconditional: no branch per entry
          if (u[w] < 0) p[w] = 0;
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) wd[w] = (p[w] == 2) ? F.word(u[w]) : 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const bool hit = p[w] == 1 || (p[w] == 2 && ((wd[w] >> (u[w] & 31)) & 1));
          if (hit) atomicMin(&s_first[wb + r[w]], w * kWave + lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int fl = s_first[wb + lane];
        const bool fresh = fl < kNone;
        int32_t gv = __shfl(u[0], fresh ? (fl & (kWave - 1)) : lane, kWave);
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          const int32_t g = __shfl(u[w], fresh ? (fl & (kWave - 1)) : lane, kWave);
          if (fl / kWave == w) gv = g;
        }
        if (fresh) {
          found = true;
          par = gv;
          s_first[wb + lane] = kNone;
          if (ACCT) cnt.nscan += (uint64_t)(j0 + fl - pre + 1);
        }
        const uint64_t fm = __ballot(fresh);
        done |= fm;
        if (done == ~0ull) break;
        if (fm) {
          // the next step starts where the next unresolved entry is: inside a
          // row that covers j0 + NW * 64 (no jump), or at the start of a later
          // row (a row start: its window needs no carry).  max(pre, nj) does
          // not decrease with the lane (pre is a prefix sum), so its minimum
          // over the live lanes is that of the lowest live lane.
          const uint32_t nj = j0 + kNone;
          const bool live = !((done >> lane) & 1) && pre + len > nj;
          const uint64_t lv = __ballot(live);
          j0 = (lv ? lane_u32(pre > nj ? pre : nj, __ffsll((unsigned long long)lv) - 1)
                   : 0xffffffffu) - kNone;
        }
      }
      if (ACCT && len > 0 && !found) cnt.nscan += len;
    }
    return;
  }
  uint64_t rem = __ballot(pending && !found && k < e);
  while (rem) {
    const int L = __ffsll((unsigned long long)rem) - 1;
    rem &= rem - 1;
    const int64_t kb = lane_i64(k, L), ke = lane_i64(e, L);
    int32_t got = -1;
    int64_t seen = ke - kb;
    for (int64_t c = kb; c < ke; c += kWave) {
      const int64_t kk = c + lane;
      bool hit = false;
      int32_t u = -1;
      if (kk < ke) {
        u = ci[kk];
        hit = F.test(u);
      }
      const uint64_t hm = __ballot(hit);
      if (hm) {
        const int hl = __ffsll((unsigned long long)hm) - 1;
        got = (int32_t)lane_u32((uint32_t)u, hl);
        seen = c - kb + hl + 1;
        break;
      }
    }
    if (lane == L) {
      if (got >= 0) {
        found = true;
        par = got;
      }
      if (ACCT) cnt.nscan += (uint64_t)seen;
    }
  }
}

// Position of the r-th set bit (from 0) of x; r < popcount(x).
__device__ __forceinline__ int select_bit(uint64_t x, uint32_t r) {
  int b = 0;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const uint32_t c = (uint32_t)__popcll(x & ((1ull << s) - 1));
    if (r >= c) {
      r -= c;
      x >>= s;
      b += s;
    }
  }
  return b;
}

// Bottom-up step (the bottom-up direction of Beamer, Asanovic and Patterson),
// vertex-parallel.  A wavefront owns chunks of 64 visited words (4096
// vertices): lane l loads word l of the chunk, a prefix sum of the unvisited
// counts numbers the chunk's unvisited vertices, and each 64-lane round hands
// the next 64 of them (R per lane with R rounds in flight) to the lanes, which
// find their vertex by a binary search over the prefix and a bit select.  Lanes
// thus work only on unvisited vertices, and a chunk whose vertices are all
// visited costs one coalesced load.
//
// Per vertex: the hint first (its highest-degree neighbour; a hot target is
// tested in fh, the frontier bits of the hot targets staged in LDS, any other
// one in the frontier), then LANE_SCAN row entries, then the wavefront-wide
// scan.  Finders write level (and parent, unless the parent array was
// pre-filled with every vertex's hint target, hint_id == nullptr, and the hint
// was the hit) and OR their bit into the chunk's next-frontier words in LDS,
// written out with the visited words at the end: no global atomics.
//
// COMPACT (one vertex per lane): rounds test hints only; the vertices whose hint
// missed and that have a row go to a ring of kRing entries per wavefront in LDS
// (s_ring), and whenever 64 are queued (and at the chunk's end) a round scans
// their rows with every lane busy.  On a dense frontier most hints hit, so
// without this nearly every round waited for the row reads of a few lanes.
constexpr uint32_t kRing = 128;

// Hints by rank (the one-vertex-per-lane step): stored for the vertices of
// degree >= 1 only, which an unvisited vertex of a bottom-up step always is,
// at their rank: the chunk's base from cbase plus the count of such vertices
// before it in the chunk, from the isolated bitmap's words (one coalesced load
// per lane and chunk).  Half the vertices of a scale-26 graph are isolated, so
// the hint lines the step reads hold twice as many useful entries.  The other
// steps (latency-bound on sparse frontiers) read hints by vertex.
template <bool RANK>
struct HintRank {
  const int32_t *hint;
  uint64_t base = 0;  // vertices of degree >= 1 before this chunk
  uint64_t ni = 0;    // this lane's word: bit set = degree >= 1
  uint32_t pre = 0;   // such vertices in the chunk's earlier words
  __device__ __forceinline__ HintRank(const int32_t *h, const uint64_t *cbase, const uint64_t *iso,
                                      int64_t c, int64_t w, int64_t words)
      : hint(h) {
    if (RANK && hint) {  // uniform: every lane takes part in the scan
      ni = w < words ? ~iso[w] : 0ull;
      const uint32_t q = (uint32_t)__popcll(ni);
      pre = wave_incl_scan<uint32_t>(q) - q;
      base = cbase[c];
    }
  }
  // hint of the vertex at bit `bit` of the chunk's word `pos` (-1 when inactive
  // or without hints); every lane calls it (the shuffles read other lanes)
  __device__ __forceinline__ int32_t at(bool act, int pos, int bit) const {
    const uint64_t x = __shfl(ni, pos, kWave);
    const uint32_t p = __shfl(pre, pos, kWave);
    if (!act || !hint) return -1;
    return hint[base + p + (uint32_t)__popcll(x & ((1ull << bit) - 1))];
  }
};

template <int LANE_SCAN, int R, bool ACCT, class Front, bool COMPACT = false, bool SPEC = false,
          int NW = 1>
__device__ __forceinline__ void bu_chunks(
    const Front &F, const uint64_t *fh, const uint32_t *__restrict__ rp,
    const int32_t *__restrict__ ci, const int32_t *__restrict__ hint,
    const int32_t *__restrict__ hint_id, const uint64_t *__restrict__ cbase,
    const uint64_t *__restrict__ iso, uint64_t *__restrict__ vis,
    uint64_t *__restrict__ next, int32_t *__restrict__ parent, int32_t *__restrict__ level,
    uint8_t *__restrict__ lev8, int64_t words, int32_t next_level, bool packed, int64_t gw,
    int64_t nw, uint32_t *s_base,
    int32_t *s_row, int32_t *s_first, unsigned long long *s_nx, BuCount &cnt,
    int32_t *s_ring = nullptr) {
  const int lane = __lane_id();
  unsigned long long *nx = s_nx + (threadIdx.x / kWave) * kWave;
  const int64_t chunks = (words + kWave - 1) / kWave;
  if constexpr (COMPACT) {
    static_assert(R == 1, "the compact form takes one vertex per lane");
    int32_t *ring = s_ring + (threadIdx.x / kWave) * kRing;
    const uint64_t lt = lanemask_lt();
    for (int64_t c = gw; c < chunks; c += nw) {
      const int64_t w = c * kWave + lane;
      const uint64_t vw = (w < words) ? vis[w] : ~0ull;  // padding past n is pre-set in iso
      const uint64_t un = ~vw;
      const uint32_t cl = (uint32_t)__popcll(un);
      const uint32_t incl = wave_incl_scan(cl);
      const uint32_t total = lane_u32(incl, kWave - 1);
      const uint32_t excl = incl - cl;
      nx[lane] = 0ull;
      HintRank<true> hr_(hint, cbase, iso, c, w, words);
      uint32_t head = 0, queued = 0;  // wavefront-uniform ring state
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // a round over `take` (<= 64) queued vertices, one per lane: row offsets,
      // the first LANE_SCAN entries, then the wavefront-wide scan
      auto rows = [&](uint32_t take) {
        const bool a = (uint32_t)lane < take;
        const int32_t vv = a ? ring[(head + (uint32_t)lane) & (kRing - 1)] : 0;
        head += take;
        queued -= take;
        uint32_t b = 0, e = 0;
        if (a) {
          uint32_t be[2];
          __builtin_memcpy(be, rp + vv, 8);
          b = be[0];
          e = be[1];
        }
        if (ACCT && a) cnt.nrows += 1;
        bool found = false;
        int32_t par = -1;
        int32_t u[LANE_SCAN];
        if (a && b < e) {
          __builtin_memcpy(u, ci + b, LANE_SCAN * sizeof(int32_t));
#pragma unroll
          for (int t = 0; t < LANE_SCAN; ++t)
            if (b + t >= e) u[t] = -1;
        } else {
#pragma unroll
          for (int t = 0; t < LANE_SCAN; ++t) u[t] = -1;
        }
        uint32_t sure = 0, need = 0;
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t) {
          const int p = F.pre(u[t] < 0 ? 0 : u[t]);
          if (u[t] >= 0) {
            sure |= (uint32_t)(p == 1) << t;
            need |= (uint32_t)(p == 2) << t;
          }
        }
        uint32_t uw[LANE_SCAN];
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t) uw[t] = ((need >> t) & 1) ? F.word(u[t]) : 0u;
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t) {
          const bool hv = ((sure >> t) & 1) || (((need >> t) & 1) && ((uw[t] >> (u[t] & 31)) & 1));
          if (a && !found && hv) {
            found = true;
            par = u[t];
            if (ACCT) cnt.nscan += (uint64_t)(t + 1);
          }
        }
        uint32_t k = b;
        if (a && !found) {
          k = std::min<uint32_t>(b + LANE_SCAN, e);
          if (ACCT) cnt.nscan += (uint64_t)(k - b);
        }
        bu_row_rest<Front, ACCT, NW>(F, ci, packed, a, (int64_t)k, (int64_t)e, found, par, s_base,
                                 s_row, s_first, cnt);
        if (found) {
          parent[vv] = par;
          put_level(lev8, level, vv, next_level);
          atomicOr(&nx[(vv >> 6) & (kWave - 1)], 1ull << (vv & 63));
        }
      };
      for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t idx = base + (uint32_t)lane;
        const bool act = idx < total;
        int pos = 0;  // last word whose exclusive prefix is <= idx
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
          if (__shfl(excl, pos + st, kWave) <= idx) pos += st;
        const uint32_t r = idx - __shfl(excl, pos, kWave);
        const uint64_t word = __shfl(un, pos, kWave);
        const int bit = act ? select_bit(word, r) : 0;
        const int32_t v = (int32_t)((c * kWave + pos) * kWave + bit);
        int32_t h = hr_.at(act, pos, bit);
        if (ACCT && act) cnt.nunvis += 1;
        int hp = 0;
        int32_t par = -1;
        const bool only = h != -1 && (h & kHintOnly);
        if (h >= 0) {
          h &= ~kHintOnly;
          hp = F.pre(h);
          par = h;
        } else if (h != -1) {
          const uint32_t hr = (uint32_t)h & (uint32_t)(kHintOnly - 1);
          hp = (int)((fh[hr >> 6] >> (hr & 63)) & 1);
        }
        const uint32_t hw = (hp == 2) ? F.word(h) : 0u;
        const bool via = hp == 1 || (hp == 2 && ((hw >> (h & 31)) & 1));
        if (via) {
          if (ACCT) cnt.nhint += 1;
          if (hint_id) parent[v] = par >= 0 ? par : hint_id[v];
          put_level(lev8, level, v, next_level);
          atomicOr(&nx[pos], 1ull << bit);
        }
        const bool miss = act && !via && !only;
        const uint64_t mb = __ballot(miss);
        if (miss) ring[(head + queued + (uint32_t)__popcll(mb & lt)) & (kRing - 1)] = v;
        queued += (uint32_t)__popcll(mb);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (queued >= (uint32_t)kWave) rows(kWave);
      }
      while (queued > 0) rows(std::min<uint32_t>(queued, kWave));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const uint64_t m = nx[lane];
      if (w < words) {
        next[w] = m;
        if (m) vis[w] = vw | m;
      }
      cnt.nnew += (uint64_t)__popcll(m);
    }
    return;
  }
  for (int64_t c = gw; c < chunks; c += nw) {
    const int64_t w = c * kWave + lane;
    const uint64_t vw = (w < words) ? vis[w] : ~0ull;  // padding lanes past n are pre-set in iso
    const uint64_t un = ~vw;
    const uint32_t cl = (uint32_t)__popcll(un);
    const uint32_t incl = wave_incl_scan(cl);
    const uint32_t total = lane_u32(incl, kWave - 1);
    const uint32_t excl = incl - cl;
    nx[lane] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t base = 0; base < total; base += kWave * R) {
      bool act[R], found[R], via[R];
      int32_t v[R], par[R], h[R];
      uint32_t b[R], e[R], k[R];  // row offsets (nnz < 2^32)
      int wl[R], bit[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t idx = base + (uint32_t)(j * kWave + lane);
        act[j] = idx < total;
        int pos = 0;  // last word whose exclusive prefix is <= idx
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
          if (__shfl(excl, pos + st, kWave) <= idx) pos += st;
        const uint32_t r = idx - __shfl(excl, pos, kWave);
        const uint64_t word = __shfl(un, pos, kWave);
        wl[j] = pos;
        bit[j] = act[j] ? select_bit(word, r) : 0;
        v[j] = (int32_t)((c * kWave + pos) * kWave + bit[j]);
        par[j] = -1;
        b[j] = e[j] = 0;
        h[j] = (act[j] && hint) ? hint[v[j]] : -1;
        if (SPEC && act[j]) {
          uint32_t be[2];
          __builtin_memcpy(be, rp + v[j], 8);  // both row offsets in one 8-byte load
          b[j] = be[0];
          e[j] = be[1];
        }
        if (ACCT && act[j]) cnt.nunvis += 1;
      }
      // The hint (highest-degree neighbour): a hot target's bit is in fh (LDS);
      // another target needs the frontier, whose word is loaded together with
      // the row offsets (taken unless the hint is already known to hit).
      // A vertex whose hint is its only neighbour has no row to read.  With
      // SPEC (sparse frontiers, where most hints miss) the row offsets come with
      // the hint and the first row entries with the hint's frontier word, one
      // dependent load fewer per vertex; a hint hit discards them.
      int hp[R];
      bool only[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        hp[j] = 0;
        only[j] = h[j] != -1 && (h[j] & kHintOnly);
        if (h[j] >= 0) {
          h[j] &= ~kHintOnly;
          hp[j] = F.pre(h[j]);
          par[j] = h[j];
        } else if (h[j] != -1) {
          const uint32_t r = (uint32_t)h[j] & (uint32_t)(kHintOnly - 1);
          hp[j] = (int)((fh[r >> 6] >> (r & 63)) & 1);
        }
      }
      uint32_t hw[R];
      // the first LANE_SCAN entries of the row in LANE_SCAN/4 16-byte loads (col_idx
      // is padded past nnz, so reading beyond the row's end stays in bounds)
      int32_t u[R][LANE_SCAN];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        hw[j] = (hp[j] == 2) ? F.word(h[j]) : 0u;
        if (!SPEC && act[j] && hp[j] != 1 && !only[j]) {
          uint32_t be[2];
          __builtin_memcpy(be, rp + v[j], 8);  // both row offsets in one 8-byte load
          b[j] = be[0];
          e[j] = be[1];
        }
        if (SPEC) {
          if (only[j] || hp[j] == 1) e[j] = b[j];  // no row to read
          if (act[j] && b[j] < e[j]) {
            __builtin_memcpy(u[j], ci + b[j], LANE_SCAN * sizeof(int32_t));
#pragma unroll
            for (int t = 0; t < LANE_SCAN; ++t)
              if (b[j] + t >= e[j]) u[j][t] = -1;
          } else {
#pragma unroll
            for (int t = 0; t < LANE_SCAN; ++t) u[j][t] = -1;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        via[j] = hp[j] == 1 || (hp[j] == 2 && ((hw[j] >> (h[j] & 31)) & 1));
        found[j] = via[j];
        if (found[j]) e[j] = b[j];   // nothing left to scan
        k[j] = b[j];
        if (ACCT && via[j]) cnt.nhint += 1;
        if (ACCT && act[j] && !found[j] && !only[j]) cnt.nrows += 1;
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (SPEC) {
          if (found[j]) {
#pragma unroll
            for (int t = 0; t < LANE_SCAN; ++t) u[j][t] = -1;
          }
        } else if (act[j] && !found[j] && k[j] < e[j]) {
          __builtin_memcpy(u[j], ci + k[j], LANE_SCAN * sizeof(int32_t));
#pragma unroll
          for (int t = 0; t < LANE_SCAN; ++t)
            if (k[j] + t >= e[j]) u[j][t] = -1;
        } else {
#pragma unroll
          for (int t = 0; t < LANE_SCAN; ++t) u[j][t] = -1;
        }
      }
      // their frontier tests: summary bits first (bit t of sure / need: entry t
      // is in the frontier / needs its bitmap word), then every needed word,
      // then the bits, so the loads are in flight together
      uint32_t sure[R], need[R];
      uint32_t uw[R][LANE_SCAN];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        sure[j] = need[j] = 0;
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t) {
          const int p = F.pre(u[j][t] < 0 ? 0 : u[j][t]);  // unconditional: no branch per entry
          if (u[j][t] >= 0) {
            sure[j] |= (uint32_t)(p == 1) << t;
            need[j] |= (uint32_t)(p == 2) << t;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t)
          uw[j][t] = ((need[j] >> t) & 1) ? F.word(u[j][t]) : 0u;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        bool hv[LANE_SCAN];
#pragma unroll
        for (int t = 0; t < LANE_SCAN; ++t)
          hv[t] = ((sure[j] >> t) & 1) || (((need[j] >> t) & 1) && ((uw[j][t] >> (u[j][t] & 31)) & 1));
        if (act[j] && !found[j]) {
#pragma unroll
          for (int t = 0; t < LANE_SCAN; ++t) {
            if (!found[j] && hv[t]) {
              found[j] = true;
              par[j] = u[j][t];
              if (ACCT) cnt.nscan += (uint64_t)(t + 1);
            }
          }
          const uint32_t k0 = k[j];
          k[j] = std::min<uint32_t>(k[j] + LANE_SCAN, e[j]);
          if (ACCT && !found[j]) cnt.nscan += (uint64_t)(k[j] - k0);
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        bu_row_rest<Front, ACCT, NW>(F, ci, packed, act[j], (int64_t)k[j], (int64_t)e[j], found[j],
                                 par[j], s_base, s_row, s_first, cnt);
        if (found[j]) {
          if (!via[j])
            parent[v[j]] = par[j];
          else if (hint_id)
            parent[v[j]] = par[j] >= 0 ? par[j] : hint_id[v[j]];
          put_level(lev8, level, v[j], next_level);
          atomicOr(&nx[wl[j]], 1ull << bit[j]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint64_t m = nx[lane];
    if (w < words) {
      next[w] = m;
      if (m) vis[w] = vw | m;
    }
    cnt.nnew += (uint64_t)__popcll(m);
  }
}

// Adds the workgroup's discoveries and takes a ticket in the same 64-bit
// atomic (count in the low 40 bits, finished workgroups above), so the last
// workgroup knows the total without a memory fence.  That workgroup takes the
// next level's direction decision (the rule the host applies to the published
// counters: back to top-down when n_f < n / beta and the frontier shrank;
// ctr[C_BUGO] = 1 lets an already queued next bottom-up step run), publishes
// the counters to the host and resets them for the next bottom-up step.  The
// accounting counters of COUNT_BYTES runs live at other addresses and are
// fenced.
constexpr int kTicketShift = 40;

struct BuNext {
  int dirmode;
  double beta;
  int64_t n;
};

template <int NT, bool ACCT>
__device__ __forceinline__ void bu_flush(const BuCount &c, uint64_t *s,
                                         unsigned long long *__restrict__ ctr,
                                         unsigned long long *__restrict__ host,
                                         unsigned long long seq, const BuNext &nx) {
  __shared__ unsigned long long s_old;
  const uint64_t tn = block_sum<NT, uint64_t>(c.nnew, s);
  uint64_t ts = 0, tu = 0, tr = 0, th = 0;
  if (ACCT) {
    ts = block_sum<NT, uint64_t>(c.nscan, s);
    tu = block_sum<NT, uint64_t>(c.nunvis, s);
    tr = block_sum<NT, uint64_t>(c.nrows, s);
    th = block_sum<NT, uint64_t>(c.nhint, s);
  }
  if (threadIdx.x == 0) {
    if (ACCT) {
      atomicAdd(ctr + C_SCAN, (unsigned long long)ts);
      atomicAdd(ctr + C_UNVIS, (unsigned long long)tu);
      atomicAdd(ctr + C_ROWS, (unsigned long long)tr);
      atomicAdd(ctr + C_HINT, (unsigned long long)th);
      __threadfence();
    }
    s_old = atomicAdd(ctr + C_NNEW, (1ull << kTicketShift) | (unsigned long long)tn);
  }
  __syncthreads();
  const unsigned long long old = s_old;
  if ((old >> kTicketShift) + 1 == gridDim.x && threadIdx.x == 0) {
    if (ACCT) __threadfence();
    // the counters without the ticket bits, as the host reads them
    const uint64_t nnew = (old & ((1ull << kTicketShift) - 1)) + tn;
    const uint64_t nf_in = ctr_ld(ctr, C_NFIN);
    const bool to_td = nx.dirmode == G5_DIR_TOPDOWN ||
                       (nx.dirmode == G5_DIR_AUTO && (double)nnew < (double)nx.n / nx.beta &&
                        nnew < nf_in);
    ctr_st(ctr, C_BUGO, (nnew > 0 && !to_td) ? 1ull : 0ull);
    ctr_st(ctr, C_NFIN, nnew);
    ctr_st(ctr, C_UNV, ctr_ld(ctr, C_UNV) - nnew);
    atomicExch(ctr + C_NNEW, nnew);
    publish(ctr, host, seq);
    atomicExch(ctr + C_NNEW, 0ull);
    ctr_st(ctr, C_QP0, 0ull);  // a switch back to top-down fills a queue from zero
    ctr_st(ctr, C_QP1, 0ull);
    if (ACCT) {
      atomicExch(ctr + C_SCAN, 0ull);
      atomicExch(ctr + C_UNVIS, 0ull);
      atomicExch(ctr + C_ROWS, 0ull);
      atomicExch(ctr + C_HINT, 0ull);
    }
  }
}

// Bottom-up step probing the frontier bitmap in HBM (L2/MALL-resident); the
// hot-target bits (fh_words words) are staged in dynamic LDS.
constexpr int kBuBlock = 512;

template <int LANE_SCAN, int R, bool ACCT>
__global__ __launch_bounds__(kBuBlock) void k_bu_step(
    const uint32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ hint, const int32_t *__restrict__ hint_id,
    const uint64_t *__restrict__ cbase, const uint64_t *__restrict__ iso,
    const uint64_t *__restrict__ fh, int64_t fh_words, uint64_t *__restrict__ vis,
    const uint64_t *__restrict__ front, uint64_t *__restrict__ next,
    int32_t *__restrict__ parent, int32_t *__restrict__ level, uint8_t *__restrict__ lev8,
    int64_t words, int32_t next_level, unsigned long long *__restrict__ ctr, bool packed,
    unsigned long long *__restrict__ host, unsigned long long seq, bool check_go, BuNext bn) {
  extern __shared__ uint64_t s_fh[];
  // queued ahead and the last step chose top-down: nothing to do
  if (check_go && !ctr_ld(ctr, C_BUGO)) return;
  __shared__ uint64_t s[kBuBlock / kWave];
  __shared__ uint32_t s_base[kBuBlock];
  __shared__ int32_t s_row[kBuBlock];
  __shared__ int32_t s_first[kBuBlock];
  __shared__ unsigned long long s_nx[kBuBlock];
  __shared__ int32_t s_ring[(R == 1) ? kBuBlock / kWave * kRing : 1];
  for (int64_t i = threadIdx.x; i < fh_words; i += kBuBlock) s_fh[i] = fh[i];
  __syncthreads();
  const int64_t gw = ((int64_t)blockIdx.x * kBuBlock + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * kBuBlock) / kWave;
  BuCount c;
  bu_chunks<LANE_SCAN, R, ACCT, FrontGlobal, R == 1>(
      FrontGlobal{(const uint32_t *)front}, s_fh, rp, ci, hint, hint_id, cbase, iso, vis, next,
      parent, level,
      lev8, words, next_level, packed, gw, nw, s_base, s_row, s_first, s_nx, c, s_ring);
  bu_flush<kBuBlock, ACCT>(c, s, ctr, host, seq, bn);
}

// Bottom-up step with the frontier summary staged in LDS as well (dynamic
// LDS: sum_words 32-bit summary words, padded to 8 bytes, then the fh_words
// hot-target words): probes of vertices whose summary bit is clear never leave
// the compute unit.
constexpr int kLdsBlock = 1024;
// 64-entry windows per step of its packed row scan
constexpr int kLdsWindows = 2;
// k_bu_step_lds's own LDS arrays (about 20 KiB), with margin
constexpr int64_t kBuStaticLds = 28 * 1024;

// At most 64 VGPRs (8 waves per SIMD, a few values spilled): with a staged
// frontier of up to ~55 KB (summary + fh) two workgroups share a compute unit,
// 32 waves instead of 16, which made the sparse-frontier steps of a scale-26
// graph ~27 % faster; with more LDS one workgroup fits and the spills only cost.
template <int LANE_SCAN, int R, bool ACCT>
__global__ __launch_bounds__(kLdsBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_bu_step_lds(
    const uint32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ hint, const int32_t *__restrict__ hint_id,
    const uint64_t *__restrict__ cbase, const uint64_t *__restrict__ iso,
    const uint64_t *__restrict__ fh, int64_t fh_words, uint64_t *__restrict__ vis,
    const uint64_t *__restrict__ front, uint64_t *__restrict__ next,
    int32_t *__restrict__ parent, int32_t *__restrict__ level, uint8_t *__restrict__ lev8,
    int64_t words, int32_t next_level, unsigned long long *__restrict__ ctr, bool packed,
    const uint32_t *__restrict__ sum, int64_t sum_words, int gs,
    unsigned long long *__restrict__ host, unsigned long long seq, BuNext bn) {
  extern __shared__ uint64_t s_dyn[];
  uint32_t *s_sum = reinterpret_cast<uint32_t *>(s_dyn);
  uint64_t *s_fh = s_dyn + (sum_words + 1) / 2;
  __shared__ uint64_t s[kLdsBlock / kWave];
  __shared__ uint32_t s_base[kLdsBlock];
  __shared__ int32_t s_row[kLdsBlock];
  __shared__ int32_t s_first[kLdsBlock];
  __shared__ unsigned long long s_nx[kLdsBlock];
  for (int64_t i = threadIdx.x; i < sum_words; i += kLdsBlock) s_sum[i] = sum[i];
  for (int64_t i = threadIdx.x; i < fh_words; i += kLdsBlock) s_fh[i] = fh[i];
  __syncthreads();
  const int64_t gw = ((int64_t)blockIdx.x * kLdsBlock + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * kLdsBlock) / kWave;
  BuCount c;
  // (compacting hint misses as k_bu_step does measured no faster here: on a
  // sparse frontier most hints miss, so its rounds are dense already)
  bu_chunks<LANE_SCAN, R, ACCT, FrontLds, false, true, kLdsWindows>(
      FrontLds{s_sum, (const uint32_t *)front, gs}, s_fh, rp, ci, hint, hint_id, cbase, iso, vis,
      next, parent,
      level, lev8, words, next_level, packed, gw, nw, s_base, s_row, s_first, s_nx, c);
  bu_flush<kLdsBlock, ACCT>(c, s, ctr, host, seq, bn);
}

// End of a traversal not finished by a top-down expansion: the unreached
// non-isolated vertices get parent -1 when the parent array was pre-filled with
// hint targets (fix), and the byte levels are widened into `level` when lev8 is
// given (also used alone before the first level deeper than kByteLevels).
__global__ void k_finish(const uint64_t *__restrict__ vis, const uint64_t *__restrict__ iso,
                         int64_t words, int32_t *__restrict__ fix,
                         const uint8_t *__restrict__ lev8, int32_t *__restrict__ level,
                         int64_t n, bool vec, int64_t root) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (fix) unreached_words(vis, iso, words, fix, stride);
  if (lev8) expand_levels(lev8, level, n, vec, stride, vis, iso, root);
}

// Frontier summary: bit i of sum = OR of front bits [i << gs, (i + 1) << gs).
// sum must be zeroed first.  One thread per frontier word.
__global__ void k_front_summary(const uint64_t *__restrict__ front, int64_t words, int gs,
                                uint32_t *__restrict__ sum) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    const uint64_t x = front[w];
    if (!x) continue;
    if (gs >= 6) {
      const uint64_t i = (uint64_t)w >> (gs - 6);
      atomicOr(sum + (i >> 5), 1u << (i & 31));
    } else {
      const int per = 64 >> gs;  // summary bits from this word
      const uint64_t gm = (gs == 0) ? 1ull : ((1ull << (1 << gs)) - 1);
      uint64_t m = 0;
      for (int j = 0; j < per; ++j)
        if ((x >> (j << gs)) & gm) m |= 1ull << j;
      const uint64_t base = (uint64_t)w * per;  // aligned to per (a power of two)
      if (per >= 32) {
        for (int h = 0; h < per / 32; ++h)
          if ((uint32_t)(m >> (32 * h))) atomicOr(sum + (base >> 5) + h, (uint32_t)(m >> (32 * h)));
      } else {
        atomicOr(sum + (base >> 5), (uint32_t)m << (base & 31));
      }
    }
  }
}

// Bitmap -> queue of the next top-down level, in rounds of kFqWords words per
// block (kFqPer consecutive words per thread).  A round's vertices are
// numbered by a block prefix sum of popcounts; when at most kFqCap of them
// (the usual case: the switch happens at fewer than n / beta vertices) they are
// staged in LDS in vertex order, their degrees loaded in parallel, and a block
// prefix sum of the degrees plus one atomic on the queue's packed counter
// (entries << 32 | degree sum, zero before) places them with their edge
// indices.  A denser round walks each thread's words serially instead.  The
// last block to finish (by a ticket) sets the direction state's previous
// frontier size and takes level lvl's decision (published under seq).
constexpr int kFqPer = 16;
constexpr int64_t kFqWords = (int64_t)kBlock * kFqPer;
constexpr uint32_t kFqCap = 2048;
constexpr int kFqItems = kFqCap / kBlock;  // staged vertices per thread at most

__global__ __launch_bounds__(kBlock) void k_front_queue(const uint64_t *__restrict__ bm,
                                                        int64_t words,
                                                        const uint32_t *__restrict__ rp,
                                                        int32_t *__restrict__ q,
                                                        uint32_t *__restrict__ qo,
                                                        unsigned long long *__restrict__ ctr,
                                                        int cur, int64_t last_nf, int32_t lvl,
                                                        TdRule rule,
                                                        unsigned long long *__restrict__ host,
                                                        unsigned long long seq) {
  __shared__ int32_t s_v[kFqCap];
  __shared__ uint32_t s32[kBlock / kWave];
  __shared__ unsigned long long s[kBlock / kWave];
  __shared__ unsigned long long s_g;
  for (int64_t r0 = (int64_t)blockIdx.x * kFqWords; r0 < words;
       r0 += (int64_t)gridDim.x * kFqWords) {
    const int64_t w0 = r0 + (int64_t)threadIdx.x * kFqPer;
    uint32_t cnt = 0;
    for (int j = 0; j < kFqPer; ++j)
      if (w0 + j < words) cnt += (uint32_t)__popcll(bm[w0 + j]);
    uint32_t total;
    const uint32_t first = block_excl_scan<kBlock, uint32_t>(cnt, s32, total);
    if (total == 0) continue;  // uniform: the block's sum
    if (total <= kFqCap) {
      uint32_t p = first;
      for (int j = 0; j < kFqPer && p < first + cnt; ++j) {
        uint64_t x = w0 + j < words ? bm[w0 + j] : 0ull;
        while (x) {
          s_v[p++] = (int32_t)((w0 + j) * kWave + __ffsll((unsigned long long)x) - 1);
          x &= x - 1;
        }
      }
      __syncthreads();
      // thread t: the staged entries [k0, k1), their degrees loaded together
      const uint32_t per = (total + kBlock - 1) / kBlock;
      const uint32_t k0 = std::min<uint32_t>(total, threadIdx.x * per);
      const uint32_t k1 = std::min<uint32_t>(total, k0 + per);
      uint32_t d[kFqItems];
      uint32_t sum = 0;
#pragma unroll
      for (int j = 0; j < kFqItems; ++j) {
        d[j] = 0;
        if (k0 + j < k1) {
          uint32_t be[2];
          __builtin_memcpy(be, rp + s_v[k0 + j], 8);
          d[j] = be[1] - be[0];
        }
      }
#pragma unroll
      for (int j = 0; j < kFqItems; ++j) sum += d[j];
      unsigned long long tot;
      const unsigned long long ex = block_excl_scan<kBlock, unsigned long long>(
          ((unsigned long long)(k1 - k0) << 32) | sum, s, tot);
      if (threadIdx.x == 0) s_g = atomicAdd(ctr + C_QP0 + cur, tot);
      __syncthreads();
      const unsigned long long g = s_g + ex;
      const uint64_t pos = g >> 32;
      uint32_t off = (uint32_t)g;
#pragma unroll
      for (int j = 0; j < kFqItems; ++j)
        if (k0 + j < k1) {
          q[pos + j] = s_v[k0 + j];
          qo[pos + j] = off;
          off += d[j];
        }
      __syncthreads();  // s_v and s_g are rewritten by the next round
      continue;
    }
    // dense round: each thread walks its own words
    unsigned long long mine = (unsigned long long)cnt << 32;  // count << 32 | degree sum
    for (int j = 0; j < kFqPer; ++j) {
      const int64_t w = w0 + j;
      uint64_t x = w < words ? bm[w] : 0ull;
      while (x) {
        const int32_t v = (int32_t)(w * kWave + __ffsll((unsigned long long)x) - 1);
        x &= x - 1;
        uint32_t be[2];
        __builtin_memcpy(be, rp + v, 8);
        mine += be[1] - be[0];
      }
    }
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<kBlock, unsigned long long>(mine, s, tot);
    if (threadIdx.x == 0) s_g = atomicAdd(ctr + C_QP0 + cur, tot);
    __syncthreads();
    const unsigned long long g = s_g + ex;
    uint64_t pos = g >> 32;
    uint32_t off = (uint32_t)g;
    __syncthreads();  // s_g is rewritten by the next round
    if (!cnt) continue;
    for (int j = 0; j < kFqPer; ++j) {
      const int64_t w = w0 + j;
      uint64_t x = w < words ? bm[w] : 0ull;
      while (x) {
        const int32_t v = (int32_t)(w * kWave + __ffsll((unsigned long long)x) - 1);
        x &= x - 1;
        uint32_t be[2];
        __builtin_memcpy(be, rp + v, 8);
        q[pos] = v;
        qo[pos++] = off;
        off += be[1] - be[0];
      }
    }
  }
  // no fences, for the reason given at the end of k_td_expand
  if (threadIdx.x == 0) {
    if (atomicAdd(ctr + C_TICKET, 1ull) + 1 == gridDim.x) {
      const unsigned long long qp = atomicAdd(ctr + C_QP0 + cur, 0ull);
      atomicExch(ctr + C_TICKET, 0ull);
      ctr_st(ctr, C_LASTNF, (unsigned long long)last_nf);
      td_decide(ctr, cur, lvl, true, rule, (int64_t)(qp >> 32), qp & 0xffffffffull, host, seq);
    }
  }
}

int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Workgroups of `fn` that fit on one compute unit (cached per kernel).
int resident_per_cu(const void *fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void *, size_t>, int>> done;
  std::lock_guard<std::mutex> lk(mu);
  for (auto &d : done)
    if (d.first.first == fn && d.first.second == lds) return d.second;
  int per_cu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  done.push_back({{fn, lds}, per_cu});
  return per_cu;
}

// Allows a kernel `bytes` of dynamic LDS (once per kernel and size).
g5_status lds_ready(const void *fn, int64_t bytes) {
  static std::mutex mu;
  static std::vector<std::pair<const void *, int64_t>> done;
  std::lock_guard<std::mutex> lk(mu);
  for (auto &d : done)
    if (d.first == fn && d.second >= bytes) return G5_OK;
  G5_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.emplace_back(fn, bytes);
  return G5_OK;
}

g5_status alloc_work(const g5_csr *g, BfsWork **out) {
  BfsWork *w = new BfsWork();
  w->n = g->n;
  w->words = g->words;
  int64_t n = g->n, W = g->words;
  hipError_t e = hipSuccess;
  auto A = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  A((void **)&w->vis, W * 8);
  A((void **)&w->lev8, ((n + 15) / 16) * 16);
  A((void **)&w->front, W * 8);
  A((void **)&w->next, W * 8);
  A((void **)&w->q[0], n * 4);
  A((void **)&w->q[1], n * 4);
  A((void **)&w->qoff[0], (n + 1) * 4);
  A((void **)&w->qoff[1], (n + 1) * 4);
  A((void **)&w->ctr, C_NCTR * 8);
  if (g->num_hot > 0) A((void **)&w->fh, ((g->num_hot + 63) / 64) * 8);
  // frontier summary for the LDS bottom-up step: as fine as the LDS allows
  const int64_t bits = (g->lds_bytes - kBuStaticLds - ((g->num_hot + 63) / 64) * 8) * 8;
  if (bits >= 1024) {
    int gs = 0;
    while (((n + (1ll << gs) - 1) >> gs) > bits) ++gs;
    w->sum_gs = gs;
    w->sum_words = (((n + (1ll << gs) - 1) >> gs) + 31) / 32;
    A((void **)&w->sum, ((w->sum_words + 1) / 2) * 8);
  }
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&w->host_pub, kPubBufs * kPubSlots * 8,
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(w->host_pub, 0, kPubBufs * kPubSlots * 8);
    e = hipHostGetDevicePointer((void **)&w->host_pub_dev, w->host_pub, 0);
  }
  if (e != hipSuccess) {
    set_error(std::string("g5_bfs workspace: ") + hipGetErrorString(e));
    delete w;
    return e == hipErrorOutOfMemory ? G5_ENOMEM : G5_EDEVICE;
  }
  *out = w;
  return G5_OK;
}

struct WorkLease {
  const g5_csr *g;
  BfsWork *w = nullptr;
  ~WorkLease() {
    if (w) {
      std::lock_guard<std::mutex> lk(g->mu);
      g->bfs_pool.push_back(w);
    }
  }
};

}  // namespace

BfsWork::~BfsWork() {
  if (vis) (void)hipFree(vis);
  if (lev8) (void)hipFree(lev8);
  if (front) (void)hipFree(front);
  if (next) (void)hipFree(next);
  if (sum) (void)hipFree(sum);
  if (fh) (void)hipFree(fh);
  if (q[0]) (void)hipFree(q[0]);
  if (q[1]) (void)hipFree(q[1]);
  for (auto *p : qoff)
    if (p) (void)hipFree(p);
  if (ctr) (void)hipFree(ctr);
  if (host_pub) (void)hipHostFree(host_pub);
  for (auto &e : ev) (void)hipEventDestroy(e);
}

// Waits until a kernel on `s` has published sequence number `want` to the
// mapped host counters and copies their values to out[0, C_NPUB); falls back to
// the stream's status so a failed launch cannot leave the host spinning.  The
// status is asked only after kQueryAfter of waiting (longer than any level
// takes): asking while the stream runs can queue a marker between kernels.
static g5_status wait_published(BfsWork &w, hipStream_t s, uint64_t want, int64_t *out) {
  volatile uint64_t *h = w.host_pub + (want % kPubBufs) * kPubSlots;
  const uint64_t tag = want & 0xffff;
  auto ready = [&]() {
    for (int i = 0; i < C_NPUB; ++i)
      if ((h[i] >> kPubShift) != tag) return false;
    return true;
  };
  using clk = std::chrono::steady_clock;
  constexpr auto kQueryAfter = std::chrono::milliseconds(2);
  constexpr auto kIdleGrace = std::chrono::milliseconds(100);
  auto next_query = clk::now() + kQueryAfter;
  for (uint32_t spin = 0;; ++spin) {
    if (ready()) break;
    if ((spin & 255) == 255 && clk::now() >= next_query) {
      next_query = clk::now() + kQueryAfter;
      hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        // The stream is idle.  The publishing stores are plain system-scope
        // stores to host memory, not ordered with the completion signal the
        // query reads, so they may still be in flight: give them a bounded
        // grace period before reporting a level that never published.
        const auto give_up = clk::now() + kIdleGrace;
        while (!ready() && clk::now() < give_up) {
        }
        if (ready()) break;
        set_error("g5_bfs: a level finished without publishing its counters");
        return G5_EDEVICE;
      }
      if (e != hipErrorNotReady) {
        set_error(std::string("g5_bfs: ") + hipGetErrorString(e));
        return G5_EDEVICE;
      }
    }
  }
  for (int i = 0; i < C_NPUB; ++i) out[i] = (int64_t)(h[i] & ((1ull << kPubShift) - 1));
  return G5_OK;
}

g5_status bfs_impl(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level,
                   hipStream_t s, const g5_bfs_params &p, g5_bfs_stats *stats) {
  WorkLease lease{g};
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->bfs_pool.empty()) {
      lease.w = g->bfs_pool.back();
      g->bfs_pool.pop_back();
    }
  }
  if (!lease.w) {
    g5_status st = alloc_work(g, &lease.w);
    if (st != G5_OK) return st;
  }
  BfsWork &w = *lease.w;
  const int64_t n = g->n, W = g->words;
  const int ncu = g->num_cu;
  const double alpha = p.alpha > 0 ? p.alpha : g->tune.alpha;
  const double beta = p.beta > 0 ? p.beta : g->tune.beta;
  const double gamma = p.gamma != 0 ? p.gamma : g->tune.gamma;  // < 0 disables
  const int lane_scan = p.bu_lane_scan > 0 ? p.bu_lane_scan : g->tune.lane_scan;
  const int bu_bpc = p.bu_blocks_per_cu > 0 ? p.bu_blocks_per_cu : g->tune.bu_blocks_per_cu;
  const double lds_density = p.lds_density > 0 ? p.lds_density : g->tune.lds_density;
  const int lds_kb = p.lds_kb > 0 ? p.lds_kb : g->tune.lds_kb;
  const int vpl = p.bu_vertices_per_lane > 0 ? p.bu_vertices_per_lane : g->tune.vertices_per_lane;
  const bool packed = (p.flags & G5_FLAG_PACKED) || (g->tune.packed && !(p.flags & G5_FLAG_ROWLOOP));
  const bool timed = stats && (p.flags & G5_FLAG_TIME_STEPS);
  const bool acct = stats && (p.flags & G5_FLAG_COUNT_BYTES);
  const bool min_parent = (p.flags & G5_FLAG_MIN_PARENT) != 0;
  const bool use_hint = !(p.flags & G5_FLAG_NO_HINT) && !min_parent;
  // staged frontier: summary granularity for this call's LDS budget
  int lds_gs = w.sum_gs;
  int64_t lds_words = w.sum_words;
  if (w.sum) {
    const int64_t fh_bytes = use_hint ? ((g->num_hot + 63) / 64) * 8 : 0;
    const int64_t bits =
        std::min<int64_t>((int64_t)lds_kb * 1024, g->lds_bytes - kBuStaticLds - fh_bytes) * 8;
    while (lds_gs < 40 && ((n + (1ll << lds_gs) - 1) >> lds_gs) > bits) ++lds_gs;
    lds_words = (((n + (1ll << lds_gs) - 1) >> lds_gs) + 31) / 32;
  }
  int lds_levels = 0;
  unsigned long long *ctr = (unsigned long long *)w.ctr;
  unsigned long long *hpub = (unsigned long long *)w.host_pub_dev;
  int64_t hc[C_NPUB] = {};  // the counters last published
  // Timed steps: every step launch is bracketed by two events of its own,
  // recorded on the stream before and after it, and a level's time is that of
  // its last step launch (a step queued ahead that its level did not use is
  // followed by the one it did).  No event is recorded twice in a call: an
  // event is bound to one launch at a time, never to two pending ones.  The
  // events are created as needed and kept with the workspace, whose calls end
  // with the stream synchronised.  (The markers between kernels slow a timed
  // traversal by ~6 %; the benchmark's timed steps carry none.)
  int ev_used = 0;
  int lv_ev[G5_MAX_STAT_LEVELS];
  for (int &x : lv_ev) x = -1;
  auto ev_take = [&](int lv) -> int {
    if (!timed || lv >= G5_MAX_STAT_LEVELS) return -1;
    if (2 * (size_t)ev_used + 2 > w.ev.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess) return -1;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1;
      }
      w.ev.push_back(a);
      w.ev.push_back(b);
    }
    lv_ev[lv] = ev_used;
    return ev_used++;
  };
#define G5_KLAUNCH(E, K, G, B, SH, S, ...)                    \
  do {                                                        \
    if ((E) >= 0) G5_HIP(hipEventRecord(w.ev[2 * (E)], S));   \
    hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);          \
    if ((E) >= 0) G5_HIP(hipEventRecord(w.ev[2 * (E) + 1], S)); \
  } while (0)

  // With hints and claims by OR, parent starts as every vertex's hint target:
  // a bottom-up hit on the hint then writes no parent (unreached vertices are
  // reset at the end).  Compare-and-swap claims need parent -1.
  const bool prefill = use_hint && p.claim != CLAIM_CAS;
  // heavy top-down levels need claims by OR over the pre-filled parents
  const uint64_t heavy_edges =
      (!prefill || min_parent || p.direction != G5_DIR_AUTO)
          ? 0
          : (p.heavy_kedges > 0 ? (uint64_t)p.heavy_kedges * 1000
                                : (p.heavy_kedges < 0 ? 0 : (uint64_t)g->nnz / 2048));
  const TdRule rule{p.direction, alpha, gamma, heavy_edges};
  const TdRule rule_light{p.direction, alpha, gamma, 0};
  bool bu_seen = false;  // a bottom-up level ran: no later level is heavy
  // the rule of the kernel that decides level L (heavy only before any
  // bottom-up level and while the byte levels hold L)
  auto rule_for = [&](int32_t L) -> TdRule {
    return (bu_seen || L >= kByteLevels) ? rule_light : rule;
  };
  const unsigned long long seq0 = ++w.seq;  // the root level's decision, taken by k_bfs_init
  hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(std::max(n / 4, W), kBlock, ncu * 16)),
                     dim3(kBlock), 0, s, root, w.lev8, parent, n,
                     prefill ? g->hint_id : nullptr, w.vis, g->iso, W,
                     ((uintptr_t)parent & 15) == 0, w.q[0], w.qoff[0], ctr, g->row_ptr, g->nnz,
                     g->nonisolated, rule, hpub, seq0, min_parent);
  G5_LAUNCH_CHECK();
  // Levels go to the byte array while they fit; the kernels of level lv (writing
  // lv + 1) get sink(lv), which widens the bytes into `level` once, before the
  // first level that does not fit, and returns nullptr from then on.
  const bool lvec = ((uintptr_t)level & 15) == 0;
  const int finish_grid = grid_for(std::max(n / 4, W), kBlock, ncu * 16);
  bool widened = false;
  auto sink = [&](int32_t lv) -> uint8_t * {
    if (lv + 1 <= kByteLevels) return w.lev8;
    if (!widened) {
      hipLaunchKernelGGL(k_finish, dim3(finish_grid), dim3(kBlock), 0, s, w.vis, g->iso, W,
                         nullptr, (const uint8_t *)w.lev8, level, n, lvec, root);
      widened = true;
    }
    return nullptr;
  };

  int cur = 0;                // queue holding the current frontier (top-down)
  bool q_from_bu = false;     // the queue was filled from a bottom-up bitmap
  bool ended_td = false;      // the traversal ended on an empty top-down queue
  int dir = 1;                // 1 top-down, 2 bottom-up
  int64_t nf_prev = 0;        // input frontier size of the bottom-up step
  int64_t last_nf = 0;        // frontier size of the previous level
  int32_t lvl = 0;
  int64_t reached = 1;
  bool bu_queued = false;     // this level's bottom-up step was queued ahead (sequence bu_seq)
  unsigned long long bu_seq = 0;
  uint64_t *front = w.front, *next = w.next;
  if (stats) *stats = g5_bfs_stats{};
  bool heavy_lv[G5_MAX_STAT_LEVELS] = {};  // heavy top-down levels (statistics)
  auto slot = [&]() -> int { return (stats && lvl < G5_MAX_STAT_LEVELS) ? lvl : -1; };
  const BuNext bn{p.direction, beta, n};
  const int32_t *hint = use_hint ? g->hint : nullptr;      // by vertex
  const int32_t *hint_r = use_hint ? g->hint_c : nullptr;  // by rank: the one-vertex-per-lane step
  const int32_t *hint_id = prefill ? nullptr : g->hint_id;
  const int64_t fh_words = use_hint ? (g->num_hot + 63) / 64 : 0;
  // expansion grid: the workgroups that fit at once, at most kTdBlocksPerCu per
  // compute unit (tiles then advance as one window over the frontier's edges),
  // unless set
  const int td_per_cu =
      p.td_blocks_per_cu > 0
          ? p.td_blocks_per_cu
          : std::min(kTdBlocksPerCu,
                     resident_per_cu(min_parent ? (const void *)&k_td_expand<CLAIM_MIN>
                                     : (p.claim == CLAIM_CAS ? (const void *)&k_td_expand<CLAIM_CAS>
                                                             : (const void *)&k_td_expand<CLAIM_OR>),
                                     kBlock, 0));
  const int td_grid = ncu * td_per_cu;

  // Top-down level lv from queue slot c: the expansion, which runs only if the
  // level's decision (already taken when the queue was completed) kept it top
  // down, and whose last workgroup takes level lv + 1's decision (published
  // under sq).  Queued ahead behind a level that did not expand, it does
  // nothing, or finishes the traversal when that level's queue was empty.
  auto launch_td = [&](int32_t lv, int c, unsigned long long sq) -> g5_status {
    const int nx = c ^ 1;
    uint8_t *l8 = sink(lv);
    const int te = ev_take(lv);
#define G5_TD(C)                                                                                 \
  G5_KLAUNCH(te, k_td_expand<C>, dim3(td_grid), dim3(kBlock), 0, s, w.q[c], w.qoff[c], ctr, c, \
             g->rp32, g->col_idx, w.vis, parent, level, l8, w.q[nx], w.qoff[nx], lv + 1,          \
             rule_for(lv + 1), hpub, sq, (const uint64_t *)g->iso, W, prefill, n, lvec, root)
    if (min_parent)
      G5_TD(CLAIM_MIN);
    else if (p.claim == CLAIM_CAS)
      G5_TD(CLAIM_CAS);
    else
      G5_TD(CLAIM_OR);
#undef G5_TD
    G5_LAUNCH_CHECK();
    return G5_OK;
  };

  // fh_ready: fh already holds the frontier bits of the hot targets
  auto launch_bu = [&](int32_t lv, const uint64_t *f, uint64_t *nfp, bool lds, bool check,
                       unsigned long long sq, bool fh_ready) -> g5_status {
    uint8_t *l8 = sink(lv);
    if (lds) {
      hipLaunchKernelGGL(k_zero_u64, dim3(grid_for((lds_words + 1) / 2, kBlock, ncu * 16)),
                         dim3(kBlock), 0, s, (uint64_t *)w.sum, (lds_words + 1) / 2);
      hipLaunchKernelGGL(k_front_summary, dim3(grid_for(W, kBlock, ncu * 16)), dim3(kBlock), 0,
                         s, f, W, lds_gs, w.sum);
    }
    if (fh_words && !fh_ready)
      hipLaunchKernelGGL(k_fh_build, dim3(grid_for(g->num_hot, kBlock, ncu * 8)), dim3(kBlock),
                         0, s, f, g->hot, g->num_hot, w.fh);
    const int te = ev_take(lv);
#define G5_BUL(K, P, A)                                                                     \
  do {                                                                                      \
    const void *fn_ = (const void *)&k_bu_step_lds<K, P, A>;                                 \
    const size_t dyn_ = (size_t)((lds_words + 1) / 2 + fh_words) * 8;                        \
    g5_status st_ = lds_ready(fn_, (int64_t)dyn_);                                          \
    if (st_ != G5_OK) return st_;                                                           \
    const int per_cu_ = resident_per_cu(fn_, kLdsBlock, dyn_);                              \
    G5_KLAUNCH(te, (k_bu_step_lds<K, P, A>), dim3(ncu * per_cu_), dim3(kLdsBlock), dyn_, s, \
               g->rp32, g->col_idx, hint, hint_id, g->chunk_ni, g->iso, w.fh, fh_words, w.vis, f,  \
               nfp, parent, level,                                                          \
               l8, W, lv + 1, ctr, packed, w.sum, lds_words, lds_gs, hpub, sq, bn);          \
  } while (0)
#define G5_BU(K, P, A)                                                                      \
  do {                                                                                      \
    const void *fn_ = (const void *)&k_bu_step<K, P, A>;                                     \
    const size_t dyn_ = (size_t)fh_words * 8;                                               \
    g5_status st_ = lds_ready(fn_, (int64_t)dyn_);                                          \
    if (st_ != G5_OK) return st_;                                                           \
    const int per_cu_ = resident_per_cu(fn_, kBuBlock, dyn_);                               \
    G5_KLAUNCH(te, (k_bu_step<K, P, A>), dim3(ncu * std::min(bu_bpc, per_cu_)),         \
               dim3(kBuBlock), dyn_, s, g->rp32, g->col_idx, (P) == 1 ? hint_r : hint, hint_id, \
               g->chunk_ni, g->iso, w.fh, fh_words,                                         \
               w.vis, f, nfp, parent, level, l8, W, lv + 1, ctr, packed, hpub, sq, check, bn); \
  } while (0)
#define G5_BU_P(M, K, A)          \
  if (vpl == 2)                   \
    M(K, 2, A);                   \
  else                            \
    M(K, 1, A);
#define G5_BU_K(M, A)                   \
  switch (lane_scan) {                  \
    case 1: G5_BU_P(M, 1, A); break;    \
    case 2: G5_BU_P(M, 2, A); break;    \
    case 8: G5_BU_P(M, 8, A); break;    \
    case 16: G5_BU_P(M, 16, A); break;  \
    default: G5_BU_P(M, 4, A); break;   \
  }
    if (lds) {  // never queued ahead
      // at most 4 entries per lane: at 8 waves per SIMD the spills grow with the
      // scan width (32 bytes per lane at 4, 72 at 8), and 4 measured ~1 % faster;
      // but 8 by default on a frontier below 1/16 of the summary bits, whose rows
      // run longer before a hit (scale 26: 6-7 % faster on 5-6 K-vertex hub
      // frontiers, 1-2 % slower on 16-21 K ones)
      const bool wide = p.bu_lane_scan <= 0 &&
                        (double)nf_prev * (double)(1ll << std::min(lds_gs, 40)) * 16.0 < (double)n;
      if (wide) {
        if (acct) {
          G5_BU_P(G5_BUL, 8, true);
        } else {
          G5_BU_P(G5_BUL, 8, false);
        }
      } else if (acct) {
        if (lane_scan >= 8) {
          G5_BU_P(G5_BUL, 4, true);
        } else {
          G5_BU_K(G5_BUL, true);
        }
      } else {
        if (lane_scan >= 8) {
          G5_BU_P(G5_BUL, 4, false);
        } else {
          G5_BU_K(G5_BUL, false);
        }
      }
    } else {
      if (acct) {
        G5_BU_K(G5_BU, true);
      } else {
        G5_BU_K(G5_BU, false);
      }
    }
#undef G5_BU_K
#undef G5_BU_P
#undef G5_BU
#undef G5_BUL
    G5_LAUNCH_CHECK();
    return G5_OK;
  };

  // Top-down levels are queued kTdAhead levels beyond the one whose decision
  // the host waits for; td_seq[L % 4] is the publication sequence of level L's
  // decision, taken by level L - 1's expansion.  A level queued behind one that
  // did not expand does nothing.  Queueing two levels ahead measured slower at
  // scale 26: the device rarely waited for the host, and every switch or end
  // ran one more empty level.  (At most kTdAhead + 2 publications are unread,
  // no more than kPubBufs.)
  constexpr int kTdAhead = 1;
  static_assert(kTdAhead + 2 <= kPubBufs, "unread decisions would share a buffer");
  unsigned long long td_seq[4] = {0, 0, 0, 0};
  int32_t td_queued = 0;  // highest top-down level queued
  td_seq[0] = seq0;
  td_seq[1] = ++w.seq;
  {
    g5_status st = launch_td(0, 0, td_seq[1]);
    if (st != G5_OK) return st;
  }
  while (true) {
    if (dir == 1) {
      // level lvl's kernels are queued; queue the next levels behind them, then
      // read level lvl's decision
      const int nxt = cur ^ 1;
      while (td_queued < lvl + kTdAhead) {
        ++td_queued;
        const unsigned long long sq = ++w.seq;
        td_seq[(td_queued + 1) & 3] = sq;
        g5_status st = launch_td(td_queued, cur ^ ((td_queued - lvl) & 1), sq);
        if (st != G5_OK) return st;
      }
      {
        g5_status st = wait_published(w, s, td_seq[lvl & 3], hc);
        if (st != G5_OK) return st;
      }
      if (hc[C_ERR]) {
        set_error(hc[C_ERR] & 1 ? "g5_bfs: top-down tile met more frontier rows than edges"
                                : "g5_bfs: a vertex found by a heavy level has no neighbour "
                                  "one level up");
        return G5_EDEVICE;
      }
      const int64_t qlen = hc[C_QLEN0 + cur];
      const int64_t mf = hc[C_MF];
      if (lvl > 0 && !q_from_bu) {  // the previous top-down level's discoveries
        reached += qlen;
        if (lvl - 1 < G5_MAX_STAT_LEVELS && stats) stats->discovered[lvl - 1] = qlen;
      }
      if (qlen == 0) {  // the traversal ended
        ended_td = true;  // this level's queued expansion finishes it
        break;
      }
      q_from_bu = false;
      if (!hc[C_GO]) {
        // bottom-up from here: frontier bitmap = the vertices of level lvl
        // (in `level` once the byte levels were widened)
        hipLaunchKernelGGL(k_front_from_level, dim3(grid_for(4 * W, kBlock, ncu * 16)),
                           dim3(kBlock), 0, s, widened ? nullptr : (const uint8_t *)w.lev8,
                           (const int32_t *)level, n, lvl, front, W, ctr, qlen, g->hot,
                           fh_words ? g->num_hot : (int64_t)0, w.fh, (const uint64_t *)w.vis,
                           (const uint64_t *)g->iso, root);
        G5_LAUNCH_CHECK();
        dir = 2;
        bu_seen = true;
        nf_prev = qlen;
        continue;  // this level runs bottom-up
      }
      if (slot() >= 0) {
        const int i = slot();
        stats->dir[i] = 1;
        stats->frontier[i] = qlen;
        stats->edges[i] = mf;
        heavy_lv[i] = hc[C_HEAVY] != 0;  // the device's flag for this level
        if (heavy_lv[i] && i < 64) stats->heavy_mask |= (int64_t)(1ull << i);
      }
      cur = nxt;
      last_nf = qlen;
      ++lvl;
    } else {
      if (!bu_queued) {
        const bool use_lds = w.sum && !(p.flags & G5_FLAG_NO_LDS) &&
                             (double)nf_prev * (double)(1ll << std::min(lds_gs, 62)) <
                                 lds_density * (double)n;
        if (use_lds) {
          ++lds_levels;
          if (stats && lvl < 64) stats->lds_mask |= (int64_t)(1ull << lvl);
        }
        bu_seq = ++w.seq;
        // the first step after top-down: k_front_from_level built fh
        g5_status st = launch_bu(lvl, front, next, use_lds, false, bu_seq, true);
        if (st != G5_OK) return st;
      }
      // queue the next level's step too; it runs only if this one chooses
      // bottom-up again
      const unsigned long long spec_seq = ++w.seq;
      {
        g5_status st = launch_bu(lvl + 1, next, front, false, true, spec_seq, false);
        if (st != G5_OK) return st;
      }
      {
        g5_status st = wait_published(w, s, bu_seq, hc);
        if (st != G5_OK) return st;
      }
      if (hc[C_ERR]) {
        set_error("g5_bfs: a vertex found by a heavy level has no neighbour one level up");
        return G5_EDEVICE;
      }
      const int64_t nnew = hc[C_NNEW];
      if (slot() >= 0) {
        const int i = slot();
        stats->dir[i] = 2;
        stats->frontier[i] = nf_prev;
        stats->discovered[i] = nnew;
        if (acct) {
          stats->edges[i] = hc[C_SCAN];
          // parent is not written for hint hits when it was pre-filled; a level
          // is one byte while levels fit the byte array
          const int64_t pw = prefill ? nnew - hc[C_HINT] : nnew;
          const int64_t lb = i + 1 <= kByteLevels ? 1 : 4;
          stats->bytes[i] = (use_hint ? 4 : 0) * hc[C_UNVIS] + 4 * hc[C_ROWS] +
                            4 * hc[C_SCAN] + 16 * W + lb * nnew + 4 * pw;
        }
      }
      reached += nnew;
      last_nf = nf_prev;
      ++lvl;
      if (nnew == 0) break;  // the queued step does nothing
      nf_prev = nnew;
      std::swap(front, next);  // `front` now holds the new frontier
      if (hc[C_BUGO]) {        // the queued step is this level's
        bu_queued = true;
        bu_seq = spec_seq;
        continue;
      }
      // top-down from here: bitmap -> queue (with edge indices) and the level's
      // decision, then its expansion
      bu_queued = false;
      td_seq[lvl & 3] = ++w.seq;
      hipLaunchKernelGGL(k_front_queue, dim3(grid_for(W, (int)kFqWords, ncu)), dim3(kBlock), 0, s,
                         (const uint64_t *)front, W, g->rp32, w.q[cur], w.qoff[cur], ctr, cur,
                         last_nf, lvl, rule_for(lvl), hpub, td_seq[lvl & 3]);
      G5_LAUNCH_CHECK();
      td_queued = lvl;  // top-down levels queued before the bottom-up steps did nothing
      td_seq[(lvl + 1) & 3] = ++w.seq;
      {
        g5_status st = launch_td(lvl, cur, td_seq[(lvl + 1) & 3]);
        if (st != G5_OK) return st;
      }
      q_from_bu = true;
      dir = 1;
    }
  }
#undef G5_KLAUNCH
  // a traversal ended by an empty top-down queue was finished by that level's
  // queued expansion
  if (!ended_td && (prefill || !widened))
    hipLaunchKernelGGL(k_finish, dim3(finish_grid), dim3(kBlock), 0, s, w.vis, g->iso, W,
                       prefill ? parent : nullptr, widened ? nullptr : (const uint8_t *)w.lev8,
                       level, n, lvec, root);
  G5_LAUNCH_CHECK();
  G5_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->nlevels = lvl;
    stats->reached = reached;
    stats->alpha = alpha;
    stats->beta = beta;
    stats->bu_lane_scan = lane_scan;
    stats->bu_blocks_per_cu = bu_bpc;
    stats->lds_levels = lds_levels;
    stats->lds_shift = lds_gs;
    if (acct)
      for (int i = 0; i < std::min<int>(lvl, G5_MAX_STAT_LEVELS); ++i)
        if (stats->dir[i] == 1)
          stats->bytes[i] = 12 * stats->frontier[i] + 4 * stats->edges[i] +
                            ((i + 1 <= kByteLevels ? 21 : 24) - (heavy_lv[i] ? 16 : 0)) *
                                stats->discovered[i];
    if (timed)
      for (int i = 0; i < std::min<int>(lvl, G5_MAX_STAT_LEVELS); ++i) {
        float a = 0;
        if (lv_ev[i] >= 0)
          G5_HIP(hipEventElapsedTime(&a, w.ev[2 * lv_ev[i]], w.ev[2 * lv_ev[i] + 1]));
        stats->step_ms[i] = a;
      }
  }
  return G5_OK;
}

}  // namespace g5
