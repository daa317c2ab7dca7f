// Kernel 1 of the paper (Section 2.2, CSR format; parallel CSR by a parallel
// sort is the direction named in Section 4.2): build the undirected CSR of a
// tuple list on the device.
//
//   pack      each non-loop tuple (u, v) -> keys (u << sb | v) and (v << sb | u);
//             self-loops and out-of-range ids -> SENT (sorts last)
//   sort      LSD radix sort of the 2*sb-bit keys, 8-bit digits: the digit
//             histograms of every pass are counted while packing, then each
//             pass is one sweep whose tiles rank their keys (wavefront match,
//             8 ballots per digit, and LDS counters) and find where their digit
//             runs go from the counts published by the tiles before them
//   compact   keep the first of each run of equal keys -> col_idx; the source of
//             each kept key opens rows (prev_source, source] -> row_ptr, so an
//             empty row repeats the next index; rows after the last key get nnz
//   iso       bitmap of degree-0 vertices (used by the traversal to skip them)
//   hubs      list of rows longer than kHubDeg and their kHubChunk-edge pieces
//             (the batched traversal splits these rows across wavefronts)
//   rp32      32-bit copy of row_ptr for the traversal (nnz < 2^32 is required)
//   hint      for each vertex, its highest-degree neighbour (over its whole
//             row; smallest id on ties): the bottom-up step
//             tests it before reading the row (hint_id keeps the ids); bit 30
//             marks a target that is the vertex's only neighbour (no row to read)
//   hot       the hint targets named by the most vertices (at most kHotMax of
//             them and at most n/16, in vertex order) get a compact index; a vertex whose hint is
//             one of them stores INT32_MIN | index instead of the id, so the
//             bottom-up step tests a per-level bitmap of kHotMax bits (small
//             enough to stay in L2) instead of a random word of the frontier
#include <algorithm>
#include <functional>
#include <vector>

#include "g5_internal.h"

namespace g5 {
namespace {

// A scatter tile of 7,168 keys puts ~28 keys (224 bytes) of each digit side
// by side, so its runs cover whole lines; two such workgroups fit a compute
// unit (measured at 2^31 random 52-bit keys, per pass: 2,048-key tiles
// 14.6 ms, 4,096 12.6 ms, 7,168 11.1 ms).
constexpr int kSortBlock = 256;
constexpr int kSortItems = 28;
constexpr int kSortTile = kSortBlock * kSortItems;  // 7,168 keys
constexpr int kWaveKeys = kWave * kSortItems;       // 1,792 keys per wavefront
constexpr int kRadix = 256;
constexpr int kScanBlock = 1024;
constexpr int kCompactBlock = 256;
// 2,048-key compaction tiles: 16 KB of LDS staging per workgroup leaves room
// for eight wavefronts per SIMD (4,096-key tiles: four; 8.9 -> 5.8 ms at scale 26)
constexpr int kCompactItems = 8;
constexpr int kCompactTile = kCompactBlock * kCompactItems;  // 2048 keys

// With weights (wb = 8) a key is (u << (sb + 8) | v << 8 | w): the sort then
// orders each run of one (u, v) by weight, and the compaction keeps its first
// key, i.e. the smallest weight of repeated tuples.  Without weights wb = 0.
// Each block also counts the digits of its keys for every sort pass:
// bh[block][pass][digit].
constexpr int kMaxPasses = 8;
__global__ __launch_bounds__(256) void k_pack(const int64_t *__restrict__ edges,
                                              const uint8_t *__restrict__ wts, int64_t m,
                                              int64_t n, int sb, int wb, uint64_t sent, int npass,
                                              uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ bh,
                                              uint32_t *__restrict__ err) {
  __shared__ uint32_t h[kMaxPasses][kRadix];
  for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += blockDim.x) (&h[0][0])[i] = 0;
  __syncthreads();
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    longlong2 t = reinterpret_cast<const longlong2 *>(edges)[i];
    uint64_t k0 = sent, k1 = sent;
    if (t.x < 0 || t.x >= n || t.y < 0 || t.y >= n) {
      bad = true;
    } else if (t.x != t.y) {
      const uint64_t w = wts ? (uint64_t)wts[i] : 0;
      k0 = ((uint64_t)t.x << (sb + wb)) | ((uint64_t)t.y << wb) | w;
      k1 = ((uint64_t)t.y << (sb + wb)) | ((uint64_t)t.x << wb) | w;
    }
    ulonglong2 o;
    o.x = k0;
    o.y = k1;
    reinterpret_cast<ulonglong2 *>(keys)[i] = o;
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) {
      if (p < npass) {
        atomicAdd(&h[p][(uint32_t)(k0 >> (8 * p)) & 0xFF], 1u);
        atomicAdd(&h[p][(uint32_t)(k1 >> (8 * p)) & 0xFF], 1u);
      }
    }
  }
  if (__ballot(bad) != 0 && __lane_id() == 0) atomicOr(err, 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < npass * kRadix; i += blockDim.x)
    bh[(int64_t)blockIdx.x * npass * kRadix + i] = (&h[0][0])[i];
}

// ghist[pass][digit] += the counts of blocks slice, slice + S, ... (S slices
// per pass; ghist starts at zero).
constexpr int kHistSlices = 32;
__global__ __launch_bounds__(kRadix) void k_hist_reduce(const uint32_t *__restrict__ bh, int nbp,
                                                        int npass,
                                                        unsigned long long *__restrict__ ghist) {
  const int p = blockIdx.x / kHistSlices, sl = blockIdx.x % kHistSlices;
  uint64_t acc = 0;
  for (int b = sl; b < nbp; b += kHistSlices)
    acc += bh[((int64_t)b * npass + p) * kRadix + threadIdx.x];
  if (acc) atomicAdd(ghist + p * kRadix + threadIdx.x, (unsigned long long)acc);
}

// dstart[pass][digit] = where the keys of that digit start in the pass's output.
__global__ __launch_bounds__(kRadix) void k_digit_starts(const unsigned long long *__restrict__ ghist,
                                                         uint64_t *__restrict__ dstart) {
  __shared__ uint64_t s[kRadix / kWave];
  const int i = blockIdx.x * kRadix + threadIdx.x;
  uint64_t tot;
  dstart[i] = block_excl_scan<kRadix, uint64_t>((uint64_t)ghist[i], s, tot);
}

// Exclusive scan of a uint32 array into uint64 (single block); *total = sum.
// Each thread takes a contiguous segment whose length is a multiple of 4, read
// 16 bytes at a time (`in` comes from hipMalloc: 16-byte aligned), so that a
// long array (a million tile counts) costs few dependent loads per thread.
__global__ __launch_bounds__(kScanBlock) void k_scan_u32(const uint32_t *__restrict__ in,
                                                        uint64_t *__restrict__ out,
                                                        int64_t len,
                                                        uint64_t *__restrict__ total) {
  __shared__ uint64_t s[kScanBlock / kWave];
  const int64_t per = ((len + kScanBlock - 1) / kScanBlock + 3) & ~int64_t(3);
  const int64_t b = std::min<int64_t>(per * threadIdx.x, len), e = std::min<int64_t>(b + per, len);
  const int64_t e4 = b + ((e - b) & ~int64_t(3));  // whole groups of 4
  uint64_t sum = 0;
#pragma unroll 4
  for (int64_t i = b; i < e4; i += 4) {
    const uint4 x = *reinterpret_cast<const uint4 *>(in + i);
    sum += (uint64_t)x.x + x.y + x.z + x.w;
  }
  for (int64_t i = e4; i < e; ++i) sum += in[i];
  uint64_t tot;
  uint64_t run = block_excl_scan<kScanBlock, uint64_t>(sum, s, tot);
#pragma unroll 4
  for (int64_t i = b; i < e4; i += 4) {
    const uint4 x = *reinterpret_cast<const uint4 *>(in + i);
    out[i] = run;
    out[i + 1] = run + x.x;
    out[i + 2] = run + x.x + x.y;
    out[i + 3] = run + x.x + x.y + x.z;
    run += (uint64_t)x.x + x.y + x.z + x.w;
  }
  for (int64_t i = e4; i < e; ++i) {
    const uint64_t x = in[i];
    out[i] = run;
    run += x;
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

// Status of (tile, digit) in one pass: the count of that digit in the tile
// (state kStAgg) or in the tile and every tile before it (kStIncl), tagged
// with the pass so that the words of an earlier pass read as not ready.
constexpr uint64_t kStCount = (1ull << 56) - 1;
constexpr uint64_t kStTagMask = 63ull << 56;
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStIncl = 2ull << 62;
// A look-back waits on a tile that a running workgroup holds; it gives up
// (and raises bit 2 of err, which ends every other wait of the launch) after
// this many polls, so the launch always ends.
constexpr int kSpinLimit = 1 << 18;

// One stable pass over one 8-bit digit.  Workgroups take tiles of kSortTile
// keys in increasing order from a counter, one ahead of the tile they work on
// (a tile only waits on tiles with smaller numbers; the smallest unfinished
// tile is one that a running workgroup works on, so every wait ends).  In a
// tile, wavefront w owns keys [w*kWaveKeys, (w+1)*kWaveKeys) in kSortItems
// steps of 64; a key's rank inside its wavefront is the count of equal digits
// in earlier steps (LDS counter) plus earlier lanes of its step (match mask
// from 8 ballots).  Thread d then publishes the tile's count of digit d, adds
// up the counts of the tiles before (walking back to the first that
// published an inclusive count) and publishes its own inclusive count.  The
// next tile's keys are loaded while the current one is ranked and written.
__global__ __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_onesweep(
    const uint64_t *__restrict__ kin, uint64_t *__restrict__ kout, uint64_t nkeys, int shift,
    uint64_t tag, uint32_t ntiles, const uint64_t *__restrict__ dstart, uint64_t *status,
    uint32_t *ctr, uint32_t *err) {
  __shared__ uint64_t base[kRadix];
  __shared__ uint32_t wh[4][kRadix];
  __shared__ uint32_t doff[kRadix];        // where each digit's run starts in the tile
  __shared__ uint64_t s_keys[kSortTile];   // the tile's keys in digit order
  __shared__ uint32_t s_scan[kSortBlock / kWave];
  __shared__ uint32_t s_tile[2];  // the first tile; the next tile
  const int tid = threadIdx.x, w = tid / kWave, lane = __lane_id();
  if (tid == 0) s_tile[0] = atomicAdd(ctr, 1u);
  __syncthreads();
  uint32_t cur = s_tile[0];
  uint64_t next[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t idx = (uint64_t)cur * kSortTile + (uint64_t)w * kWaveKeys + (uint64_t)j * kWave + lane;
    next[j] = (cur < ntiles && idx < nkeys) ? kin[idx] : 0;
  }
  while (cur < ntiles) {
    const uint64_t tbase = (uint64_t)cur * kSortTile;
    for (int d = lane; d < kRadix; d += kWave) wh[w][d] = 0;
    uint64_t key[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) key[j] = next[j];
    if (tid == 0) s_tile[1] = atomicAdd(ctr, 1u);
    __syncthreads();  // the previous tile's readers of s_tile[1] passed the barrier that ended it
    const uint32_t nxt = s_tile[1];
    if (nxt < ntiles) {
#pragma unroll
      for (int j = 0; j < kSortItems; ++j) {
        const uint64_t idx = (uint64_t)nxt * kSortTile + (uint64_t)w * kWaveKeys + (uint64_t)j * kWave + lane;
        next[j] = idx < nkeys ? kin[idx] : 0;
      }
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      uint64_t idx = tbase + (uint64_t)w * kWaveKeys + (uint64_t)j * kWave + lane;
      bool valid = idx < nkeys;
      uint64_t k = key[j];
      uint32_t d = (uint32_t)(k >> shift) & 0xFF;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        uint64_t bal = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? bal : ~bal;
      }
      int leader = peers ? (__ffsll((unsigned long long)peers) - 1) : 0;
      uint32_t old = 0;
      if (valid && lane == leader) old = atomicAdd(&wh[w][d], (uint32_t)__popcll(peers));
      old = __shfl(old, leader, kWave);
      // old + the number of peers in lower lanes
      rank[j] = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)peers, old));
    }
    __syncthreads();
    uint32_t cnt = 0;  // kSortBlock == kRadix: thread tid owns digit tid
    {
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        uint32_t c = wh[ww][tid];
        wh[ww][tid] = cnt;
        cnt += c;
      }
      uint32_t total;
      doff[tid] = block_excl_scan<kSortBlock, uint32_t>(cnt, s_scan, total);
    }
    // publish this tile's count of digit tid for the tiles after it
    uint64_t *const st = status + (uint64_t)cur * kRadix + tid;
    __hip_atomic_store(st, tag | (cur == 0 ? kStIncl : kStAgg) | cnt, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();  // doff and wh complete
    // Stage the tile in LDS in digit order (stable: within a digit, keys keep
    // their input order), then write each digit's run out contiguously, so a
    // wavefront's stores cover few lines instead of one line per lane.
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      uint64_t idx = tbase + (uint64_t)w * kWaveKeys + (uint64_t)j * kWave + lane;
      if (idx < nkeys) {
        uint32_t d = (uint32_t)(key[j] >> shift) & 0xFF;
        const uint32_t lp = doff[d] + wh[w][d] + rank[j];
        if (lp < (uint32_t)kSortTile) s_keys[lp] = key[j];
      }
    }
    // decoupled look-back over the tiles before this one, for digit tid
    uint64_t excl = 0;
    if (cur != 0) {
      uint64_t k = cur - 1;
      int spins = 0;
      while (true) {
        const uint64_t v = __hip_atomic_load(status + k * kRadix + tid, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if ((v & kStTagMask) != tag || (v & (3ull << 62)) == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(err, 2u);
            break;
          }
          if ((spins & 63) == 0 &&
              (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2u) != 0)
            break;
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v & kStCount;
        if ((v & kStIncl) != 0 || k == 0) break;
        --k;
      }
      __hip_atomic_store(st, tag | kStIncl | (excl + cnt), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    base[tid] = dstart[tid] + excl;
    __syncthreads();  // s_keys and base complete
    const uint32_t tile_n = (uint32_t)std::min<uint64_t>(kSortTile, nkeys - tbase);
    for (uint32_t i = tid; i < tile_n; i += kSortBlock) {
      const uint64_t k = s_keys[i];
      const uint32_t d = (uint32_t)(k >> shift) & 0xFF;
      const uint64_t pos = base[d] + (i - doff[d]);
      if (pos < nkeys) kout[pos] = k;
    }
    __syncthreads();
    cur = nxt;
  }
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }

// Key i opens a run of one (u, v) (the weight bits below wb are ignored).
__device__ __forceinline__ bool is_head(const uint64_t *keys, uint64_t i, uint64_t sent, int wb) {
  uint64_t k = keys[i];
  return k != sent && (i == 0 || (keys[i - 1] >> wb) != (k >> wb));
}

// Distinct keys per compaction tile of kCompactTile keys (only the count, so
// the threads take the tile's keys strided by the block: coalesced loads).
__global__ __launch_bounds__(kCompactBlock) void k_heads_count(const uint64_t *__restrict__ keys,
                                                               uint64_t nkeys, uint64_t sent,
                                                               int wb,
                                                               uint32_t *__restrict__ bsum) {
  __shared__ uint32_t s[kCompactBlock / kWave];
  const uint64_t b = (uint64_t)blockIdx.x * kCompactTile + threadIdx.x;
  uint32_t c = 0;
  for (int j = 0; j < kCompactItems; ++j) {
    uint64_t i = b + (uint64_t)j * kCompactBlock;
    if (i < nkeys && is_head(keys, i, sent, wb)) ++c;
  }
  uint32_t tot = block_sum<kCompactBlock, uint32_t>(c, s);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kCompactBlock) void k_compact(
    const uint64_t *__restrict__ keys, uint64_t nkeys, uint64_t sent, int sb, int wb, int64_t n,
    const uint64_t *__restrict__ boff, int32_t *__restrict__ col_idx,
    int64_t *__restrict__ row_ptr, uint8_t *__restrict__ wt) {
  __shared__ uint32_t s[kCompactBlock / kWave];
  // The tile (and the key before it) staged in LDS by coalesced loads: thread t
  // then takes its 8 consecutive keys from there (the compaction keeps key
  // order, so a thread's keys must be consecutive).  Past the end: sentinels.
  // The same LDS then gathers the tile's kept entries, which the block writes
  // out with coalesced stores.
  __shared__ uint64_t s_k[kCompactTile + 1];
  const uint64_t t0 = (uint64_t)blockIdx.x * kCompactTile;
  for (int x = threadIdx.x; x <= kCompactTile; x += kCompactBlock) {
    const uint64_t i = t0 + (uint64_t)x;  // key i - 1 goes to s_k[x]
    s_k[x] = (i == 0 || i - 1 >= nkeys) ? sent : keys[i - 1];
  }
  __syncthreads();
  const int x0 = threadIdx.x * kCompactItems + 1;  // s_k index of this thread's first key
  const uint64_t b = t0 + (uint64_t)threadIdx.x * kCompactItems;
  uint64_t kk[kCompactItems + 1];  // kk[0]: the key before this thread's first
#pragma unroll
  for (int j = 0; j <= kCompactItems; ++j) kk[j] = s_k[x0 - 1 + j];
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kCompactItems; ++j) {
    const uint64_t k = kk[j + 1];
    if (b + j < nkeys && k != sent && (kk[j] >> wb) != (k >> wb)) ++c;
  }
  uint32_t tot;
  const uint32_t local0 = block_excl_scan<kCompactBlock, uint32_t>(c, s, tot);
  __syncthreads();  // every thread holds its keys: s_k is reused for the output
  int32_t *s_col = reinterpret_cast<int32_t *>(s_k);
  uint8_t *s_wt = reinterpret_cast<uint8_t *>(s_col + kCompactTile);
  uint64_t pos = boff[blockIdx.x] + local0;
  uint32_t local = local0;
  const uint64_t vmask = (1ull << sb) - 1;
#pragma unroll
  for (int j = 0; j < kCompactItems; ++j) {
    const uint64_t i = b + j;
    if (i >= nkeys) break;
    const uint64_t k = kk[j + 1];
    const uint64_t prev = kk[j];  // the sentinel before key 0
    const int64_t up = i ? (int64_t)(prev >> (sb + wb)) : -1;
    if (k != sent) {
      if (i == 0 || (prev >> wb) != (k >> wb)) {
        s_col[local] = (int32_t)((k >> wb) & vmask);
        if (wt) s_wt[local] = (uint8_t)(k & 0xffu);
        const int64_t u = std::min<int64_t>((int64_t)(k >> (sb + wb)), n - 1);
        for (int64_t r = up + 1; r <= u; ++r) row_ptr[r] = (int64_t)pos;
        ++pos;
        ++local;
      }
    } else if (i == 0 || prev != sent) {
      // first sentinel: rows after the last stored key are empty
      for (int64_t r = up + 1; r <= n; ++r) row_ptr[r] = (int64_t)pos;
    }
  }
  __syncthreads();
  const uint64_t base = boff[blockIdx.x];
  for (uint32_t x = threadIdx.x; x < tot; x += kCompactBlock) {
    col_idx[base + x] = s_col[x];
    if (wt) wt[base + x] = s_wt[x];
  }
}

// iso[w] bit l = vertex 64w+l has degree 0 (or lies past n).
__global__ __launch_bounds__(256) void k_iso(const int64_t *__restrict__ rp, int64_t n,
                                             int64_t words, uint64_t *__restrict__ iso,
                                             unsigned long long *__restrict__ nonisolated) {
  __shared__ uint64_t s[4];
  int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  uint64_t cnt = 0;
  for (int64_t w = gw; w < words; w += nw) {
    int64_t v = w * kWave + __lane_id();
    bool d0 = v >= n || rp[v + 1] == rp[v];
    uint64_t mk = __ballot(d0);
    if (__lane_id() == 0) {
      iso[w] = mk;
      cnt += (uint64_t)__popcll(~mk);
    }
  }
  uint64_t tot = block_sum<256, uint64_t>(cnt, s);
  if (threadIdx.x == 0 && tot) atomicAdd(nonisolated, (unsigned long long)tot);
}

__global__ void k_find_hubs(const int64_t *__restrict__ rp, int64_t n,
                            int32_t *__restrict__ list, unsigned long long *__restrict__ count) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (rp[v + 1] - rp[v] > kHubDeg) list[atomicAdd(count, 1ull)] = (int32_t)v;
}

__global__ void k_hub_chunks(const int64_t *__restrict__ rp, const int32_t *__restrict__ list,
                             int64_t h, uint64_t *__restrict__ chunks) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < h) {
    int32_t v = list[i];
    chunks[i] = (uint64_t)((rp[v + 1] - rp[v] + kHubChunk - 1) / kHubChunk);
  }
}


// deg16[v] = min(degree, 0xffff): the degrees the hint scan compares, in an
// array small enough to stay cached (2 bytes per vertex instead of the two
// 8-byte row offsets); the few saturated ones are read exactly from rp.
__global__ void k_deg16(const int64_t *__restrict__ rp, int64_t n, uint16_t *__restrict__ d16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    d16[v] = (uint16_t)std::min<int64_t>(rp[v + 1] - rp[v], 0xffff);
}

__device__ __forceinline__ uint64_t hint_key(const int64_t *rp, const uint16_t *d16, int32_t u) {
  // larger degree first, then smaller id
  uint64_t d = d16[u];
  if (d == 0xffff) d = (uint64_t)(rp[u + 1] - rp[u]);
  return (d << 32) | (uint64_t)(0x7fffffffu - (uint32_t)u);
}

// Hint candidates: the kHintCand vertices of largest key (degree, then smaller
// id), in key order, held by every workgroup in an LDS hash table (id -> rank).
// Any candidate's key exceeds that of every other vertex, so when a row holds
// a candidate its best key is that of its smallest-rank candidate; only rows
// without one need the degrees of their entries (about 1 % of the entries of
// the Kronecker graphs).
constexpr int kHintCand = 2048;
constexpr int kCandSlots = 8192;  // load factor 1/4
constexpr uint64_t kNone = ~0ull;

struct CandSet {
  int32_t *id;     // kCandSlots, -1 = empty
  uint16_t *rank;  // kCandSlots
  __device__ __forceinline__ static uint32_t slot(int32_t u) {
    return ((uint32_t)u * 0x9E3779B1u) >> (32 - 13);
  }
  // every thread of the block takes part
  __device__ void fill(const int32_t *__restrict__ cand, int kc) {
    for (int x = threadIdx.x; x < kCandSlots; x += blockDim.x) id[x] = -1;
    __syncthreads();
    for (int r = threadIdx.x; r < kc; r += blockDim.x) {
      const int32_t u = cand[r];
      uint32_t x = slot(u);
      while (atomicCAS(&id[x], -1, u) != -1) x = (x + 1) & (kCandSlots - 1);
      rank[x] = (uint16_t)r;
    }
    __syncthreads();
  }
  __device__ __forceinline__ uint64_t rank_of(int32_t u) const {
    uint32_t x = slot(u);
    while (true) {
      const int32_t y = id[x];
      if (y == u) return rank[x];
      if (y < 0) return kNone;
      x = (x + 1) & (kCandSlots - 1);
    }
  }
};

// Rows of a wavefront's 64 lanes (len entries from 32-bit offset b32 each)
// laid end to end, one entry per lane per 64-entry window; f(u) maps each
// entry to a value and the values of a row are combined by `comb` (a minimum
// or maximum, taken by LDS atomics into the row's slot).  Returns the lane's
// own row's value (ident for an empty row).
template <class F, class C>
__device__ uint64_t packed_rows(uint32_t len, uint32_t b32, uint64_t ident, const int32_t *ci,
                                F f, C comb, uint32_t *s_base, int32_t *s_row, uint64_t *s_acc) {
  const int lane = __lane_id();
  const int wb = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) * kWave;  // scalar
  const uint64_t upto_mask = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
  const uint32_t incl = wave_incl_scan(len);
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  const uint32_t pre = incl - len;
  // row entry j of the window sits at s_base[r] + j: b - pre + j lies in
  // [0, nnz) < 2^32, so 32-bit wrap-around arithmetic gives it exactly
  s_base[wb + lane] = b32 - pre;
  s_acc[wb + lane] = ident;
  // s_row[p] = tag << 6 | lane when that lane's row starts at position p of
  // the window with that tag (tags count windows from 1 in this call): a lane
  // reads its own slot and one ballot gives the window's row starts
  s_row[wb + lane] = 0;
  uint32_t tag = 0;
  int carry = 0;
  for (uint32_t j0 = 0; j0 < total; j0 += kWave) {
    ++tag;
    const bool starts = len > 0 && pre >= j0 && pre < j0 + kWave;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (starts) s_row[wb + (int)(pre - j0)] = (int32_t)((tag << 6) | (uint32_t)lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint64_t S = __ballot(((uint32_t)s_row[wb + lane] >> 6) == tag);
    const uint64_t upto = S & upto_mask;
    const int r = upto ? (s_row[wb + (kWave - 1 - __clzll((long long)upto))] & (kWave - 1)) : carry;
    const uint32_t j = j0 + lane;
    uint64_t val = ident;
    if (j < total) val = f(ci[(uint32_t)(s_base[wb + r] + j)]);
    // each entry with a value combines it into its row's slot by an LDS
    // atomic (min and max do not depend on the order)
    if (val != ident) comb.into(&s_acc[wb + r], val);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    carry = (int)__builtin_amdgcn_readlane(r, kWave - 1);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint64_t out = s_acc[wb + lane];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  return out;
}

struct MinOp {
  __device__ __forceinline__ void into(uint64_t *slot, uint64_t v) const {
    atomicMin((unsigned long long *)slot, (unsigned long long)v);
  }
};
struct MaxOp {
  __device__ __forceinline__ void into(uint64_t *slot, uint64_t v) const {
    atomicMax((unsigned long long *)slot, (unsigned long long)v);
  }
};

// hint_id[v] = the target (or -1); hint[v] = the same with kHintOnly set when
// it is v's only neighbour (only used while n <= 2^30, so ids leave bit 30 free).
// A wavefront takes 64 consecutive vertices (hub rows aside, see k_hint_hubs):
// first the candidate ranks of their entries (LDS lookups), then, for rows
// without a candidate, the keys of their entries.
// 1,024-thread workgroups: the 48 KB candidate table in LDS is shared by 16
// wavefronts, and two workgroups fit a compute unit.
constexpr int kHintBlock = 1024;
__global__ __launch_bounds__(kHintBlock) void k_hint(const int64_t *__restrict__ rp,
                                              const uint16_t *__restrict__ d16,
                                              const int32_t *__restrict__ ci, int64_t n,
                                              int64_t words, const int32_t *__restrict__ cand,
                                              int kc, int32_t *__restrict__ hint,
                                              int32_t *__restrict__ hint_id) {
  __shared__ uint32_t s_base[kHintBlock];
  __shared__ int32_t s_row[kHintBlock];
  __shared__ uint64_t s_acc[kHintBlock];
  __shared__ int32_t s_cid[kCandSlots];
  __shared__ uint16_t s_crank[kCandSlots];
  CandSet cs{s_cid, s_crank};
  cs.fill(cand, kc);
  const int lane = __lane_id();
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t w = gw; w < words; w += nw) {
    const int64_t v = w * kWave + lane;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = rp[v];
      e = rp[v + 1];
    }
    const int64_t d = e - b;
    const uint32_t len = d <= kHubDeg ? (uint32_t)d : 0u;
    uint64_t rank = kNone;
    if (kc > 0)
      rank = packed_rows(len, (uint32_t)b, kNone, ci, [&](int32_t u) { return cs.rank_of(u); },
                         MinOp(), s_base, s_row, s_acc);
    const uint64_t best =
        packed_rows(rank == kNone ? len : 0u, (uint32_t)b, 0ull, ci,
                    [&](int32_t u) { return hint_key(rp, d16, u); }, MaxOp(), s_base, s_row, s_acc);
    if (v < n && d <= kHubDeg) {
      const int32_t t = rank != kNone ? cand[rank]
                                      : (best ? (int32_t)(0x7fffffffu - (uint32_t)(best & 0xffffffffu))
                                              : -1);
      hint_id[v] = t;
      hint[v] = (t >= 0 && d == 1 && n <= (1ll << 30)) ? (t | kHintOnly) : t;
    }
  }
}

// Hub rows (longer than kHubDeg) in kHubChunk-edge pieces, one wavefront per
// piece.  RANKED: the piece's smallest candidate rank goes to best[h] by an
// atomic minimum; otherwise (hubs left without a candidate, best[h] = kNone)
// the piece's best key goes to key[h] by an atomic maximum.
// off[h] = the first piece of hub h (off[nh] = pieces in all).
template <bool RANKED>
__global__ __launch_bounds__(kHintBlock) void k_hint_hubs(const int64_t *__restrict__ rp,
                                                   const uint16_t *__restrict__ d16,
                                                   const int32_t *__restrict__ ci,
                                                   const int32_t *__restrict__ hubs,
                                                   const uint64_t *__restrict__ off, int64_t nh,
                                                   const int32_t *__restrict__ cand, int kc,
                                                   unsigned long long *__restrict__ best,
                                                   unsigned long long *__restrict__ key) {
  __shared__ int32_t s_cid[RANKED ? kCandSlots : 1];
  __shared__ uint16_t s_crank[RANKED ? kCandSlots : 1];
  CandSet cs{s_cid, s_crank};
  if (RANKED) cs.fill(cand, kc);
  const int lane = __lane_id();
  const int64_t pieces = (int64_t)off[nh];
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < pieces; c += nw) {
    // the hub of piece c: the last h with off[h] <= c
    int64_t lo = 0, hi = nh;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)off[mid] <= c) lo = mid; else hi = mid;
    }
    if (!RANKED && best[lo] != kNone) continue;  // wave-uniform
    const int32_t v = hubs[lo];
    const int64_t kb = rp[v] + (c - (int64_t)off[lo]) * kHubChunk;
    const int64_t ke = std::min<int64_t>(kb + kHubChunk, rp[v + 1]);
    uint64_t m = RANKED ? kNone : 0;
    for (int64_t k = kb + lane; k < ke; k += kWave) {
      const int32_t u = ci[k];
      if (RANKED)
        m = std::min(m, cs.rank_of(u));
      else
        m = std::max(m, hint_key(rp, d16, u));
    }
#pragma unroll
    for (int dd = kWave / 2; dd >= 1; dd >>= 1) {
      const uint64_t o = __shfl_xor(m, dd, kWave);
      m = RANKED ? std::min(m, o) : std::max(m, o);
    }
    if (lane == 0) {
      if (RANKED && m != kNone) atomicMin(best + lo, (unsigned long long)m);
      if (!RANKED && m) atomicMax(key + lo, (unsigned long long)m);
    }
  }
}

// key[h] = hint_key of hub h (degree, then smaller id).
__global__ void k_hub_keys(const int64_t *__restrict__ rp, const int32_t *__restrict__ hubs,
                           int64_t nh, uint64_t *__restrict__ key) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < nh) {
    const int32_t u = hubs[h];
    key[h] = ((uint64_t)(rp[u + 1] - rp[u]) << 32) | (uint64_t)(0x7fffffffu - (uint32_t)u);
  }
}

// The hubs' hints from their best candidate ranks, or else their best keys (a
// hub has more than one neighbour, so never kHintOnly).
__global__ void k_hint_hubs_write(const int32_t *__restrict__ hubs, int64_t nh,
                                  const unsigned long long *__restrict__ best,
                                  const unsigned long long *__restrict__ key,
                                  const int32_t *__restrict__ cand,
                                  int32_t *__restrict__ hint, int32_t *__restrict__ hint_id) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < nh) {
    const uint64_t r = best[h], b = key[h];
    const int32_t t = r != kNone ? cand[r]
                                 : (b ? (int32_t)(0x7fffffffu - (uint32_t)(b & 0xffffffffu)) : -1);
    hint_id[hubs[h]] = t;
    hint[hubs[h]] = t;
  }
}

constexpr int kHotBins = 1024;
constexpr int kHotTile = 4096;  // vertices per workgroup when numbering hot targets

// cnt[t] = number of vertices whose hint is t.  Most vertices name one of the
// hint candidates (the hubs of largest degree): those are counted in LDS by
// candidate rank and added to cnt once per workgroup, since a device-scope
// atomic per wavefront on one hub's counter would serialise at that address.
// The other targets take one atomic per distinct target per wavefront.
__global__ __launch_bounds__(256) void k_hint_count(const int32_t *__restrict__ hint, int64_t n,
                                                    const int32_t *__restrict__ cand, int kc,
                                                    uint32_t *__restrict__ cnt) {
  __shared__ int32_t s_cid[kCandSlots];
  __shared__ uint16_t s_crank[kCandSlots];
  __shared__ uint32_t s_cnt[kHintCand];
  CandSet cs{s_cid, s_crank};
  for (int i = threadIdx.x; i < kHintCand; i += blockDim.x) s_cnt[i] = 0;
  cs.fill(cand, kc);
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;  // a multiple of kWave
  const int64_t span = ((n + kWave - 1) / kWave) * kWave;    // every lane runs each round
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < span; v += stride) {
    const int32_t h = v < n ? hint[v] : -1;
    const int32_t t = h >= 0 ? (h & ~kHintOnly) : -1;
    bool todo = t >= 0;
    if (todo && kc > 0) {
      const uint64_t r = cs.rank_of(t);
      if (r != kNone) {
        atomicAdd(&s_cnt[r], 1u);
        todo = false;
      }
    }
    uint64_t m;
    while ((m = __ballot(todo)) != 0) {
      const int L = __ffsll((unsigned long long)m) - 1;
      const int32_t tl = __shfl(t, L, kWave);
      const bool same = todo && t == tl;
      const uint64_t grp = __ballot(same);
      if (lane == L) atomicAdd(cnt + tl, (uint32_t)__popcll(grp));
      if (same) todo = false;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kc; i += blockDim.x)
    if (s_cnt[i]) atomicAdd(cnt + cand[i], s_cnt[i]);
}

// hist[c] = number of targets named by c vertices (c >= kHotBins - 1 share the last bin)
__global__ __launch_bounds__(256) void k_hint_hist(const uint32_t *__restrict__ cnt, int64_t n,
                                                   uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[kHotBins];
  for (int i = threadIdx.x; i < kHotBins; i += 256) h[i] = 0;
  __syncthreads();
  int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const uint32_t c = cnt[i];
    if (c) atomicAdd(h + std::min<uint32_t>(c, kHotBins - 1), 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHotBins; i += 256)
    if (h[i]) atomicAdd(hist + i, h[i]);
}

__global__ __launch_bounds__(256) void k_hot_count(const uint32_t *__restrict__ cnt, int64_t n,
                                                   uint32_t cmin, uint32_t *__restrict__ bsum) {
  __shared__ uint32_t s[256 / kWave];
  const int64_t b = (int64_t)blockIdx.x * kHotTile, e = std::min<int64_t>(b + kHotTile, n);
  uint32_t c = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) c += cnt[i] >= cmin;
  const uint32_t tot = block_sum<256, uint32_t>(c, s);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Numbers the selected targets in vertex order: hot[r] = t and, in place,
// cnt[t] = r (0xffffffff for targets not selected).
__global__ __launch_bounds__(256) void k_hot_write(uint32_t *__restrict__ cnt, int64_t n,
                                                   uint32_t cmin, const uint64_t *__restrict__ boff,
                                                   int32_t *__restrict__ hot) {
  __shared__ uint32_t s[256 / kWave];
  const int64_t b = (int64_t)blockIdx.x * kHotTile, e = std::min<int64_t>(b + kHotTile, n);
  uint32_t base = (uint32_t)boff[blockIdx.x];
  for (int64_t i0 = b; i0 < e; i0 += 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool sel = i < e && cnt[i] >= cmin;
    uint32_t tot;
    const uint32_t pos = base + block_excl_scan<256, uint32_t>(sel ? 1u : 0u, s, tot);
    if (sel) hot[pos] = (int32_t)i;
    if (i < e) cnt[i] = sel ? pos : 0xffffffffu;
    base += tot;
  }
}

__global__ void k_hint_encode(int32_t *__restrict__ hint, int64_t n,
                              const uint32_t *__restrict__ rank) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t h = hint[v];
    if (h >= 0) {
      const uint32_t r = rank[h & ~kHintOnly];
      if (r != 0xffffffffu) hint[v] = (int32_t)(0x80000000u | (h & kHintOnly) | r);
    }
  }
}

// Vertices of degree >= 1 in each chunk of 64 bitmap words (one wavefront per
// chunk; the isolated bitmap has its padding bits past n set).
__global__ __launch_bounds__(256) void k_chunk_count(const uint64_t *__restrict__ iso,
                                                     int64_t words, int64_t chunks,
                                                     uint32_t *__restrict__ cnt) {
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * (256 / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave; c < chunks; c += stride) {
    const int64_t w = c * kWave + lane;
    const uint32_t q = w < words ? (uint32_t)__popcll(~iso[w]) : 0u;
    const uint32_t t = wave_sum<uint32_t>(q);
    if (lane == 0) cnt[c] = t;
  }
}

// hint_c[rank] = hint[v] for the rank-th vertex v of degree >= 1: lane l of the
// chunk's wavefront takes bitmap word l and writes its vertices' hints in order
// from its exclusive prefix of the chunk's counts.
__global__ __launch_bounds__(256) void k_hint_compact(const int32_t *__restrict__ hint,
                                                      const uint64_t *__restrict__ iso,
                                                      int64_t words, int64_t chunks,
                                                      const uint64_t *__restrict__ cbase,
                                                      int32_t *__restrict__ hint_c) {
  const int lane = __lane_id();
  const int64_t stride = (int64_t)gridDim.x * (256 / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave; c < chunks; c += stride) {
    const int64_t w = c * kWave + lane;
    uint64_t x = w < words ? ~iso[w] : 0ull;
    const uint32_t q = (uint32_t)__popcll(x);
    uint64_t r = cbase[c] + (wave_incl_scan<uint32_t>(q) - q);
    while (x) {
      const int b = __ffsll((unsigned long long)x) - 1;
      x &= x - 1;
      hint_c[r++] = hint[w * 64 + b];
    }
  }
}

__global__ void k_rp32(const int64_t *__restrict__ rp, int64_t len, uint32_t *__restrict__ out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    out[i] = (uint32_t)rp[i];
}

int grid_cap(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

struct DevBuf {
  void *p = nullptr;
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

g5_status build_csr_impl(const int64_t *edges, const uint8_t *weights, bool weighted, int64_t m,
                         int64_t n, hipStream_t s, g5_csr **out) {
  *out = nullptr;
  if (m < 0 || n < 1 || n > 2147483647LL || (m > 0 && !edges) || (weighted && m > 0 && !weights)) {
    set_error("g5_build_csr: need m >= 0, 1 <= n <= 2^31-1 and a non-NULL edge list (and weight "
              "list)");
    return G5_EINVAL;
  }
  int dev = 0, ncu = 256;
  G5_HIP(hipGetDevice(&dev));
  G5_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

  int sb = 1;
  while ((1ll << sb) < n) ++sb;
  const int wb = weighted ? 8 : 0;
  if (2 * sb + wb > 64) {
    set_error("g5_build_csr_w: weighted graphs need n <= 2^28");
    return G5_EINVAL;
  }
  const int key_bits = 2 * sb + wb;
  const uint64_t sent = (key_bits >= 64) ? ~0ull : ((1ull << key_bits) - 1);
  const uint64_t nkeys = 2ull * (uint64_t)m;

  DevBuf ka, kb, counts, offs, misc;
  G5_HIP(hipMalloc(&ka.p, (nkeys + 1) * sizeof(uint64_t)));
  G5_HIP(hipMalloc(&kb.p, (nkeys + 1) * sizeof(uint64_t)));
  G5_HIP(hipMalloc(&misc.p, 64));
  uint32_t *err = (uint32_t *)misc.p;
  uint64_t *nnz_dev = (uint64_t *)((char *)misc.p + 8);
  unsigned long long *noniso_dev = (unsigned long long *)((char *)misc.p + 16);
  G5_HIP(hipMemsetAsync(misc.p, 0, 64, s));
  uint64_t *keys = (uint64_t *)ka.p, *alt = (uint64_t *)kb.p;

  if (m > 0) {
    const int nbp = grid_cap(m, 256, ncu * 16);
    // radix sort: one sweep per pass over tiles taken in order by resident
    // workgroups (the pass counters and the status words start at zero)
    const int npass = (key_bits + 7) / 8;
    const uint64_t ntiles = (nkeys + kSortTile - 1) / kSortTile;
    if (ntiles >= (1ull << 32)) {
      set_error("g5_build_csr: too many tuples for the sort");
      return G5_ERANGE;
    }
    const size_t hist_bytes = (size_t)nbp * npass * kRadix * sizeof(uint32_t);
    const size_t status_bytes = (size_t)ntiles * kRadix * sizeof(uint64_t);
    G5_HIP(hipMalloc(&counts.p, hist_bytes + 2 * kMaxPasses * kRadix * sizeof(uint64_t) +
                                    kMaxPasses * sizeof(uint32_t)));
    G5_HIP(hipMalloc(&offs.p, status_bytes));
    uint32_t *bh = (uint32_t *)counts.p;
    unsigned long long *ghist = (unsigned long long *)((char *)counts.p + hist_bytes);
    uint64_t *dstart = (uint64_t *)(ghist + kMaxPasses * kRadix);
    uint32_t *ctr = (uint32_t *)(dstart + kMaxPasses * kRadix);
    G5_HIP(hipMemsetAsync(ghist, 0, kMaxPasses * kRadix * sizeof(uint64_t), s));
    G5_HIP(hipMemsetAsync(ctr, 0, kMaxPasses * sizeof(uint32_t), s));
    G5_HIP(hipMemsetAsync(offs.p, 0, status_bytes, s));
    hipLaunchKernelGGL(k_pack, dim3(nbp), dim3(256), 0, s, edges, weighted ? weights : nullptr,
                       m, n, sb, wb, sent, npass, keys, bh, err);
    hipLaunchKernelGGL(k_hist_reduce, dim3(npass * kHistSlices), dim3(kRadix), 0, s,
                       (const uint32_t *)bh, nbp, npass, ghist);
    hipLaunchKernelGGL(k_digit_starts, dim3(npass), dim3(kRadix), 0, s,
                       (const unsigned long long *)ghist, dstart);
    G5_LAUNCH_CHECK();
    int per_cu = 0;
    G5_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_onesweep, kSortBlock, 0));
    const int nb = (int)std::min<uint64_t>(ntiles, (uint64_t)ncu * std::max(per_cu, 1));
    for (int p = 0; p < npass; ++p) {
      hipLaunchKernelGGL(k_onesweep, dim3(nb), dim3(kSortBlock), 0, s, keys, alt, nkeys, 8 * p,
                         (uint64_t)(p + 1) << 56, (uint32_t)ntiles,
                         (const uint64_t *)(dstart + p * kRadix), (uint64_t *)offs.p, ctr + p,
                         err);
      G5_LAUNCH_CHECK();
      std::swap(keys, alt);
    }
  }
  // keys[nkeys] = SENT guarantees a first sentinel for the tail rows
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, keys + nkeys, sent);
  const uint64_t ntot = nkeys + 1;
  int64_t cblocks = (int64_t)((ntot + kCompactTile - 1) / kCompactTile);
  DevBuf cb, cbo;
  G5_HIP(hipMalloc(&cb.p, cblocks * sizeof(uint32_t)));
  G5_HIP(hipMalloc(&cbo.p, cblocks * sizeof(uint64_t)));
  hipLaunchKernelGGL(k_heads_count, dim3(cblocks), dim3(kCompactBlock), 0, s, keys, ntot, sent,
                     wb, (uint32_t *)cb.p);
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(kScanBlock), 0, s, (const uint32_t *)cb.p,
                     (uint64_t *)cbo.p, cblocks, nnz_dev);
  G5_LAUNCH_CHECK();
  uint64_t hv[2] = {0, 0};
  uint32_t herr = 0;
  G5_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
  G5_HIP(hipMemcpyAsync(hv, nnz_dev, 8, hipMemcpyDeviceToHost, s));
  G5_HIP(hipStreamSynchronize(s));
  if (herr & 1u) {
    set_error("g5_build_csr: an edge names a vertex outside [0, n)");
    return G5_EINVAL;
  }
  if (herr & 2u) {
    set_error("g5_build_csr: a radix sort pass did not see the counts of an earlier tile");
    return G5_EDEVICE;
  }
  const uint64_t nnz = hv[0];
  if (nnz >= (1ull << 32)) {
    set_error("g5_build_csr: nnz >= 2^32 is not supported");
    return G5_ERANGE;
  }
  // the sort buffer that is not the result is no longer needed
  if (alt == (uint64_t *)ka.p) {
    G5_HIP(hipFree(ka.p));
    ka.p = nullptr;
  } else {
    G5_HIP(hipFree(kb.p));
    kb.p = nullptr;
  }

  g5_csr *g = new g5_csr();
  g->n = n;
  g->nnz = (int64_t)nnz;
  g->sb = sb;
  g->device = dev;
  g->num_cu = ncu;
  g->words = (n + 63) / 64;
  g->tune = pick_tuning(sb);
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 0)
      g->lds_bytes = lds;
  }
  auto fail = [&](hipError_t e, const char *what) {
    set_error(std::string("g5_build_csr: ") + what + ": " + hipGetErrorString(e));
    g5_csr_free(g);
    return e == hipErrorOutOfMemory ? G5_ENOMEM : G5_EDEVICE;
  };
  hipError_t e;
  if ((e = hipMalloc(&g->row_ptr, (n + 1) * sizeof(int64_t))) != hipSuccess)
    return fail(e, "row_ptr");
  if ((e = hipMalloc(&g->col_idx, (nnz + kColPad) * sizeof(int32_t))) != hipSuccess)
    return fail(e, "col_idx");
  if ((e = hipMemsetAsync(g->col_idx + nnz, 0, kColPad * sizeof(int32_t), s)) != hipSuccess)
    return fail(e, "memset");
  if ((e = hipMalloc(&g->iso, g->words * sizeof(uint64_t))) != hipSuccess)
    return fail(e, "iso");
  if (weighted) {
    if ((e = hipMalloc(&g->wt, nnz + kColPad)) != hipSuccess) return fail(e, "weights");
    if ((e = hipMemsetAsync(g->wt + nnz, 0, kColPad, s)) != hipSuccess) return fail(e, "memset");
  }
  hipLaunchKernelGGL(k_compact, dim3(cblocks), dim3(kCompactBlock), 0, s, keys, ntot, sent, sb,
                     wb, n, (const uint64_t *)cbo.p, g->col_idx, g->row_ptr, g->wt);
  hipLaunchKernelGGL(k_iso, dim3(grid_cap(g->words, 4, ncu * 16)), dim3(256), 0, s, g->row_ptr,
                     n, g->words, g->iso, noniso_dev);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
  unsigned long long noniso = 0;
  if ((e = hipMemcpyAsync(&noniso, noniso_dev, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  g->nonisolated = (int64_t)noniso;
  if ((e = hipMalloc(&g->rp32, (n + 1) * sizeof(uint32_t))) != hipSuccess) return fail(e, "rp32");
  hipLaunchKernelGGL(k_rp32, dim3(grid_cap(n + 1, 256, ncu * 16)), dim3(256), 0, s, g->row_ptr,
                     n + 1, g->rp32);
  // hub list (order does not matter) and its chunk prefix
  const int64_t max_hubs = (int64_t)(nnz / kHubDeg) + 1;
  if ((e = hipMalloc(&g->hub_list, max_hubs * sizeof(int32_t))) != hipSuccess)
    return fail(e, "hub list");
  if ((e = hipMemsetAsync(noniso_dev, 0, 8, s)) != hipSuccess) return fail(e, "memset");
  hipLaunchKernelGGL(k_find_hubs, dim3(grid_cap(n, 256, ncu * 16)), dim3(256), 0, s, g->row_ptr,
                     n, g->hub_list, noniso_dev);
  unsigned long long nh = 0;
  if ((e = hipMemcpyAsync(&nh, noniso_dev, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  g->num_hubs = (int64_t)nh;
  std::vector<uint64_t> off(nh + 1, 0);
  if ((e = hipMalloc(&g->hub_off, (nh + 1) * sizeof(uint64_t))) != hipSuccess)
    return fail(e, "hub offsets");
  if (nh) {
    hipLaunchKernelGGL(k_hub_chunks, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s,
                       g->row_ptr, g->hub_list, (int64_t)nh, g->hub_off);
    if ((e = hipMemcpyAsync(off.data() + 1, g->hub_off, nh * 8, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return fail(e, "copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
    for (size_t i = 1; i <= nh; ++i) off[i] += off[i - 1];
  }
  g->hub_chunks = (int64_t)off[nh];
  if ((e = hipMemcpyAsync(g->hub_off, off.data(), (nh + 1) * 8, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return fail(e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  if ((e = hipMalloc(&g->hint, n * sizeof(int32_t))) != hipSuccess) return fail(e, "hint");
  if ((e = hipMalloc(&g->hint_id, n * sizeof(int32_t))) != hipSuccess) return fail(e, "hint");
  DevBuf cand;  // the hint candidates (hubs of largest key), kept for the hot count
  int kc = 0;
  {
    DevBuf d16, hkeys, best, key;
    if ((e = d16.alloc(n * sizeof(uint16_t))) != hipSuccess) return fail(e, "degrees");
    hipLaunchKernelGGL(k_deg16, dim3(grid_cap(n, 256, ncu * 16)), dim3(256), 0, s, g->row_ptr, n,
                       (uint16_t *)d16.p);
    // hint candidates: the hubs of largest key (every hub outranks every other
    // vertex), ordered on the host
    const int64_t nh = g->num_hubs;
    kc = (int)std::min<int64_t>(nh, kHintCand);
    if (nh > 0) {
      if ((e = hkeys.alloc(nh * sizeof(uint64_t))) != hipSuccess ||
          (e = cand.alloc(kc * sizeof(int32_t))) != hipSuccess ||
          (e = best.alloc(nh * sizeof(uint64_t))) != hipSuccess ||
          (e = key.alloc(nh * sizeof(uint64_t))) != hipSuccess)
        return fail(e, "hints");
      hipLaunchKernelGGL(k_hub_keys, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s,
                         g->row_ptr, g->hub_list, nh, (uint64_t *)hkeys.p);
      std::vector<uint64_t> hk(nh);
      if ((e = hipMemcpyAsync(hk.data(), hkeys.p, nh * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail(e, "copy");
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
      std::partial_sort(hk.begin(), hk.begin() + kc, hk.end(), std::greater<uint64_t>());
      std::vector<int32_t> ids(kc);
      for (int r = 0; r < kc; ++r) ids[r] = (int32_t)(0x7fffffffu - (uint32_t)(hk[r] & 0xffffffffu));
      if ((e = hipMemcpyAsync(cand.p, ids.data(), kc * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
          (e = hipMemsetAsync(best.p, 0xff, nh * 8, s)) != hipSuccess ||
          (e = hipMemsetAsync(key.p, 0, nh * 8, s)) != hipSuccess)
        return fail(e, "copy");
      // ids is read by the copy: keep it until the stream has taken it
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
    }
    hipLaunchKernelGGL(k_hint, dim3(grid_cap(g->words, kHintBlock / kWave, ncu * 4)),
                       dim3(kHintBlock), 0, s, g->row_ptr,
                       (const uint16_t *)d16.p, g->col_idx, n, g->words,
                       (const int32_t *)cand.p, kc, g->hint, g->hint_id);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
    if (nh > 0) {
      const dim3 grid(grid_cap(g->hub_chunks, kHintBlock / kWave, ncu * 4));
      hipLaunchKernelGGL(k_hint_hubs<true>, grid, dim3(kHintBlock), 0, s, g->row_ptr,
                         (const uint16_t *)d16.p, g->col_idx, g->hub_list,
                         (const uint64_t *)g->hub_off, nh, (const int32_t *)cand.p, kc,
                         (unsigned long long *)best.p, (unsigned long long *)key.p);
      hipLaunchKernelGGL(k_hint_hubs<false>, grid, dim3(kHintBlock), 0, s, g->row_ptr,
                         (const uint16_t *)d16.p, g->col_idx, g->hub_list,
                         (const uint64_t *)g->hub_off, nh, (const int32_t *)cand.p, kc,
                         (unsigned long long *)best.p, (unsigned long long *)key.p);
      hipLaunchKernelGGL(k_hint_hubs_write, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s,
                         g->hub_list, nh, (const unsigned long long *)best.p,
                         (const unsigned long long *)key.p, (const int32_t *)cand.p, g->hint,
                         g->hint_id);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
    }
    // the buffers of this scope are freed on return from it: the stream must
    // be done with them
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  }
  {
    // hot hint targets: the most-named ones, at most kHotMax, numbered in vertex order
    const int64_t nb = (n + kHotTile - 1) / kHotTile;
    DevBuf cnt, hist, bsum, boff;
    if ((e = cnt.alloc(n * 4)) != hipSuccess || (e = hist.alloc(kHotBins * 4)) != hipSuccess ||
        (e = bsum.alloc(nb * 4)) != hipSuccess || (e = boff.alloc(nb * 8)) != hipSuccess)
      return fail(e, "hot hints");
    if ((e = hipMemsetAsync(cnt.p, 0, n * 4, s)) != hipSuccess ||
        (e = hipMemsetAsync(hist.p, 0, kHotBins * 4, s)) != hipSuccess)
      return fail(e, "memset");
    hipLaunchKernelGGL(k_hint_count, dim3(grid_cap(n, 256, ncu * 8)), dim3(256), 0, s, g->hint,
                       n, (const int32_t *)cand.p, kc, (uint32_t *)cnt.p);
    hipLaunchKernelGGL(k_hint_hist, dim3(grid_cap(n, 256, ncu * 4)), dim3(256), 0, s,
                       (const uint32_t *)cnt.p, n, (uint32_t *)hist.p);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
    std::vector<uint32_t> hh(kHotBins);
    if ((e = hipMemcpyAsync(hh.data(), hist.p, kHotBins * 4, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return fail(e, "copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
    // at most kHotMax targets, and at most one per 16 vertices (a frontier bitmap
    // of a smaller graph stays in L2 by itself)
    const uint64_t cap = (uint64_t)std::min<int64_t>(kHotMax, std::max<int64_t>(64, n >> 4));
    uint64_t above = 0;
    uint32_t cmin = kHotBins;
    for (int c = kHotBins - 1; c >= 1; --c) {
      if (above + hh[c] > cap) break;
      above += hh[c];
      cmin = (uint32_t)c;
    }
    if (above > 0) {
      if ((e = hipMalloc(&g->hot, above * sizeof(int32_t))) != hipSuccess)
        return fail(e, "hot hints");
      hipLaunchKernelGGL(k_hot_count, dim3((unsigned)nb), dim3(256), 0, s,
                         (const uint32_t *)cnt.p, n, cmin, (uint32_t *)bsum.p);
      hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(kScanBlock), 0, s, (const uint32_t *)bsum.p,
                         (uint64_t *)boff.p, nb, (uint64_t *)nullptr);
      hipLaunchKernelGGL(k_hot_write, dim3((unsigned)nb), dim3(256), 0, s, (uint32_t *)cnt.p, n,
                         cmin, (const uint64_t *)boff.p, g->hot);
      hipLaunchKernelGGL(k_hint_encode, dim3(grid_cap(n, 256, ncu * 16)), dim3(256), 0, s,
                         g->hint, n, (const uint32_t *)cnt.p);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
      g->num_hot = (int64_t)above;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  }
  {
    // hints of the vertices of degree >= 1 only, by rank: the dense-frontier
    // bottom-up step then reads lines that hold no isolated vertex (half of
    // them at scale 26)
    const int64_t chunks = (g->words + kWave - 1) / kWave;
    DevBuf cnt;
    if ((e = cnt.alloc(chunks * 4)) != hipSuccess ||
        (e = hipMalloc(&g->chunk_ni, chunks * 8)) != hipSuccess ||
        (e = hipMalloc(&g->hint_c, std::max<int64_t>(1, g->nonisolated) * sizeof(int32_t))) !=
            hipSuccess)
      return fail(e, "compact hints");
    const int cgrid = grid_cap(chunks, 256 / kWave, ncu * 16);
    hipLaunchKernelGGL(k_chunk_count, dim3(cgrid), dim3(256), 0, s, g->iso, g->words, chunks,
                       (uint32_t *)cnt.p);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(kScanBlock), 0, s, (const uint32_t *)cnt.p,
                       g->chunk_ni, chunks, (uint64_t *)nullptr);
    hipLaunchKernelGGL(k_hint_compact, dim3(cgrid), dim3(256), 0, s, g->hint, g->iso, g->words,
                       chunks, (const uint64_t *)g->chunk_ni, g->hint_c);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e, "launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  }

  *out = g;
  return G5_OK;
}

}  // namespace g5
