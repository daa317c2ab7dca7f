/* Host build of the seeded Kronecker input generator (definition in
 * kron_core.h).  OpenMP across tuples; every tuple is a pure function of
 * (scale, seed, index), so the output does not depend on the thread count. */
#include <stdint.h>
#include <string.h>

#include "kron_core.h"

/* Writes tuples [i0, i1) of the list for (scale, seed) into out[2*(i-i0)],
 * out[2*(i-i0)+1] as (start, end).  relabel = 0 skips the vertex permutation
 * (used only to test the quadrant statistics).  Returns 0, or -1 on a bad
 * scale. */
int kron_edges_host(int scale, uint64_t seed, int relabel, int64_t i0,
                    int64_t i1, int64_t *out) {
  if (scale < 1 || scale > KRON_MAX_SCALE || i0 < 0 || i1 < i0) return -1;
  kron_params p = kron_make_params(scale, seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = i0; i < i1; ++i) {
    uint64_t r, c;
    kron_raw_tuple(&p, (uint64_t)i, &r, &c);
    if (relabel) {
      r = kron_relabel(&p, r);
      c = kron_relabel(&p, c);
    }
    out[2 * (i - i0)] = (int64_t)r;
    out[2 * (i - i0) + 1] = (int64_t)c;
  }
  return 0;
}

/* Applies the relabel bijection of (scale, seed) to x[0..len). */
int kron_relabel_host(int scale, uint64_t seed, const int64_t *x, int64_t len,
                      int64_t *out) {
  if (scale < 1 || scale > KRON_MAX_SCALE) return -1;
  kron_params p = kron_make_params(scale, seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < len; ++i) out[i] = (int64_t)kron_relabel(&p, (uint64_t)x[i]);
  return 0;
}

/* mask[v] = 1 if v is an endpoint of some tuple (u, w) with u != w, else 0.
 * These are the vertices of degree >= 1 once self-loops are ignored; root
 * selection draws from them.  Returns -1 if an id is outside [0, n). */
int kron_nonisolated_host(const int64_t *edges, int64_t m, int64_t n,
                          uint8_t *mask) {
  int bad = 0;
  memset(mask, 0, (size_t)n);
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], w = edges[2 * i + 1];
    if (u < 0 || u >= n || w < 0 || w >= n) {
      bad = 1;
      continue;
    }
    if (u == w) continue;
    __atomic_store_n(&mask[u], (uint8_t)1, __ATOMIC_RELAXED);
    __atomic_store_n(&mask[w], (uint8_t)1, __ATOMIC_RELAXED);
  }
  return bad ? -1 : 0;
}

/* Weights of tuples [i0, i1) of (seed): out[i - i0] in [1, 255]. */
int kron_weights_host(uint64_t seed, int64_t i0, int64_t i1, uint8_t *out) {
  if (i0 < 0 || i1 < i0) return -1;
  const uint64_t base = kron_weight_base(seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = i0; i < i1; ++i) out[i - i0] = kron_weight(base, (uint64_t)i);
  return 0;
}

uint64_t kron_splitmix64_at(uint64_t state, uint64_t c) { return splitmix64_at(state, c); }
