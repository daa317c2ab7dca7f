/* Counter-based Kronecker edge generator: the definition shared by the host
 * (kron_host.c) and device (kron_dev.hip) builds of the seeded input generator.
 *
 * This file holds input generation only.  It contains no part of graph
 * construction or traversal.
 *
 * Data set (Section 2.1 of the paper): #V = 2^scale vertices and
 * #E = #V * edgefactor generated tuples (start, end).  Multi-edges, self-loops
 * and isolated vertices stay in the list; vertex numbers are randomly
 * permuted.  The paper defers the exact generator to the Graph500
 * specification, which is not reproduced here.  This generator follows the
 * recursive-quadrant (R-MAT / Kronecker) construction with initiator
 * probabilities (A, B, C, D) = (0.57, 0.19, 0.19, 0.05) and no per-level
 * noise:
 *
 *   for tuple i and level k = 0 .. scale-1 (most significant bit first) a
 *   32-bit uniform draw r(i, k) picks a quadrant:
 *       r <  TA            -> A: neither bit
 *       TA   <= r < TAB    -> B: column bit (end vertex)
 *       TAB  <= r < TABC   -> C: row bit (start vertex)
 *       TABC <= r          -> D: both bits
 *   where TA = floor(0.57 * 2^32), TAB = floor(0.76 * 2^32),
 *   TABC = floor(0.95 * 2^32).
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  splitmix64_at(s, c) is the
 * c-th output (c = 0, 1, ...) of a SplitMix64 generator whose state starts at
 * s: mix(s + (c + 1) * gamma).  Draw r(i, k) is the low (k even) or high
 * (k odd) 32-bit half of splitmix64_at(edge_base, 32 * i + k / 2), where
 * edge_base = splitmix64_at(seed, 0).
 *
 * Relabel: a seeded bijection of [0, 2^scale) built from three rounds of
 * (multiply by an odd constant, add a constant, mod 2^scale) followed by
 * x ^= x >> h with h = ceil(scale / 2).  Each step is invertible on
 * scale-bit integers, so the composition is a permutation.  Its six constants
 * are splitmix64_at(perm_base, 0 .. 5) with perm_base = splitmix64_at(seed, 1)
 * (multipliers forced odd).
 *
 * Weights (the third row of the paper's 3 x #E tuple matrix, Section 2.1):
 * tuple i carries the integer weight 1 + (splitmix64_at(weight_base, i) mod
 * 255), in [1, 255], with weight_base = splitmix64_at(seed, 3).
 */
#ifndef KRON_CORE_H
#define KRON_CORE_H

#include <stdint.h>

#ifdef __HIPCC__
#define KRON_FN static inline __host__ __device__
#else
#define KRON_FN static inline
#endif

#define KRON_GAMMA 0x9E3779B97F4A7C15ULL
#define KRON_TA   2448131358U  /* floor(0.57 * 2^32) */
#define KRON_TAB  3264175144U  /* floor(0.76 * 2^32) */
#define KRON_TABC 4080218931U  /* floor(0.95 * 2^32) */
#define KRON_MAX_SCALE 31

KRON_FN uint64_t kron_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

KRON_FN uint64_t splitmix64_at(uint64_t state, uint64_t c) {
  return kron_mix64(state + (c + 1) * KRON_GAMMA);
}

typedef struct {
  int scale;
  uint64_t edge_base;
  uint64_t mask;
  int h;
  uint64_t k[6];
} kron_params;

KRON_FN kron_params kron_make_params(int scale, uint64_t seed) {
  kron_params p;
  p.scale = scale;
  p.edge_base = splitmix64_at(seed, 0);
  p.mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1ULL);
  p.h = (scale + 1) / 2;
  if (p.h < 1) p.h = 1;
  uint64_t pb = splitmix64_at(seed, 1);
  for (int j = 0; j < 6; ++j) p.k[j] = splitmix64_at(pb, (uint64_t)j);
  p.k[0] |= 1ULL;
  p.k[2] |= 1ULL;
  p.k[4] |= 1ULL;
  return p;
}

KRON_FN uint64_t kron_relabel(const kron_params *p, uint64_t x) {
  for (int r = 0; r < 3; ++r) {
    x = (x * p->k[2 * r] + p->k[2 * r + 1]) & p->mask;
    x ^= x >> p->h;
  }
  return x;
}

/* Tuple i before relabelling: (row, col) from scale quadrant draws. */
KRON_FN void kron_raw_tuple(const kron_params *p, uint64_t i, uint64_t *row,
                            uint64_t *col) {
  uint64_t r0 = 0, c0 = 0, w = 0;
  for (int k = 0; k < p->scale; ++k) {
    if ((k & 1) == 0) w = splitmix64_at(p->edge_base, 32ULL * i + (uint64_t)(k >> 1));
    uint32_t r = (k & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
    uint64_t bit = 1ULL << (p->scale - 1 - k);
    if (r >= KRON_TABC) {
      r0 |= bit;
      c0 |= bit;
    } else if (r >= KRON_TAB) {
      r0 |= bit;
    } else if (r >= KRON_TA) {
      c0 |= bit;
    }
  }
  *row = r0;
  *col = c0;
}

/* Weight of tuple i (see above). */
KRON_FN uint8_t kron_weight(uint64_t weight_base, uint64_t i) {
  return (uint8_t)(1 + splitmix64_at(weight_base, i) % 255);
}

KRON_FN uint64_t kron_weight_base(uint64_t seed) { return splitmix64_at(seed, 3); }

#endif
