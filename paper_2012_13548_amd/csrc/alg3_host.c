/* Host experiment: the paper's level-synchronous parallel BFS (Algorithm 3,
 * Section 2.3.2) with OpenMP threads, to measure its speedup over thread
 * counts on the host.  It is not part of the GPU path and nothing calls it as
 * a fallback: g5_alg3_bfs is its own entry point.
 *
 * Each level is one parallel loop over the frontier (dynamic schedule, so hub
 * rows do not stall a static share); a neighbour not reached yet is claimed by
 * a compare-and-swap of its level from -1 to l + 1, which makes the paper's
 * check-then-set race-free (each vertex joins the next frontier once); the
 * winner records the parent.  Appends go through a per-thread buffer flushed
 * with one atomic add. */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#include "g5_alg3.h"

enum { kBuf = 1024 };

int g5_alg3_bfs(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root, int32_t *level,
                int32_t *parent, int threads, double *seconds) {
  if (!rp || !ci || !level || !parent || n <= 0 || root < 0 || root >= n || threads < 1)
    return -1;
  int32_t *cur = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *nxt = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!cur || !nxt) {
    free(cur);
    free(nxt);
    return -2;
  }
  const double t0 = omp_get_wtime();
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    level[v] = -1;
    parent[v] = -1;
  }
  level[root] = 0;
  parent[root] = (int32_t)root;
  cur[0] = (int32_t)root;
  int64_t ncur = 1;
  for (int32_t l = 0; ncur > 0; ++l) {
    int64_t nnext = 0;
#pragma omp parallel num_threads(threads)
    {
      int32_t buf[kBuf];
      int nb = 0;
#pragma omp for schedule(dynamic, 64)
      for (int64_t i = 0; i < ncur; ++i) {
        const int32_t u = cur[i];
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
          const int32_t v = ci[e];
          int32_t expect = -1;
          if (__atomic_load_n(&level[v], __ATOMIC_RELAXED) == -1 &&
              __atomic_compare_exchange_n(&level[v], &expect, l + 1, 0, __ATOMIC_RELAXED,
                                          __ATOMIC_RELAXED)) {
            parent[v] = u;
            buf[nb++] = v;
            if (nb == kBuf) {
              const int64_t at = __atomic_fetch_add(&nnext, (int64_t)nb, __ATOMIC_RELAXED);
              for (int j = 0; j < nb; ++j) nxt[at + j] = buf[j];
              nb = 0;
            }
          }
        }
      }
      if (nb) {
        const int64_t at = __atomic_fetch_add(&nnext, (int64_t)nb, __ATOMIC_RELAXED);
        for (int j = 0; j < nb; ++j) nxt[at + j] = buf[j];
      }
    }
    int32_t *t = cur;
    cur = nxt;
    nxt = t;
    ncur = nnext;
  }
  if (seconds) *seconds = omp_get_wtime() - t0;
  free(cur);
  free(nxt);
  return 0;
}
