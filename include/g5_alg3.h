/* Host experiment beside the GPU library: the paper's level-synchronous
 * parallel BFS (Algorithm 3, Section 2.3.2) with OpenMP threads, for a
 * speedup curve over thread counts.  Built as libg5alg3.so (gcc, OpenMP);
 * the GPU path never calls it. */
#ifndef G5_ALG3_H
#define G5_ALG3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* BFS from `root` over a CSR in host memory, with `threads` OpenMP threads.
 *   rp       host, int64 [n + 1]: row offsets (row v is ci[rp[v] .. rp[v + 1])).
 *   ci       host, int32 [rp[n]]: neighbour ids in [0, n).
 *   level    host, int32 [n], written: hop distance from root, -1 if unreached.
 *   parent   host, int32 [n], written: a neighbour one level closer (the
 *            claiming frontier vertex), root for root, -1 if unreached.
 *   seconds  optional (NULL to skip): wall time of the traversal, including
 *            the initialisation of level and parent.
 * All buffers are borrowed for the call.  Returns 0; -1 on a NULL pointer,
 * n <= 0, root outside [0, n) or threads < 1; -2 if the two frontier arrays
 * (int32 [n] each) cannot be allocated. */
int g5_alg3_bfs(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root, int32_t *level,
                int32_t *parent, int threads, double *seconds);

#ifdef __cplusplus
}
#endif

#endif
