// Batched multi-source BFS (placeholder until the persistent kernel lands).
#include "g5_internal.h"

namespace g5 {
BatchWork::~BatchWork() {
  if (seen) (void)hipFree(seen);
  if (front) (void)hipFree(front);
  if (next) (void)hipFree(next);
  if (sync) (void)hipFree(sync);
  if (host_ctr) (void)hipHostFree(host_ctr);
}

g5_status bfs_batch_impl(const g5_csr *, const int64_t *, int, int32_t *, int8_t *, hipStream_t) {
  set_error("g5_bfs_batch: not available in this build");
  return G5_EINVAL;
}
}  // namespace g5
