// C-ABI entry points of libg5 (declared in include/g5.h): argument checks,
// error state and dispatch to the device implementations.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "g5_internal.h"

namespace g5 {
namespace {
thread_local std::string t_err;
const Tuning kTuned[] = {
#include "tuned_table.inc"
};
}  // namespace
void set_error(const std::string &msg) { t_err = msg; }

Tuning pick_tuning(int scale) {
  const Tuning *best = &kTuned[0];
  for (const Tuning &t : kTuned)
    if (std::abs(t.scale - scale) < std::abs(best->scale - scale)) best = &t;
  return *best;
}
}  // namespace g5

using g5::set_error;

extern "C" {

const char *g5_last_error(void) { return g5::t_err.c_str(); }

g5_status g5_build_csr(const int64_t *edges, int64_t m, int64_t n_vertices, void *stream,
                       g5_csr **out) {
  if (!out) {
    set_error("g5_build_csr: out is NULL");
    return G5_EINVAL;
  }
  *out = nullptr;
  try {
    return g5::build_csr_impl(edges, nullptr, false, m, n_vertices, (hipStream_t)stream, out);
  } catch (const std::bad_alloc &) {
    set_error("g5_build_csr: host allocation failed");
    return G5_ENOMEM;
  }
}

g5_status g5_build_csr_w(const int64_t *edges, const uint8_t *weights, int64_t m,
                         int64_t n_vertices, void *stream, g5_csr **out) {
  if (!out) {
    set_error("g5_build_csr_w: out is NULL");
    return G5_EINVAL;
  }
  *out = nullptr;
  try {
    return g5::build_csr_impl(edges, weights, true, m, n_vertices, (hipStream_t)stream, out);
  } catch (const std::bad_alloc &) {
    set_error("g5_build_csr_w: host allocation failed");
    return G5_ENOMEM;
  }
}

g5_status g5_csr_copy_weights(const g5_csr *g, uint8_t *weights, void *stream) {
  if (!g || !weights) {
    set_error("g5_csr_copy_weights: graph and weights must be non-NULL");
    return G5_EINVAL;
  }
  if (!g->wt) {
    set_error("g5_csr_copy_weights: the graph has no weights (built by g5_build_csr)");
    return G5_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (g->nnz) G5_HIP(hipMemcpyAsync(weights, g->wt, g->nnz, hipMemcpyDefault, s));
  G5_HIP(hipStreamSynchronize(s));
  return G5_OK;
}

g5_status g5_csr_info(const g5_csr *g, int64_t *n, int64_t *nnz, const int64_t **row_ptr,
                      const int32_t **col_idx) {
  if (!g) {
    set_error("g5_csr_info: graph is NULL");
    return G5_EINVAL;
  }
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (row_ptr) *row_ptr = g->row_ptr;
  if (col_idx) *col_idx = g->col_idx;
  return G5_OK;
}

g5_status g5_csr_copy(const g5_csr *g, int64_t *row_ptr, int32_t *col_idx, void *stream) {
  if (!g) {
    set_error("g5_csr_copy: graph is NULL");
    return G5_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (row_ptr)
    G5_HIP(hipMemcpyAsync(row_ptr, g->row_ptr, (g->n + 1) * sizeof(int64_t), hipMemcpyDefault, s));
  if (col_idx && g->nnz)
    G5_HIP(hipMemcpyAsync(col_idx, g->col_idx, g->nnz * sizeof(int32_t), hipMemcpyDefault, s));
  G5_HIP(hipStreamSynchronize(s));
  return G5_OK;
}

void g5_csr_free(g5_csr *g) {
  if (!g) return;
  for (auto *w : g->bfs_pool) delete w;
  for (auto *w : g->batch_pool) delete w;
  for (auto *w : g->sssp_pool) delete w;
  if (g->row_ptr) (void)hipFree(g->row_ptr);
  if (g->col_idx) (void)hipFree(g->col_idx);
  if (g->wt) (void)hipFree(g->wt);
  if (g->iso) (void)hipFree(g->iso);
  if (g->hint) (void)hipFree(g->hint);
  if (g->hot) (void)hipFree(g->hot);
  if (g->hint_id) (void)hipFree(g->hint_id);
  if (g->hint_c) (void)hipFree(g->hint_c);
  if (g->chunk_ni) (void)hipFree(g->chunk_ni);
  if (g->rp32) (void)hipFree(g->rp32);
  if (g->hub_list) (void)hipFree(g->hub_list);
  if (g->hub_off) (void)hipFree(g->hub_off);
  delete g;
}

g5_status g5_bfs_ex(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level,
                    void *stream, const g5_bfs_params *params, g5_bfs_stats *stats) {
  if (!g || !parent || !level) {
    set_error("g5_bfs: graph, parent and level must be non-NULL");
    return G5_EINVAL;
  }
  if (root < 0 || root >= g->n) {
    set_error("g5_bfs: root " + std::to_string(root) + " outside [0, " + std::to_string(g->n) +
              ")");
    return G5_EINVAL;
  }
  g5_bfs_params p;
  std::memset(&p, 0, sizeof(p));
  if (params) p = *params;
  if (p.direction < 0 || p.direction > 2 || p.claim < 0 || p.claim > 1 || p.bu_lane_scan < 0 ||
      p.bu_lane_scan > 16 || (p.bu_lane_scan & (p.bu_lane_scan - 1)) != 0 || p.alpha < 0 ||
      p.beta < 0 || p.lds_density < 0 || p.bu_blocks_per_cu < 0 || p.bu_blocks_per_cu > 32 ||
      (p.lds_kb != 0 && (p.lds_kb < 16 || p.lds_kb > 160)) ||
      (p.bu_vertices_per_lane != 0 && p.bu_vertices_per_lane != 1 &&
       p.bu_vertices_per_lane != 2) ||
      p.td_blocks_per_cu < 0 || p.td_blocks_per_cu > 256) {
    set_error("g5_bfs: direction must be 0..2, claim 0..1, bu_lane_scan 0 or a power of two "
              "up to 16, alpha, beta, lds_density >= 0, bu_blocks_per_cu 0..32, lds_kb 0 or "
              "16..160, bu_vertices_per_lane 0, 1 or 2, td_blocks_per_cu 0..256");
    return G5_EINVAL;
  }
  try {
    return g5::bfs_impl(g, root, parent, level, (hipStream_t)stream, p, stats);
  } catch (const std::bad_alloc &) {
    set_error("g5_bfs: host allocation failed");
    return G5_ENOMEM;
  }
}

g5_status g5_bfs(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level, void *stream) {
  return g5_bfs_ex(g, root, parent, level, stream, nullptr, nullptr);
}

g5_status g5_bfs_batch_ex(const g5_csr *g, const int64_t *roots, int32_t k, int32_t *parents,
                          int8_t *levels, void *stream, const g5_batch_params *params,
                          g5_batch_stats *stats) {
  if (!g || !roots || !levels) {
    set_error("g5_bfs_batch: graph, roots and levels must be non-NULL");
    return G5_EINVAL;
  }
  if (k < 1 || k > 64) {
    set_error("g5_bfs_batch: k must be in [1, 64]");
    return G5_EINVAL;
  }
  for (int i = 0; i < k; ++i)
    if (roots[i] < 0 || roots[i] >= g->n) {
      set_error("g5_bfs_batch: root " + std::to_string(roots[i]) + " outside [0, n)");
      return G5_EINVAL;
    }
  g5_batch_params p;
  std::memset(&p, 0, sizeof(p));
  if (params) p = *params;
  if (p.direction < 0 || p.direction > 2 || p.alpha < 0 || p.blocks_per_cu < 0 ||
      p.blocks_per_cu > 32) {
    set_error("g5_bfs_batch: direction must be 0..2, alpha >= 0, blocks_per_cu 0..32");
    return G5_EINVAL;
  }
  try {
    return g5::bfs_batch_impl(g, roots, k, parents, levels, (hipStream_t)stream, p, stats);
  } catch (const std::bad_alloc &) {
    set_error("g5_bfs_batch: host allocation failed");
    return G5_ENOMEM;
  }
}

g5_status g5_bfs_batch(const g5_csr *g, const int64_t *roots, int32_t k, int32_t *parents,
                       int8_t *levels, void *stream) {
  return g5_bfs_batch_ex(g, roots, k, parents, levels, stream, nullptr, nullptr);
}

g5_status g5_bfs_batch_noalloc(const g5_csr *g, const int64_t *roots, int32_t k,
                               int32_t *parents, int8_t *levels, void *stream) {
  if (!g || !roots || !levels) {
    set_error("g5_bfs_batch_noalloc: graph, roots and levels must be non-NULL");
    return G5_EINVAL;
  }
  if (k < 1 || k > 64) {
    set_error("g5_bfs_batch_noalloc: k must be in [1, 64]");
    return G5_EINVAL;
  }
  for (int i = 0; i < k; ++i)
    if (roots[i] < 0 || roots[i] >= g->n) {
      set_error("g5_bfs_batch_noalloc: root " + std::to_string(roots[i]) + " outside [0, n)");
      return G5_EINVAL;
    }
  return g5::bfs_batch_noalloc_impl(g, roots, k, parents, levels, (hipStream_t)stream);
}

g5_status g5_sssp_ex(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, void *stream,
                     const g5_sssp_params *params, g5_sssp_stats *stats) {
  if (!g || !dist || !prev) {
    set_error("g5_sssp: graph, dist and prev must be non-NULL");
    return G5_EINVAL;
  }
  if (src < 0 || src >= g->n) {
    set_error("g5_sssp: source " + std::to_string(src) + " outside [0, " + std::to_string(g->n) +
              ")");
    return G5_EINVAL;
  }
  g5_sssp_params p;
  std::memset(&p, 0, sizeof(p));
  if (params) p = *params;
  try {
    return g5::sssp_impl(g, src, dist, prev, (hipStream_t)stream, p, stats);
  } catch (const std::bad_alloc &) {
    set_error("g5_sssp: host allocation failed");
    return G5_ENOMEM;
  }
}

g5_status g5_sssp(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, void *stream) {
  return g5_sssp_ex(g, src, dist, prev, stream, nullptr, nullptr);
}

g5_status g5_level_work(const g5_csr *g, const int32_t *level, int32_t lvl, int32_t bottom_up,
                        int64_t *out, void *stream) {
  if (!g || !level || !out) {
    set_error("g5_level_work: graph, level and out must be non-NULL");
    return G5_EINVAL;
  }
  if (lvl < 0) {
    set_error("g5_level_work: lvl must be >= 0");
    return G5_EINVAL;
  }
  return g5::level_work_impl(g, level, lvl, bottom_up != 0, out, (hipStream_t)stream);
}

}  // extern "C"
