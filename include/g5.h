/*
 * g5 -- breadth-first search over an undirected Kronecker graph stored as CSR,
 * on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the pipeline of the paper "Graph500 from OCaml-Multicore
 * Perspective" (algorithm "Basic Outline of Graph500"): Kernel 1 constructs a
 * graph from the generated edge list (Section 2.2, CSR format), Kernel 2
 * computes the parent array and BFS tree from a root (Section 2.3), and the
 * metric is taken over 64 start vertices (Section 4.3).
 *
 * Conventions shared by every call
 *   - Device pointers are HIP device memory of the current device; host
 *     pointers are ordinary host memory.  Each argument below says which.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     Every call returns after its work on `stream` has completed.
 *   - Status codes are negative on failure (g5_status).  On failure no output
 *     contents are promised; g5_last_error() describes the failure.
 *   - Vertex ids are 0 .. n-1 with n <= 2^31 - 1.  Levels and parents use -1
 *     for "not reached"; parent[root] = root.
 *   - Calls on the same g5_csr from several host threads are allowed; each
 *     BFS call takes a private workspace from a pool owned by the g5_csr.
 */
#ifndef G5_H
#define G5_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct g5_csr g5_csr; /* opaque, device-resident, owned by the library */

typedef enum {
  G5_OK = 0,
  G5_EINVAL = -1,  /* bad argument: NULL pointer, id or root outside [0, n), k outside [1, 64] */
  G5_ENOMEM = -2,  /* a device or pinned-host allocation failed */
  G5_EDEVICE = -3, /* a HIP runtime error */
  G5_ERANGE = -4   /* a result does not fit its type (batched level > 127, nnz >= 2^32) */
} g5_status;

/* Kernel 1 (Section 2.2): builds the undirected CSR of an edge list.
 *   edges       device, int64 [m][2] tuples (start, end), borrowed for the call.
 *   m           number of tuples (>= 0).
 *   n_vertices  number of vertices n (1 .. 2^31-1); every id must lie in [0, n).
 *   out         host, receives the new graph; *out = NULL on any error.
 * Each non-loop tuple (u, v) gives both u->v and v->u (the graph is
 * undirected, Section 2); self-loops and repeated edges are dropped (they may
 * be ignored by the kernels, Section 2.1).  Row v lists v's distinct
 * neighbours in ascending order; row_ptr has n+1 entries, an empty row repeats
 * the previous index and row_ptr[n] = nnz (the CSR description of Section 2.2).
 * Errors: G5_EINVAL (id outside [0, n), m < 0, n out of range, NULL pointer),
 * G5_ERANGE (nnz >= 2^32), G5_ENOMEM, G5_EDEVICE. */
g5_status g5_build_csr(const int64_t *edges, int64_t m, int64_t n_vertices, void *stream,
                       g5_csr **out);

/* Sizes and borrowed device pointers of a graph built by g5_build_csr:
 * row_ptr int64 [n+1], col_idx int32 [nnz].  Any output pointer may be NULL.
 * The pointers stay valid until g5_csr_free. */
g5_status g5_csr_info(const g5_csr *g, int64_t *n, int64_t *nnz, const int64_t **row_ptr,
                      const int32_t **col_idx);

/* Kernel 1 for Kernel 3 (Sections 2.1, 2.2 and 2.4): the undirected CSR of
 * a weighted tuple list (the generator's 3 x #E matrix of start, end and
 * weight).  As g5_build_csr, plus
 *   weights  device, uint8 [m]: the integer weight (0..255) of each tuple,
 *            borrowed for the call (may be NULL only when m = 0).
 * Every non-loop tuple gives both directions with its weight; of repeated
 * tuples joining the same two vertices the CSR keeps the smallest weight
 * (the only one a shortest path can use).  Weights are stored beside col_idx
 * (g5_csr_copy_weights).  Needs n <= 2^28 (a sort key holds two vertex ids
 * and the weight).  The graph also serves g5_bfs.  Errors as g5_build_csr. */
g5_status g5_build_csr_w(const int64_t *edges, const uint8_t *weights, int64_t m,
                         int64_t n_vertices, void *stream, g5_csr **out);

/* Copies the weights of a graph built by g5_build_csr_w (uint8 [nnz], aligned
 * with col_idx) into a caller buffer (device or host memory).  G5_EINVAL if
 * the graph has no weights. */
g5_status g5_csr_copy_weights(const g5_csr *g, uint8_t *weights, void *stream);

/* Copies the CSR arrays into caller buffers (device or host memory):
 * row_ptr int64 [n+1], col_idx int32 [nnz]; either may be NULL. */
g5_status g5_csr_copy(const g5_csr *g, int64_t *row_ptr, int32_t *col_idx, void *stream);

/* Frees a graph and every workspace it owns.  NULL-safe. */
void g5_csr_free(g5_csr *g);

/* Kernel 2 (Section 2.3): breadth-first search from `root`.
 *   parent, level  device, int32 [n], written in full (caller-owned).
 * level[v] is the hop distance from root to v, or -1 if v is not in root's
 * component.  parent[root] = root; for another reached v, parent[v] is a
 * neighbour of v at level[v] - 1 (which one is not specified); -1 if
 * unreached.  The traversal is level-synchronous (Section 2.3.2) and
 * direction-optimising (top-down steps on small frontiers, bottom-up steps on
 * large ones).  A root of degree 0 is valid: only the root is reached.
 * Errors: G5_EINVAL (root outside [0, n), NULL pointer), G5_ENOMEM,
 * G5_EDEVICE. */
g5_status g5_bfs(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level, void *stream);

/* Direction policy of one traversal. */
typedef enum {
  G5_DIR_AUTO = 0,     /* direction-optimising switch on alpha / beta */
  G5_DIR_TOPDOWN = 1,  /* every level top-down */
  G5_DIR_BOTTOMUP = 2  /* every level after the root's bottom-up */
} g5_direction;

/* Tuning knobs of g5_bfs_ex.  Zero fields take the defaults that g5_build_csr
 * picked for the graph from the autotuned table compiled into the library
 * (the entry tuned at the scale nearest to log2 n). */
typedef struct {
  int32_t direction;      /* g5_direction */
  int32_t bu_lane_scan;   /* neighbours a lane tests before its row goes wave-wide: 1, 2, 4, 8
                             or 16 (steps with the frontier staged in LDS use at most 4) */
  double alpha;           /* top-down -> bottom-up when m_f > m_u / alpha and the frontier grew */
  double beta;            /* bottom-up -> top-down when n_f < n / beta and the frontier shrank */
  double lds_density;     /* bottom-up steps stage the frontier (or a summary of it) in LDS when
                             the fraction of summary bits set is expected below this */
  int32_t claim;          /* top-down claim: 0 atomic OR on the visited bitmap, 1 compare-and-swap
                             of parent from -1 */
  int32_t flags;          /* G5_FLAG_* */
  int32_t bu_blocks_per_cu; /* bottom-up grid: workgroups per compute unit (1..32) */
  int32_t lds_kb;         /* LDS for the staged frontier per workgroup, KiB (16..160) */
  int32_t bu_vertices_per_lane; /* bottom-up: unvisited vertices a lane works on at once: 1 or 2 */
  int32_t td_blocks_per_cu; /* top-down expansion grid: workgroups per compute unit (1..256);
                               0 = those that fit at once, at most 6 */
  int32_t heavy_kedges;   /* a growing top-down level whose frontier has more than this many
                             thousand edges claims without reading the claimed vertices' row
                             offsets or writing its queue (only the count), and the next level
                             goes bottom-up; 0 takes the default (nnz / 2048 edges), < 0
                             disables.  Only with G5_DIR_AUTO. */
  int32_t reserved;
  double gamma;           /* also top-down -> bottom-up when the frontier grew and m_f > gamma *
                             (unvisited non-isolated vertices); 0 takes the default, < 0 disables */
} g5_bfs_params;

/* Time each level's step kernel (the top-down expansion or the bottom-up step)
 * with HIP start/stop events carried by that kernel's own dispatch on `stream`
 * (step_ms in the stats); no extra packets are queued between kernels. */
#define G5_FLAG_TIME_STEPS 1
/* Count the algorithmic bytes and edges of each level (slower kernels; use in
 * an untimed run).  Levels are written as bytes during the traversal while they
 * fit (levels 0..254) and widened into `level` once at the end; past level 254
 * they are written as int32.  Bytes per level:
 *   top-down   12 per frontier vertex (queue entry, its edge-index word, its
 *              row start) + 4 per frontier edge + 21 per discovered vertex
 *              (byte level, parent, queue entry, its edge index and its two row
 *              offsets; 24 past level 254);
 *   bottom-up  4 per unvisited non-isolated vertex (its neighbour hint) + 4 per
 *              vertex whose hint missed (its 32-bit row offset) + 4 per row
 *              entry read up to the first frontier hit + n/4 (visited words
 *              read, next-frontier words written) + 1 per discovered vertex
 *              (byte level; 4 past level 254) + 4 per parent written (a hint
 *              hit writes none when the parent array was pre-filled with the
 *              hint targets).
 * Frontier-bitmap probes (one per examined neighbour) and the final widening
 * pass are not counted. */
#define G5_FLAG_COUNT_BYTES 2
/* Do not test each vertex's highest-degree neighbour (built by g5_build_csr)
 * before its row in bottom-up steps. */
#define G5_FLAG_NO_HINT 4
/* g5_bfs_batch_ex: one plain launch per level (the default; the flag is kept
 * for callers that set it).  Stepped batches can overlap other work on other
 * streams, and on MI355X they are also faster than the persistent launch. */
#define G5_FLAG_STEPPED 8
/* g5_bfs_ex: bottom-up rows left unresolved by a lane's own scan are packed end
 * to end across the wavefront (one entry per lane) instead of being scanned
 * one row per 64-lane step. */
#define G5_FLAG_PACKED 16
/* g5_bfs_ex: deterministic parents.  parent[v] is the smallest-id neighbour of
 * v at level[v] - 1 (top-down steps take an atomic minimum over every frontier
 * edge into v; bottom-up steps take the first frontier hit of the ascending
 * row, without the neighbour hint).  Slower; results do not depend on timing. */
#define G5_FLAG_MIN_PARENT 32
/* g5_bfs_ex: bottom-up steps always probe the frontier bitmap in HBM instead of
 * staging it (or, when it does not fit, a summary of it) in LDS. */
#define G5_FLAG_NO_LDS 64
/* g5_bfs_ex: bottom-up steps scan unresolved rows one row per 64-lane step
 * even where the tuned defaults pack them (G5_FLAG_PACKED forces packing). */
#define G5_FLAG_ROWLOOP 128
/* g5_bfs_batch_ex: every level in one cooperative persistent launch with a
 * grid barrier per level (same results).  It waits at the barriers for all of
 * its workgroups, so it should own the device. */
#define G5_FLAG_PERSISTENT 512
/* g5_bfs_batch_ex: the level loop runs as replays of one instantiated HIP
 * graph of 8 level kernels (each takes the level's direction decision on the
 * device and does nothing past the end), built once per workspace from kernel
 * nodes only; the host reads the level counters after each replay.  Same
 * results. */
#define G5_FLAG_GRAPH 1024

#define G5_MAX_STAT_LEVELS 64

/* Per-traversal statistics of g5_bfs_ex (host memory, filled on success); the
 * per-level arrays cover the first G5_MAX_STAT_LEVELS levels. */
typedef struct {
  int32_t nlevels;                          /* levels processed, root level included */
  int32_t dir[G5_MAX_STAT_LEVELS];          /* 1 top-down, 2 bottom-up */
  int64_t frontier[G5_MAX_STAT_LEVELS];     /* vertices in the frontier the level expands */
  int64_t discovered[G5_MAX_STAT_LEVELS];   /* vertices the level discovers */
  int64_t edges[G5_MAX_STAT_LEVELS];        /* top-down: frontier degree sum; bottom-up:
                                               neighbours examined (COUNT_BYTES only) */
  int64_t bytes[G5_MAX_STAT_LEVELS];        /* algorithmic bytes (COUNT_BYTES only) */
  double step_ms[G5_MAX_STAT_LEVELS];       /* device time of the step (TIME_STEPS only) */
  int64_t reached;                          /* vertices with level >= 0 */
  double alpha, beta;                       /* switch thresholds used */
  int32_t bu_lane_scan, bu_blocks_per_cu;   /* bottom-up shape used */
  int32_t lds_levels;                       /* bottom-up levels that staged the frontier in LDS */
  int32_t lds_shift;                        /* log2 vertices per staged bit (0: exact bitmap) */
  int64_t lds_mask;                         /* bit i (i < 64): level i's bottom-up step staged the
                                               frontier in LDS */
  int64_t heavy_mask;                       /* bit i (i < 64): level i was a heavy top-down level */
  int64_t reserved[3];
} g5_bfs_stats;

/* g5_bfs with explicit parameters (NULL = defaults) and optional statistics
 * (NULL = none).  Same results and errors as g5_bfs. */
g5_status g5_bfs_ex(const g5_csr *g, int64_t root, int32_t *parent, int32_t *level,
                    void *stream, const g5_bfs_params *params, g5_bfs_stats *stats);

/* Batched BFS from k roots (multi-source BFS: each vertex carries a 64-bit
 * mask whose bit b stands for roots[b]; one pass over the graph per level
 * serves every root).  Levels stay synchronous as in Section 2.3.2: by default
 * each level is one plain launch (the kernel boundary is the level barrier)
 * that takes its own direction decision on the device, and the host reads the
 * level counters once per group of queued levels; G5_FLAG_PERSISTENT in
 * g5_bfs_batch_ex runs every level in one cooperative launch with a grid-wide
 * barrier instead.  Returns once the work on `stream` is complete.
 *   roots    host, int64 [k], each in [0, n); duplicates allowed.
 *   k        1 .. 64.
 *   parents  device, int32 [k][n] (row b for roots[b]), or NULL to skip parents.
 *   levels   device, int8 [k][n].
 * Row b of levels equals the level array of g5_bfs(g, roots[b]) as int8, and
 * row b of parents is a valid parent array for roots[b].  Errors: G5_EINVAL,
 * G5_ERANGE (some vertex lies deeper than 127, the int8 maximum; fall back to
 * g5_bfs), G5_ENOMEM, G5_EDEVICE. */
g5_status g5_bfs_batch(const g5_csr *g, const int64_t *roots, int32_t k, int32_t *parents,
                       int8_t *levels, void *stream);

/* Knobs of g5_bfs_batch_ex.  Zero fields take the defaults. */
typedef struct {
  int32_t direction; /* g5_direction applied to every level of the batch */
  double alpha;      /* top-down while m_f <= m_u / alpha (tuned default), where m_f is the degree
                        sum of vertices with a nonzero frontier mask and m_u the degree sum of
                        vertices not yet reached by every root */
  int32_t flags;     /* G5_FLAG_TIME_STEPS: time the launch(es); G5_FLAG_PERSISTENT */
  int32_t blocks_per_cu; /* grid: workgroups per compute unit (persistent: capped by occupancy) */
  int32_t reserved[4];
} g5_batch_params;

/* Statistics of g5_bfs_batch_ex (host memory). */
typedef struct {
  int32_t nlevels;                         /* levels processed */
  int32_t dir[G5_MAX_STAT_LEVELS];         /* 1 top-down, 2 bottom-up */
  int64_t frontier[G5_MAX_STAT_LEVELS];    /* vertices with a nonzero frontier mask */
  double launch_ms;                        /* device time of the traversal: root statistics and
                                              every level (TIME_STEPS) */
  int32_t grid_blocks;                     /* workgroups per launch */
  int32_t pad;
  double alpha;                            /* switch threshold used */
  int32_t reserved[6];
} g5_batch_stats;

/* g5_bfs_batch with explicit parameters (NULL = defaults) and statistics
 * (NULL = none). */
g5_status g5_bfs_batch_ex(const g5_csr *g, const int64_t *roots, int32_t k, int32_t *parents,
                          int8_t *levels, void *stream, const g5_batch_params *params,
                          g5_batch_stats *stats);

/* Kernel 3 (Section 2.4): single-source shortest paths from `src` over a
 * graph built by g5_build_csr_w, by parallel delta-stepping (the direction
 * named in Section 4.1; buckets of width delta, relaxations by atomic
 * minimum, one queue per round; a round whose queue holds a large share of
 * the edges pulls instead).
 *   dist  device, uint32 [n]: the shortest-path distance from src, or
 *         0xFFFFFFFF (infinity) where v is not in src's component.
 *   prev  device, int32 [n]: prev[src] = src; for another reached v, the
 *         smallest-id neighbour u with dist[u] + w(u, v) = dist[v] (a
 *         shortest-path tree, the same on every run); -1 where unreached.
 * Errors: G5_EINVAL (src outside [0, n), NULL pointer, a graph without
 * weights), G5_ERANGE (a distance above 2^32 - 2), G5_ENOMEM, G5_EDEVICE. */
g5_status g5_sssp(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, void *stream);

typedef struct {
  uint32_t delta;   /* bucket width (0 = the default, 32) */
  int32_t flags;    /* G5_FLAG_TIME_STEPS: time the call on the device (ms) */
  int32_t pull_div; /* a round whose queue's rows hold at least nnz / pull_div
                       edges pulls (each vertex takes the best relaxation from
                       its neighbours in the queue) instead of pushing;
                       0 = the default (4), negative = never pull */
  int32_t reserved[5];
} g5_sssp_params;

typedef struct {
  int64_t rounds;   /* relaxation rounds (one launch each, plus hub pieces) */
  int64_t scans;    /* scans of the far set */
  int64_t buckets;  /* thresholds used */
  int64_t relaxed;  /* queue entries relaxed (a vertex counts once per round it is in) */
  int64_t delta;    /* bucket width used */
  double ms;        /* device time of the call (G5_FLAG_TIME_STEPS) */
  int64_t edges;    /* edges relaxed (the rows of the relaxed queue entries) */
  int64_t pulls;    /* rounds done by pulling */
  int64_t reserved[2];
} g5_sssp_stats;

/* g5_sssp with explicit parameters (NULL = defaults) and statistics (NULL =
 * none).  Same results and errors. */
g5_status g5_sssp_ex(const g5_csr *g, int64_t src, uint32_t *dist, int32_t *prev, void *stream,
                     const g5_sssp_params *params, g5_sssp_stats *stats);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * traversal as g5_bfs_batch (one launch per level, default parameters) with
 * its workspace (the seen and frontier masks, 32 bytes per vertex, and the
 * level counters) in a fixed device array inside the library instead of
 * memory it allocates: 32 * G5_NOALLOC_MAX_N bytes + 4 KiB on each GPU the
 * library runs on, held until the process ends.  The call allocates nothing;
 * it reads the level counters back with a device-to-host copy into a host
 * stack buffer.  Calls on one GPU share the array, so calls that overlap on
 * one GPU race (serialise them); each call clears what must start at zero.
 * Arguments, results and errors as g5_bfs_batch, plus G5_EINVAL when the
 * graph has more than G5_NOALLOC_MAX_N vertices or its device is not the
 * current device. */
#define G5_NOALLOC_MAX_N (1 << 20)
g5_status g5_bfs_batch_noalloc(const g5_csr *g, const int64_t *roots, int32_t k,
                               int32_t *parents, int8_t *levels, void *stream);

/* Measurement (not part of a traversal): the work that level `lvl` of a
 * finished traversal had to do, computed from its level array alone.  The
 * level array is unique (hop distances), so the counts do not depend on how
 * the traversal ran; they define the algorithmic bytes of a step:
 *   top-down   (Section 2.3.2, the parallel loops over the frontier and each
 *              frontier vertex's neighbours) 4 per queue entry + 16 per row's
 *              two 64-bit offsets + 4 per row entry, over Q, and 12 per
 *              claimed vertex (level, parent, next-queue entry):
 *              20 |Q| + 4 m_f + 12 claimed;
 *   bottom-up  16 row offsets + 4 per row entry read in row order up to and
 *              including the first frontier neighbour, over the unvisited
 *              vertices of degree >= 1, + n/8 (visited bitmap read) + n/8
 *              (next-frontier bitmap written) + 8 per claimed vertex:
 *              16 U + 4 S + n/4 + 8 claimed.
 *   level   device, int32 [n]: the level array of a traversal of g.
 *   lvl     the level whose step is counted (its frontier is level lvl).
 *   bottom_up  nonzero: also count U and S (a row scan per unvisited vertex);
 *           zero: out[3] = out[4] = 0 (a top-down step needs neither).
 *   out     host, int64 [5]: |Q| (vertices at level lvl), m_f (their degree
 *           sum), claimed (vertices at level lvl + 1), U (vertices of degree
 *           >= 1 at a level above lvl or unreached), S (over those, row
 *           entries up to and including the first one at level lvl, or the
 *           whole row).
 * Allocates a small device buffer per call; returns when the counts are on
 * the host.  Errors: G5_EINVAL (NULL pointer, lvl < 0), G5_ENOMEM, G5_EDEVICE. */
g5_status g5_level_work(const g5_csr *g, const int32_t *level, int32_t lvl, int32_t bottom_up,
                        int64_t *out, void *stream);

/* Message for the last non-OK status returned on the calling host thread. */
const char *g5_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
