/* CPU oracle for breadth-first search over a CSR graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may call this code; the GPU library never links
 * or calls it, and it shares no code with the GPU library.
 *
 * What it computes (paper: "Graph500 from OCaml-Multicore Perspective"):
 *   - Kernel 1 (Section 2.2): the graph of the tuple list as CSR.  The graph is
 *     undirected (Section 2), so every non-loop tuple (u, v) gives both u->v
 *     and v->u; self-loops and repeated edges may be ignored (Section 2.1) and
 *     are dropped.  Row v holds the distinct neighbours of v in ascending
 *     order.  An empty row repeats the previous row index and the end index of
 *     the last row is stored (the CSR description of Section 2.2), i.e.
 *     rp[0] = 0, rp[v+1] = rp[v] + deg(v), rp[n] = nnz.
 *   - Kernel 2 (Section 2.3.1, Algorithm "Sequential BFS"): a queue BFS
 *     returning the level array, plus the parent array that Algorithm
 *     "Basic Outline of Graph500" step 3 asks for.  Readings of the printed
 *     algorithm: the initialisation runs over vertices (it is printed over
 *     E); the "->" in the neighbour test is an equality test; a vertex is
 *     marked visited when it is discovered (the printed algorithm marks it
 *     after its neighbour loop, which can enqueue a vertex twice and overwrite
 *     its level); parent[v] is the vertex that discovered v and
 *     parent[root] = root; unreached vertices keep level -1 and parent -1.
 *   - Validation of a BFS result, and the traversed-edge count m_r used for
 *     TEPS (Section 4.3 names TEPS over 64 roots as the Graph500 metric).
 *   - The deterministic parent choice: for a reached v other than the root,
 *     the smallest-id neighbour one level closer to the root.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Kernel 1.  edges: [m][2] int64 tuples; rp: int64[n+1] (output);
 * ci: int32 buffer with room for 2*m entries (output, packed to nnz).
 * Returns nnz, or -1 if a tuple names a vertex outside [0, n), -2 if n or m
 * is out of range. */
int64_t orc_build_csr(const int64_t *edges, int64_t m, int64_t n, int64_t *rp,
                      int32_t *ci) {
  if (n < 1 || n > 2147483647LL || m < 0) return -2;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < 2 * m; ++i)
    if (edges[i] < 0 || edges[i] >= n) bad = 1;
  if (bad) return -1;
  /* degree counts of both directions, self-loops skipped */
  int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *cur = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  if (!cnt || !cur) {
    free(cnt);
    free(cur);
    return -3;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u == v) continue;
#pragma omp atomic
    cnt[u]++;
#pragma omp atomic
    cnt[v]++;
  }
  /* exclusive prefix sum: start of each (not yet deduplicated) row */
  cur[0] = 0;
  for (int64_t v = 0; v < n; ++v) cur[v + 1] = cur[v] + cnt[v];
  memcpy(rp, cur, (size_t)(n + 1) * sizeof(int64_t));
  /* scatter both directions (the order inside a row does not matter: rows
   * are sorted next) */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u == v) continue;
    int64_t pu, pv;
#pragma omp atomic capture
    pu = cur[u]++;
#pragma omp atomic capture
    pv = cur[v]++;
    ci[pu] = (int32_t)v;
    ci[pv] = (int32_t)u;
  }
  /* sort each row and count its distinct entries (rows are independent) */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = rp[v], e = rp[v + 1];
    if (e - b > 1) qsort(ci + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
    int64_t d = 0;
    for (int64_t k = b; k < e; ++k)
      if (k == b || ci[k] != ci[k - 1]) ci[b + d++] = ci[k];
    cnt[v] = d;
  }
  /* pack rows left and write the final row index */
  int64_t w = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = rp[v];
    if (w != b) memmove(ci + w, ci + b, (size_t)cnt[v] * sizeof(int32_t));
    rp[v] = w;
    w += cnt[v];
  }
  rp[n] = w;
  free(cnt);
  free(cur);
  return w;
}

/* Kernel 2, sequential queue BFS from root.  parent, level: int32[n]
 * (outputs).  Returns the number of reached vertices, or -1 for a bad root,
 * -3 if the queue cannot be allocated. */
int64_t orc_bfs(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root,
                int32_t *parent, int32_t *level) {
  if (root < 0 || root >= n) return -1;
  int32_t *q = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!q) return -3;
  for (int64_t v = 0; v < n; ++v) {
    level[v] = -1;
    parent[v] = -1;
  }
  level[root] = 0;
  parent[root] = (int32_t)root;
  int64_t head = 0, tail = 0;
  q[tail++] = (int32_t)root;
  while (head < tail) {
    int32_t x = q[head++];
    for (int64_t k = rp[x]; k < rp[x + 1]; ++k) {
      int32_t u = ci[k];
      if (level[u] == -1) {
        level[u] = level[x] + 1;
        parent[u] = x;
        q[tail++] = u;
      }
    }
  }
  free(q);
  return tail;
}

/* Connected components of the tuple list (self-loops contribute nothing) by
 * union-find with path halving and union by size; an algorithm independent
 * of BFS.  label[v] = the representative of v's component.  Returns the
 * number of components, or -1 for an id outside [0, n). */
static int64_t uf_find(int64_t *p, int64_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

int64_t orc_components(const int64_t *edges, int64_t m, int64_t n, int64_t *label) {
  int64_t *sz = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!sz) return -3;
  for (int64_t v = 0; v < n; ++v) {
    label[v] = v;
    sz[v] = 1;
  }
  int64_t comps = n;
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      free(sz);
      return -1;
    }
    int64_t a = uf_find(label, u), b = uf_find(label, v);
    if (a == b) continue;
    if (sz[a] < sz[b]) {
      int64_t t = a;
      a = b;
      b = t;
    }
    label[b] = a;
    sz[a] += sz[b];
    comps--;
  }
  for (int64_t v = 0; v < n; ++v) label[v] = uf_find(label, v);
  free(sz);
  return comps;
}

/* Binary search for x in the ascending row [b, e) of ci. */
static int row_has(const int32_t *ci, int64_t b, int64_t e, int32_t x) {
  while (b < e) {
    int64_t mid = b + (e - b) / 2;
    if (ci[mid] == x) return 1;
    if (ci[mid] < x)
      b = mid + 1;
    else
      e = mid;
  }
  return 0;
}

/* Validation of a BFS result against the oracle CSR and the union-find labels.
 * Returns 0 if valid, else the number of the first rule broken:
 *   1  parent[root] != root or level[root] != 0
 *   2  a value out of range, or parent = -1 and level != -1 (or vice versa)
 *   3  for a reached v != root, parent[v] is not a neighbour of v
 *   4  for a reached v != root, level[parent[v]] != level[v] - 1
 *   5  the reached set differs from the root's connected component
 *   6  an edge whose two reached ends differ in level by more than 1
 *   7  a vertex other than the root has level 0 */
int orc_validate(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root,
                 const int32_t *parent, const int32_t *level, const int64_t *label) {
  if (root < 0 || root >= n) return 2;
  if (parent[root] != root || level[root] != 0) return 1;
  for (int64_t v = 0; v < n; ++v) {
    int32_t p = parent[v], l = level[v];
    if (p < -1 || p >= n || l < -1) return 2;
    if ((p == -1) != (l == -1)) return 2;
    int reached = l >= 0;
    if (reached != (label[v] == label[root])) return 5;
    if (!reached || v == root) continue;
    if (l == 0) return 7;
    if (!row_has(ci, rp[v], rp[v + 1], p)) return 3;
    if (level[p] != l - 1) return 4;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (level[v] < 0) continue;
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      int32_t u = ci[k];
      if (level[u] < 0) return 5;
      int32_t d = level[u] - level[v];
      if (d > 1 || d < -1) return 6;
    }
  }
  return 0;
}

/* The same validation from the tuple list alone (no CSR), for graphs too
 * large to give the oracle its own CSR in a test.  Checks, in one pass over
 * the tuples:
 *   (a) parent[root] = root, level[root] = 0, no other vertex at level 0,
 *       parent = -1 exactly when level = -1, values in range;
 *   (b) every non-loop tuple has both ends reached or both unreached, and
 *       reached ends differ in level by at most 1;
 *   (c) every reached v != root has level[parent[v]] = level[v] - 1 and
 *       (parent[v], v) occurs as a tuple in some orientation.
 * (b) makes the reached set a union of components and, along any shortest
 * path from the root, gives level[v] <= dist(root, v); (c) gives each reached
 * vertex a graph path of length level[v] back to level 0, which is the root
 * alone, so level[v] >= dist(root, v) and the reached set is exactly the
 * root's component.  Hence levels equal hop distances and parents form a BFS
 * tree.  Returns 0 or the rule number of orc_validate (3 = no tuple joins a
 * vertex to its parent). */
int orc_validate_edges(const int64_t *edges, int64_t m, int64_t n, int64_t root,
                       const int32_t *parent, const int32_t *level) {
  if (root < 0 || root >= n) return 2;
  if (parent[root] != root || level[root] != 0) return 1;
  for (int64_t v = 0; v < n; ++v) {
    int32_t p = parent[v], l = level[v];
    if (p < -1 || p >= n || l < -1) return 2;
    if ((p == -1) != (l == -1)) return 2;
    if (l == 0 && v != root) return 7;
    if (l > 0 && level[p] != l - 1) return 4;
  }
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  if (!seen) return -3;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : bad)
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      bad = bad > 2 ? bad : 2;
      continue;
    }
    if (u == v) continue;
    int32_t lu = level[u], lv = level[v];
    if ((lu < 0) != (lv < 0)) {
      bad = bad > 5 ? bad : 5;
      continue;
    }
    if (lu < 0) continue;
    int32_t d = lu - lv;
    if (d > 1 || d < -1) {
      bad = bad > 6 ? bad : 6;
      continue;
    }
    if (parent[v] == u && lv == lu + 1) __atomic_store_n(&seen[v], (uint8_t)1, __ATOMIC_RELAXED);
    if (parent[u] == v && lu == lv + 1) __atomic_store_n(&seen[u], (uint8_t)1, __ATOMIC_RELAXED);
  }
  if (!bad) {
    for (int64_t v = 0; v < n; ++v)
      if (v != root && level[v] > 0 && !seen[v]) {
        bad = 3;
        break;
      }
  }
  free(seen);
  return bad;
}

/* Edges traversed from a root, for TEPS: the number of distinct undirected
 * non-loop edges in the root's component, (1/2) * sum of deg(v) over reached
 * v. */
int64_t orc_teps_edges(const int64_t *rp, int64_t n, const int32_t *level) {
  int64_t s = 0;
  for (int64_t v = 0; v < n; ++v)
    if (level[v] >= 0) s += rp[v + 1] - rp[v];
  return s / 2;
}

/* Deterministic parents from a level array: parent[root] = root; for a reached
 * v != root, the smallest-id neighbour u with level[u] = level[v] - 1; -1 if v
 * is unreached.  Returns 0, or -1 if some reached v has no such neighbour. */
int orc_min_parents(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root,
                    const int32_t *level, int32_t *parent) {
  int bad = 0;
  for (int64_t v = 0; v < n; ++v) {
    parent[v] = -1;
    if (level[v] < 0) continue;
    if (v == root) {
      parent[v] = (int32_t)v;
      continue;
    }
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k)
      if (level[ci[k]] == level[v] - 1) {
        parent[v] = ci[k];  /* rows are ascending: the first match is the smallest */
        break;
      }
    if (parent[v] < 0) bad = 1;
  }
  return bad ? -1 : 0;
}
