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

/* Parent check for a level array already known to be exact (compared with
 * orc_bfs's levels beforehand): parent[root] = root, level[root] = 0, and for
 * every other v either parent[v] = level[v] = -1 (unreached) or parent[v] is a
 * neighbour of v (binary search in its ascending row) one level closer to the
 * root, with no other vertex at level 0.  With exact levels these are the
 * rules of orc_validate that concern the parent array; the rules about the
 * reached set and edge spans hold because the levels are the hop distances.
 * One parallel pass over the vertices.  Returns 0 or the rule number of
 * orc_validate (1, 2, 3, 4 or 7); when several rules are broken, the largest
 * number found. */
int orc_check_parents(const int64_t *rp, const int32_t *ci, int64_t n, int64_t root,
                      const int32_t *parent, const int32_t *level) {
  if (root < 0 || root >= n) return 2;
  if (parent[root] != root || level[root] != 0) return 1;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : bad)
  for (int64_t v = 0; v < n; ++v) {
    const int32_t p = parent[v], l = level[v];
    int r = 0;
    if (p < -1 || p >= n || l < -1 || (p == -1) != (l == -1))
      r = 2;
    else if (l >= 0 && v != root) {
      if (l == 0)
        r = 7;
      else if (!row_has(ci, rp[v], rp[v + 1], p))
        r = 3;
      else if (level[p] != l - 1)
        r = 4;
    }
    if (r > bad) bad = r;
  }
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

/* ------------------------------------------------------------------------
 * Kernel 3 (Section 2.4, Algorithm "Sequential SSSP"): shortest paths from
 * one source over the weighted graph.  The tuple list carries a weight per
 * tuple (Section 2.1: the generator's 3 x #E matrix of start, end and weight
 * columns).  Readings: weights are integers (0..255 here, so sums and ties
 * are exact); the graph is undirected, so each non-loop tuple gives both
 * directions with its weight; of repeated tuples joining the same two
 * vertices only the smallest weight can lie on a shortest path, so the CSR
 * keeps that one; self-loops are dropped; dist[v] = infinity (UINT32_MAX)
 * and prev[v] = -1 for unreached v; prev[source] = source, as for the BFS
 * parent array (the printed algorithm leaves it at -1).
 * ------------------------------------------------------------------------ */

typedef struct {
  int32_t v;
  uint8_t w;
} orc_vw;

static int cmp_vw(const void *a, const void *b) {
  const orc_vw *x = (const orc_vw *)a, *y = (const orc_vw *)b;
  if (x->v != y->v) return (x->v > y->v) - (x->v < y->v);
  return (x->w > y->w) - (x->w < y->w);
}

/* Weighted Kernel 1.  edges [m][2], weights [m]; rp int64[n+1], ci int32 and
 * wt uint8 buffers with room for 2*m entries (outputs, packed to nnz).  Row v
 * holds v's distinct neighbours ascending, each with the smallest weight of
 * the tuples joining them.  Returns nnz, or -1 / -2 / -3 as orc_build_csr. */
int64_t orc_build_csr_w(const int64_t *edges, const uint8_t *weights, int64_t m, int64_t n,
                        int64_t *rp, int32_t *ci, uint8_t *wt) {
  if (n < 1 || n > 2147483647LL || m < 0) return -2;
  for (int64_t i = 0; i < 2 * m; ++i)
    if (edges[i] < 0 || edges[i] >= n) return -1;
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  orc_vw *tmp = (orc_vw *)malloc((size_t)(2 * m + 1) * sizeof(orc_vw));
  if (!cnt || !tmp) {
    free(cnt);
    free(tmp);
    return -3;
  }
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u == v) continue;
    cnt[u + 1]++;
    cnt[v + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  for (int64_t v = 0; v <= n; ++v) rp[v] = cnt[v];
  for (int64_t i = 0; i < m; ++i) {
    int64_t u = edges[2 * i], v = edges[2 * i + 1];
    if (u == v) continue;
    tmp[cnt[u]].v = (int32_t)v;
    tmp[cnt[u]++].w = weights[i];
    tmp[cnt[v]].v = (int32_t)u;
    tmp[cnt[v]++].w = weights[i];
  }
  /* sort each row by (neighbour, weight); the first of each neighbour's run
   * carries the smallest weight */
  int64_t w = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = rp[v], e = rp[v + 1];
    if (e - b > 1) qsort(tmp + b, (size_t)(e - b), sizeof(orc_vw), cmp_vw);
    rp[v] = w;
    for (int64_t k = b; k < e; ++k)
      if (k == b || tmp[k].v != tmp[k - 1].v) {
        ci[w] = tmp[k].v;
        wt[w] = tmp[k].w;
        ++w;
      }
  }
  rp[n] = w;
  free(cnt);
  free(tmp);
  return w;
}

/* Binary min-heap of (distance, vertex) with lazy deletion: the "vertex in Q
 * with min dist" selection of the algorithm. */
typedef struct {
  uint64_t d;
  int32_t v;
} orc_hn;

static void heap_push(orc_hn *h, int64_t *len, uint64_t d, int32_t v) {
  int64_t i = (*len)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= d) break;
    h[i] = h[p];
    i = p;
  }
  h[i].d = d;
  h[i].v = v;
}

static orc_hn heap_pop(orc_hn *h, int64_t *len) {
  orc_hn top = h[0], last = h[--(*len)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *len) break;
    if (c + 1 < *len && h[c + 1].d < h[c].d) ++c;
    if (h[c].d >= last.d) break;
    h[i] = h[c];
    i = c;
  }
  if (*len > 0) h[i] = last;
  return top;
}

/* Dijkstra from src (Algorithm "Sequential SSSP"): dist starts at infinity
 * and prev at -1 everywhere, dist[src] = 0; repeatedly take the unsettled
 * vertex of smallest dist and relax every unsettled neighbour, setting
 * dist[v] = dist[u] + w(u, v) and prev[v] = u when that is smaller.
 * dist uint32 [n] (UINT32_MAX = unreached), prev int32 [n]; prev[src] = src.
 * Returns the number of reached vertices, -1 for a bad source, -3 if memory
 * runs out, -4 if a distance exceeds UINT32_MAX - 1. */
int64_t orc_sssp(const int64_t *rp, const int32_t *ci, const uint8_t *wt, int64_t n, int64_t src,
                 uint32_t *dist, int32_t *prev) {
  if (src < 0 || src >= n) return -1;
  uint64_t *d = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
  orc_hn *h = (orc_hn *)malloc((size_t)(rp[n] + 1) * sizeof(orc_hn));
  if (!d || !done || !h) {
    free(d);
    free(done);
    free(h);
    return -3;
  }
  const uint64_t INF = ~0ull;
  for (int64_t v = 0; v < n; ++v) {
    d[v] = INF;
    prev[v] = -1;
  }
  d[src] = 0;
  prev[src] = (int32_t)src;
  int64_t len = 0, reached = 0;
  heap_push(h, &len, 0, (int32_t)src);
  while (len > 0) {
    orc_hn t = heap_pop(h, &len);
    int32_t u = t.v;
    if (done[u] || t.d != d[u]) continue; /* a stale entry */
    done[u] = 1;
    ++reached;
    for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
      int32_t v = ci[k];
      if (done[v]) continue;
      uint64_t alt = d[u] + wt[k];
      if (alt < d[v]) {
        d[v] = alt;
        prev[v] = u;
        heap_push(h, &len, alt, v);
      }
    }
  }
  int64_t rc = reached;
  for (int64_t v = 0; v < n; ++v) {
    if (d[v] != INF && d[v] >= 0xffffffffull) rc = -4;
    dist[v] = d[v] == INF ? 0xffffffffu : (uint32_t)d[v];
  }
  free(d);
  free(done);
  free(h);
  return rc;
}

/* Weight of the edge (u, v) in u's ascending row, or -1 if there is none. */
static int row_weight(const int32_t *ci, const uint8_t *wt, int64_t b, int64_t e, int32_t x) {
  while (b < e) {
    int64_t mid = b + (e - b) / 2;
    if (ci[mid] == x) return wt[mid];
    if (ci[mid] < x)
      b = mid + 1;
    else
      e = mid;
  }
  return -1;
}

/* Validation of an SSSP result (dist, prev) from src, independent of the
 * Dijkstra above.  Returns 0 if valid, else the first rule broken:
 *   1  dist[src] != 0 or prev[src] != src
 *   2  dist is infinity exactly where prev is -1 fails, or a value out of range
 *   3  prev[v] is not a neighbour of v
 *   4  dist[v] != dist[prev[v]] + w(prev[v], v)
 *   5  an edge (u, v) with dist[v] > dist[u] + w(u, v) (or one end unreached)
 *   6  the prev pointers of some reached vertex do not lead back to src
 * Rule 5 makes dist a lower bound of every path length and rules 3, 4, 6 give
 * each reached v a path of length dist[v] from src, so dist is exactly the
 * shortest-path distance and prev a shortest-path tree. */
int orc_check_sssp(const int64_t *rp, const int32_t *ci, const uint8_t *wt, int64_t n, int64_t src,
                   const uint32_t *dist, const int32_t *prev) {
  const uint32_t INF = 0xffffffffu;
  if (src < 0 || src >= n) return 2;
  if (dist[src] != 0 || prev[src] != src) return 1;
  for (int64_t v = 0; v < n; ++v) {
    int32_t p = prev[v];
    if (p < -1 || p >= n) return 2;
    if ((p == -1) != (dist[v] == INF)) return 2;
    if (p < 0 || v == src) continue;
    int w = row_weight(ci, wt, rp[v], rp[v + 1], p);
    if (w < 0) return 3;
    if (dist[p] == INF || (uint64_t)dist[v] != (uint64_t)dist[p] + (uint64_t)w) return 4;
  }
  for (int64_t u = 0; u < n; ++u)
    for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
      int32_t v = ci[k];
      if ((dist[u] == INF) != (dist[v] == INF)) return 5;
      if (dist[u] != INF && (uint64_t)dist[v] > (uint64_t)dist[u] + wt[k]) return 5;
    }
  /* children lists of the prev tree, then a walk from src over them */
  int64_t *cs = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *kids = (int32_t *)malloc((size_t)n * sizeof(int32_t) + 4);
  int32_t *stack = (int32_t *)malloc((size_t)n * sizeof(int32_t) + 4);
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  if (!cs || !kids || !stack || !seen) {
    free(cs);
    free(kids);
    free(stack);
    free(seen);
    return -3;
  }
  for (int64_t v = 0; v < n; ++v)
    if (prev[v] >= 0 && v != src) cs[prev[v] + 1]++;
  for (int64_t v = 0; v < n; ++v) cs[v + 1] += cs[v];
  for (int64_t v = 0; v < n; ++v)
    if (prev[v] >= 0 && v != src) kids[cs[prev[v]]++] = (int32_t)v;
  for (int64_t v = n; v > 0; --v) cs[v] = cs[v - 1];
  cs[0] = 0;
  int64_t top = 0;
  stack[top++] = (int32_t)src;
  seen[src] = 1;
  while (top > 0) {
    int32_t u = stack[--top];
    for (int64_t k = cs[u]; k < cs[u + 1]; ++k)
      if (!seen[kids[k]]) {
        seen[kids[k]] = 1;
        stack[top++] = kids[k];
      }
  }
  int bad = 0;
  for (int64_t v = 0; v < n; ++v)
    if (prev[v] >= 0 && !seen[v]) bad = 6;
  free(cs);
  free(kids);
  free(stack);
  free(seen);
  return bad;
}

/* Deterministic predecessors from a distance array: prev[src] = src; for a
 * reached v != src, the smallest-id neighbour u with
 * dist[u] + w(u, v) = dist[v]; -1 if v is unreached.  Returns 0, or -1 if
 * some reached v has no such neighbour. */
int orc_min_prev(const int64_t *rp, const int32_t *ci, const uint8_t *wt, int64_t n, int64_t src,
                 const uint32_t *dist, int32_t *prev) {
  int bad = 0;
  for (int64_t v = 0; v < n; ++v) {
    prev[v] = -1;
    if (dist[v] == 0xffffffffu) continue;
    if (v == src) {
      prev[v] = (int32_t)v;
      continue;
    }
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      int32_t u = ci[k];
      if (dist[u] != 0xffffffffu && (uint64_t)dist[u] + wt[k] == (uint64_t)dist[v]) {
        prev[v] = u; /* rows are ascending: the first match is the smallest id */
        break;
      }
    }
    if (prev[v] < 0) bad = 1;
  }
  return bad ? -1 : 0;
}
