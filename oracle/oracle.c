/*
 * oracle.c -- plain, slow, single-threaded CPU reference for cover-edge
 * triangle counting (Bader et al., "Triangle Counting Through Cover-Edges",
 * arXiv 2210.00389).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * compared against.  It shares no code, header, table or build step with the
 * library; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  No product code path may call it.
 *
 * What it computes, in the paper's order and notation:
 *   oracle_build_csr     G = (V, E) as a simple undirected graph (Sec. II-A):
 *                        loops dropped, both orientations kept, repeats
 *                        merged, neighbour lists N(v) sorted ascending.
 *   oracle_bfs_levels    L(v) = BFS distance from the root (Def. 2), with the
 *                        scan of Alg. 1 (every vertex left unvisited starts a
 *                        BFS of its own, so its component's levels count from
 *                        it).
 *   oracle_cover_edges   the horizontal edges (u, v), L(u) = L(v), u < v, in
 *                        the edge order of the CSR (Alg. 1, edge selection;
 *                        Thm. 1 says they form a cover-edge set).
 *   oracle_count         for every horizontal edge and every w in N(u) ∩ N(v):
 *                        count w when L(u) != L(w), or L(u) = L(w) and v < w
 *                        (Alg. 1, counting test; Thm. 2 proves it exact).
 *                        Full integer levels are compared, never parities.
 *   oracle_list_triangles  triangle finding: every (u, v, w) the count
 *                        accepts, written as its three ids ascending, in the
 *                        order Alg. 1 visits them.
 *   oracle_edge_supports the number of triangles on each edge, from that
 *                        enumeration (+1 on both orientations of the three
 *                        edges of every found triangle).
 *   oracle_edge_count    the plain direction-oriented edge iterator of the
 *                        related-work section: every edge (u, v), u < v,
 *                        counts the w in N(u) ∩ N(v) with w > v.  It uses no
 *                        levels, so it is an independent second count.
 *
 * Two intersection modes (both literal):
 *   mode 0  "hash" -- the paper's hashing-based intersection with a
 *           direct-address table: N(u) is stamped once per u (stamp = u),
 *           then every element of N(v) is looked up.  The loop order is
 *           Alg. 1's (u ascending, then v ascending).
 *   mode 1  "merge" -- two-pointer merge of the sorted lists N(u), N(v).
 *
 * Status codes are this file's own.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OR_OK = 0,
  OR_EINVAL = -1,
  OR_ENOMEM = -2,
  OR_EOFFSETS = -3,
  OR_ERANGE = -4,
  OR_EUNSORTED = -5,
  OR_EDUP = -6,
  OR_ESELF = -7,
  OR_EASYM = -8
};

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* ---------------------------------------------------------------- CSR */
/* Simple undirected graph from raw pairs: every pair (s, d) with s != d gives
 * the two directed entries s->d and d->s; each row is then sorted and its
 * repeats dropped.  cols must hold 2*num_pairs entries.  *nnz_out receives
 * the final number of directed entries (twice the edge count m). */
int oracle_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                     int64_t* row_offsets, int32_t* cols, int64_t* nnz_out) {
  if (n < 0 || num_pairs < 0 || !row_offsets || !nnz_out) return OR_EINVAL;
  if (num_pairs > 0 && (!src || !dst || !cols)) return OR_EINVAL;
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) return OR_ENOMEM;
  for (int64_t e = 0; e < num_pairs; ++e) {
    int64_t s = src[e], d = dst[e];
    if (s < 0 || s >= n || d < 0 || d >= n) { free(deg); return OR_ERANGE; }
    if (s == d) continue;
    deg[s] += 1;
    deg[d] += 1;
  }
  /* provisional offsets (with repeats) */
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!start) { free(deg); return OR_ENOMEM; }
  start[0] = 0;
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
  for (int64_t v = 0; v < n; ++v) deg[v] = start[v]; /* reuse as fill cursor */
  for (int64_t e = 0; e < num_pairs; ++e) {
    int32_t s = src[e], d = dst[e];
    if (s == d) continue;
    cols[deg[s]++] = d;
    cols[deg[d]++] = s;
  }
  /* sort every row, drop repeats, pack rows to the left */
  int64_t out = 0;
  row_offsets[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = start[v], e = start[v + 1];
    if (e > b) qsort(cols + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
    int64_t row_begin = out;
    for (int64_t i = b; i < e; ++i) {
      if (out > row_begin && cols[out - 1] == cols[i]) continue;
      cols[out++] = cols[i];
    }
    row_offsets[v + 1] = out;
  }
  *nnz_out = out;
  free(start);
  free(deg);
  return OR_OK;
}

/* Checks that (row_offsets, cols) is a simple undirected graph: offsets start
 * at 0 and never decrease, ids are in range, rows strictly ascending (so no
 * repeats), no loops, and every u->v has its v->u. */
int oracle_validate_csr(int64_t n, const int64_t* off, const int32_t* cols) {
  if (n < 0 || !off) return OR_EINVAL;
  if (off[0] != 0) return OR_EOFFSETS;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return OR_EOFFSETS;
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t i = off[v]; i < off[v + 1]; ++i) {
      int32_t w = cols[i];
      if (w < 0 || w >= n) return OR_ERANGE;
      if (w == v) return OR_ESELF;
      if (i > off[v]) {
        if (cols[i - 1] == w) return OR_EDUP;
        if (cols[i - 1] > w) return OR_EUNSORTED;
      }
    }
  }
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t i = off[v]; i < off[v + 1]; ++i) {
      int32_t w = cols[i];
      /* linear search of v in N(w): slow and obviously right */
      int found = 0;
      for (int64_t j = off[w]; j < off[w + 1]; ++j)
        if (cols[j] == v) { found = 1; break; }
      if (!found) return OR_EASYM;
    }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------- BFS */
/* Default first root: the vertex of largest degree, the smallest id among
 * ties.  -1 for an empty graph. */
int64_t oracle_default_root(int64_t n, const int64_t* off) {
  int64_t best = -1, bestd = -1;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = off[v + 1] - off[v];
    if (d > bestd) { bestd = d; best = v; }
  }
  return best;
}

/* FIFO breadth-first search from r over vertices not yet levelled; levels
 * count from 0 at r.  Returns the number of levels reached. */
static int32_t bfs_from(int64_t r, const int64_t* off, const int32_t* cols, int32_t* L,
                        int32_t* queue) {
  int64_t head = 0, tail = 0;
  int32_t depth = 0;
  L[r] = 0;
  queue[tail++] = (int32_t)r;
  while (head < tail) {
    int32_t x = queue[head++];
    for (int64_t i = off[x]; i < off[x + 1]; ++i) {
      int32_t y = cols[i];
      if (L[y] < 0) {
        L[y] = L[x] + 1;
        if (L[y] > depth) depth = L[y];
        queue[tail++] = y;
      }
    }
  }
  return depth + 1;
}

/* Levels of Alg. 1: BFS from `root` (root < 0 picks the default root), then
 * scan v = 0..n-1 and start a new BFS at every vertex still unvisited.
 * *num_levels (nullable) receives the largest level count of any one BFS;
 * *num_roots (nullable) the number of BFS started. */
int oracle_bfs_levels(int64_t n, const int64_t* off, const int32_t* cols, int64_t root,
                      int32_t* L, int32_t* num_levels, int64_t* num_roots) {
  if (n < 0 || !off || (n > 0 && !L)) return OR_EINVAL;
  if (root >= n) return OR_EINVAL;
  if (n == 0) {
    if (num_levels) *num_levels = 0;
    if (num_roots) *num_roots = 0;
    return OR_OK;
  }
  if (root < 0) root = oracle_default_root(n, off);
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return OR_ENOMEM;
  for (int64_t v = 0; v < n; ++v) L[v] = -1;
  int32_t most = bfs_from(root, off, cols, L, queue);
  int64_t roots = 1;
  for (int64_t v = 0; v < n; ++v) {
    if (L[v] < 0) {
      int32_t d = bfs_from(v, off, cols, L, queue);
      if (d > most) most = d;
      ++roots;
    }
  }
  free(queue);
  if (num_levels) *num_levels = most;
  if (num_roots) *num_roots = roots;
  return OR_OK;
}

/* ------------------------------------------------------- cover edges */
/* Horizontal edges (u, v) with L(u) = L(v) and u < v, u ascending then v
 * ascending.  h_u / h_v may be NULL to only count.  Returns |H|. */
int64_t oracle_cover_edges(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L,
                           int32_t* h_u, int32_t* h_v) {
  int64_t h = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t v = cols[i];
      if (v > u && L[u] == L[v]) {
        if (h_u) { h_u[h] = (int32_t)u; h_v[h] = v; }
        ++h;
      }
    }
  }
  return h;
}

/* ------------------------------------------------------------ count */
/* The counting test of Alg. 1 for apex w of horizontal edge (u, v). */
static inline int counts(const int32_t* L, int32_t u, int32_t v, int32_t w) {
  return (L[u] != L[w]) || (L[u] == L[w] && v < w);
}

/* Triangle count over the horizontal edges.
 *   T (required)        total count
 *   per_edge (nullable) c(u,v) for the i-th horizontal edge, in the order of
 *                       oracle_cover_edges
 *   per_vertex (null.)  number of counted triangles containing each vertex
 *   mode                0 = direct-address table, 1 = two-pointer merge
 * (count_rows runs the loop over the rows u = u_begin, u_begin + stride, ...
 * below u_end only; the full count is stride 1 over [0, n).) */
static int count_rows(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode,
                      int64_t u_begin, int64_t u_end, int64_t stride, int64_t* T, int64_t* per_edge,
                      int64_t* per_vertex) {
  if (n < 0 || !off || !T || (n > 0 && !L)) return OR_EINVAL;
  if (mode != 0 && mode != 1) return OR_EINVAL;
  if (u_begin < 0 || u_end > n || u_begin > u_end || stride < 1) return OR_EINVAL;
  int64_t total = 0, hidx = 0;
  int64_t* stamp = NULL;
  if (per_vertex)
    for (int64_t v = 0; v < n; ++v) per_vertex[v] = 0;
  if (mode == 0) {
    stamp = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!stamp && n > 0) return OR_ENOMEM;
    for (int64_t v = 0; v < n; ++v) stamp[v] = -1;
  }
  for (int64_t u = u_begin; u < u_end; u += stride) {
    int stamped = 0;
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t v = cols[i];
      if (!(v > u && L[u] == L[v])) continue; /* (u, v) is not a cover edge */
      int64_t c = 0;
      if (mode == 0) {
        if (!stamped) {
          for (int64_t a = off[u]; a < off[u + 1]; ++a) stamp[cols[a]] = u;
          stamped = 1;
        }
        for (int64_t b = off[v]; b < off[v + 1]; ++b) {
          int32_t w = cols[b];
          if (stamp[w] == u && counts(L, (int32_t)u, v, w)) {
            ++c;
            if (per_vertex) { per_vertex[u]++; per_vertex[v]++; per_vertex[w]++; }
          }
        }
      } else {
        int64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1];
        while (a < ae && b < be) {
          if (cols[a] < cols[b]) ++a;
          else if (cols[a] > cols[b]) ++b;
          else {
            int32_t w = cols[a];
            if (counts(L, (int32_t)u, v, w)) {
              ++c;
              if (per_vertex) { per_vertex[u]++; per_vertex[v]++; per_vertex[w]++; }
            }
            ++a;
            ++b;
          }
        }
      }
      if (per_edge) per_edge[hidx] = c;
      ++hidx;
      total += c;
    }
  }
  free(stamp);
  *T = total;
  return OR_OK;
}

int oracle_count(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode,
                 int64_t* T, int64_t* per_edge, int64_t* per_vertex) {
  return count_rows(n, off, cols, L, mode, 0, n, 1, T, per_edge, per_vertex);
}

/* The same count restricted to the cover edges (u, v) with u in
 * [u_begin, u_end); summing over a partition of [0, n) gives T.  Used to time
 * a bounded sample of the work. */
int oracle_count_rows(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode,
                      int64_t u_begin, int64_t u_end, int64_t* T) {
  return count_rows(n, off, cols, L, mode, u_begin, u_end, 1, T, NULL, NULL);
}

/* The same count restricted to the rows u_begin, u_begin + stride, ... below
 * u_end: the phases 0 .. stride-1 partition the rows, so their counts sum to
 * T.  A systematic sample across the whole id range, used to time a bounded
 * share of the work. */
int oracle_count_rows_strided(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode,
                              int64_t u_begin, int64_t u_end, int64_t stride, int64_t* T) {
  return count_rows(n, off, cols, L, mode, u_begin, u_end, stride, T, NULL, NULL);
}

/* c(u, v) for a single horizontal edge u < v, by two-pointer merge.  Used to
 * check sampled per-edge outputs on graphs too large for a full count. */
int64_t oracle_edge_support(const int64_t* off, const int32_t* cols, const int32_t* L, int32_t u,
                            int32_t v) {
  int64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1], c = 0;
  while (a < ae && b < be) {
    if (cols[a] < cols[b]) ++a;
    else if (cols[a] > cols[b]) ++b;
    else {
      if (counts(L, u, v, cols[a])) ++c;
      ++a;
      ++b;
    }
  }
  return c;
}

/* Position of v in the sorted row of u, or -1 (binary search). */
static int64_t find_in_row(const int64_t* off, const int32_t* cols, int32_t u, int32_t v) {
  int64_t lo = off[u], hi = off[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (cols[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < off[u + 1] && cols[lo] == v) ? lo : -1;
}

static void sort3(int32_t* t) {
  int32_t x;
  if (t[0] > t[1]) { x = t[0]; t[0] = t[1]; t[1] = x; }
  if (t[1] > t[2]) { x = t[1]; t[1] = t[2]; t[2] = x; }
  if (t[0] > t[1]) { x = t[0]; t[0] = t[1]; t[1] = x; }
}

/* Alg. 1's enumeration with a two-pointer merge per horizontal edge: every
 * accepted (u, v, w) is handed to `emit` as an ascending triple. */
static int enumerate(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L,
                     void (*emit)(void*, const int32_t*), void* ctx, int64_t* T) {
  if (n < 0 || !off || !T || (n > 0 && !L)) return OR_EINVAL;
  int64_t total = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t v = cols[i];
      if (v <= u || L[u] != L[v]) continue; /* only the horizontal edges */
      int64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1];
      while (a < ae && b < be) {
        if (cols[a] < cols[b]) ++a;
        else if (cols[a] > cols[b]) ++b;
        else {
          int32_t w = cols[a];
          if (counts(L, (int32_t)u, v, w)) {
            int32_t t[3] = {(int32_t)u, v, w};
            sort3(t);
            emit(ctx, t);
            ++total;
          }
          ++a;
          ++b;
        }
      }
    }
  }
  *T = total;
  return OR_OK;
}

struct list_ctx {
  int32_t* tri;
  int64_t cap, at;
};

static void emit_list(void* p, const int32_t* t) {
  struct list_ctx* c = (struct list_ctx*)p;
  if (c->at < c->cap) {
    c->tri[3 * c->at] = t[0];
    c->tri[3 * c->at + 1] = t[1];
    c->tri[3 * c->at + 2] = t[2];
  }
  c->at++;
}

/* Triangle finding: writes the first min(T, cap) triangles found (each as
 * three ascending ids) to tri[3 * cap]; *T is the total. */
int oracle_list_triangles(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int32_t* tri,
                          int64_t cap, int64_t* T) {
  if (cap < 0 || (cap > 0 && !tri)) return OR_EINVAL;
  struct list_ctx c = {tri, cap, 0};
  return enumerate(n, off, cols, L, emit_list, &c, T);
}

struct support_ctx {
  const int64_t* off;
  const int32_t* cols;
  int64_t* support;
};

static void add_edge(struct support_ctx* c, int32_t a, int32_t b) {
  c->support[find_in_row(c->off, c->cols, a, b)]++;
  c->support[find_in_row(c->off, c->cols, b, a)]++;
}

static void emit_support(void* p, const int32_t* t) {
  struct support_ctx* c = (struct support_ctx*)p;
  add_edge(c, t[0], t[1]);
  add_edge(c, t[0], t[2]);
  add_edge(c, t[1], t[2]);
}

/* Triangles on each edge: support[e] for every CSR entry e (both
 * orientations of an edge hold the same number). */
int oracle_edge_supports(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int64_t* support) {
  if (n < 0 || !off) return OR_EINVAL;
  int64_t nnz = n > 0 ? off[n] : 0;
  if (nnz > 0 && !support) return OR_EINVAL;
  for (int64_t e = 0; e < nnz; ++e) support[e] = 0;
  struct support_ctx c = {off, cols, support};
  int64_t T = 0;
  return enumerate(n, off, cols, L, emit_support, &c, &T);
}

/* Plain edge iterator, direction-oriented by vertex id: every edge (u, v)
 * with u < v counts the common neighbours w > v.  Each triangle a < b < c is
 * found exactly once, at edge (a, b). */
int64_t oracle_edge_count(int64_t n, const int64_t* off, const int32_t* cols) {
  int64_t total = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t i = off[u]; i < off[u + 1]; ++i) {
      int32_t v = cols[i];
      if (v <= u) continue;
      int64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1];
      while (a < ae && b < be) {
        if (cols[a] < cols[b]) ++a;
        else if (cols[a] > cols[b]) ++b;
        else {
          if (cols[a] > v) ++total;
          ++a;
          ++b;
        }
      }
    }
  }
  return total;
}
