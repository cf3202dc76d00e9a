/*
 * oracle_checks.c -- a C driver that runs a subset of the oracle's pins with
 * the oracle (oracle/oracle.c) and the input generator (graphgen/graphgen.c)
 * compiled under AddressSanitizer and UndefinedBehaviorSanitizer (built and
 * run by tests/test_sanitize.py).  Test infrastructure: it checks the C
 * reference and the generator, never the GPU library.
 *
 * Pins exercised: closed forms (K_n: C(n,3) triangles, C(n-1,2) horizontal
 * edges; W_n: n-1 triangles and n-1 horizontal edges; C_n: 0 triangles,
 * |H| = n mod 2), the two intersection modes agreeing, the edge iterator
 * agreeing, per-vertex counts summing to 3T, edge supports summing to 6T,
 * the listing holding T triangles, strided row samples summing to T, the
 * validation codes of mutated CSRs, and the generators' graphs (R-MAT with a
 * relabel, Erdos-Renyi, Barabasi-Albert, Chung-Lu).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* oracle/oracle.c */
int oracle_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, int64_t* row_offsets,
                     int32_t* cols, int64_t* nnz_out);
int oracle_validate_csr(int64_t n, const int64_t* off, const int32_t* cols);
int oracle_bfs_levels(int64_t n, const int64_t* off, const int32_t* cols, int64_t root, int32_t* L,
                      int32_t* num_levels, int64_t* num_roots);
int64_t oracle_cover_edges(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int32_t* h_u,
                           int32_t* h_v);
int oracle_count(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode, int64_t* T,
                 int64_t* per_edge, int64_t* per_vertex);
int oracle_count_rows_strided(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int mode,
                              int64_t u_begin, int64_t u_end, int64_t stride, int64_t* T);
int oracle_list_triangles(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int32_t* tri,
                          int64_t cap, int64_t* count);
int oracle_edge_supports(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* L, int64_t* support);
int64_t oracle_edge_count(int64_t n, const int64_t* off, const int32_t* cols);
/* graphgen/graphgen.c */
void gg_rmat(int scale, int64_t num_edges, uint64_t ta, uint64_t tab, uint64_t tabc, uint64_t seed, int32_t* src,
             int32_t* dst);
void gg_permutation(int64_t n, uint64_t seed, int32_t* perm);
void gg_relabel(int64_t num_pairs, const int32_t* perm, int32_t* src, int32_t* dst);
int64_t gg_er(int64_t n, double p, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap);
int64_t gg_ba(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst);
int64_t gg_chung_lu(int64_t n, const double* w, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap);

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      fprintf(stderr, "FAILED: " __VA_ARGS__); \
      fprintf(stderr, "\n");                  \
      ++failures;                             \
    }                                         \
  } while (0)

typedef struct {
  int64_t n, nnz;
  int64_t* off;
  int32_t* cols;
} Csr;

static Csr build(int64_t n, int64_t np, const int32_t* s, const int32_t* d) {
  Csr c;
  c.n = n;
  c.off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  c.cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * np + 1));
  int rc = oracle_build_csr(n, np, s, d, c.off, c.cols, &c.nnz);
  CHECK(rc == 0, "build_csr status %d", rc);
  CHECK(oracle_validate_csr(n, c.off, c.cols) == 0, "validate of a built CSR");
  return c;
}

static void release(Csr* c) {
  free(c->off);
  free(c->cols);
}

/* Every cross-check of one graph; returns T. */
static int64_t check_graph(const Csr* c, const char* name) {
  const int64_t n = c->n;
  int32_t* L = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t nl = 0;
  int64_t roots = 0;
  CHECK(oracle_bfs_levels(n, c->off, c->cols, -1, L, &nl, &roots) == 0, "%s levels", name);
  for (int64_t u = 0; u < n; ++u)
    for (int64_t i = c->off[u]; i < c->off[u + 1]; ++i) {
      const int32_t dl = L[u] - L[c->cols[i]];
      CHECK(dl >= -1 && dl <= 1, "%s: edge across more than one level", name);
    }
  const int64_t h = oracle_cover_edges(n, c->off, c->cols, L, NULL, NULL);
  int32_t* hu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(h + 1));
  int32_t* hv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(h + 1));
  CHECK(oracle_cover_edges(n, c->off, c->cols, L, hu, hv) == h, "%s cover edges", name);
  int64_t T0 = -1, T1 = -2;
  int64_t* pv = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
  int64_t* pe = (int64_t*)calloc((size_t)(h + 1), sizeof(int64_t));
  CHECK(oracle_count(n, c->off, c->cols, L, 0, &T0, pe, pv) == 0, "%s count mode 0", name);
  CHECK(oracle_count(n, c->off, c->cols, L, 1, &T1, NULL, NULL) == 0, "%s count mode 1", name);
  CHECK(T0 == T1, "%s: modes disagree %lld %lld", name, (long long)T0, (long long)T1);
  CHECK(oracle_edge_count(n, c->off, c->cols) == T0, "%s: edge iterator disagrees", name);
  int64_t s = 0, se = 0;
  for (int64_t v = 0; v < n; ++v) s += pv[v];
  for (int64_t e = 0; e < h; ++e) se += pe[e];
  CHECK(s == 3 * T0 && se == T0, "%s: per-vertex or per-edge sums", name);
  int64_t parts = 0;
  for (int64_t ph = 0; ph < 7; ++ph) {
    int64_t t = 0;
    CHECK(oracle_count_rows_strided(n, c->off, c->cols, L, 0, ph < n ? ph : n, n, 7, &t) == 0, "%s strided", name);
    parts += t;
  }
  CHECK(parts == T0, "%s: strided samples do not sum to T", name);
  int64_t nt = 0;
  int32_t* tri = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * T0 + 3));
  CHECK(oracle_list_triangles(n, c->off, c->cols, L, tri, T0, &nt) == 0 && nt == T0, "%s listing", name);
  int64_t* sup = (int64_t*)calloc((size_t)(c->nnz + 1), sizeof(int64_t));
  CHECK(oracle_edge_supports(n, c->off, c->cols, L, sup) == 0, "%s supports", name);
  int64_t ss = 0;
  for (int64_t e = 0; e < c->nnz; ++e) ss += sup[e];
  CHECK(ss == 6 * T0, "%s: supports sum %lld, want 6T", name, (long long)ss);
  free(L);
  free(hu);
  free(hv);
  free(pv);
  free(pe);
  free(tri);
  free(sup);
  return T0;
}

static int64_t cover_h(const Csr* c) {
  int32_t* L = (int32_t*)malloc(sizeof(int32_t) * (size_t)(c->n + 1));
  oracle_bfs_levels(c->n, c->off, c->cols, -1, L, NULL, NULL);
  const int64_t h = oracle_cover_edges(c->n, c->off, c->cols, L, NULL, NULL);
  free(L);
  return h;
}

int main(void) {
  /* closed forms */
  for (int64_t k = 3; k <= 24; k += 7) {
    int64_t np = k * (k - 1) / 2, e = 0;
    int32_t* s = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    for (int64_t u = 0; u < k; ++u)
      for (int64_t v = u + 1; v < k; ++v) s[e] = (int32_t)u, d[e++] = (int32_t)v;
    Csr c = build(k, np, s, d);
    CHECK(check_graph(&c, "complete") == k * (k - 1) * (k - 2) / 6, "K%lld triangles", (long long)k);
    CHECK(cover_h(&c) == (k - 1) * (k - 2) / 2, "K%lld cover edges", (long long)k);
    release(&c);
    free(s);
    free(d);
  }
  for (int64_t k = 5; k <= 41; k += 9) { /* wheel: hub 0, rim 1..k-1 */
    int64_t np = 2 * (k - 1), e = 0;
    int32_t* s = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    for (int64_t r = 1; r < k; ++r) {
      s[e] = 0, d[e++] = (int32_t)r;
      s[e] = (int32_t)r, d[e++] = (int32_t)(r + 1 < k ? r + 1 : 1);
    }
    Csr c = build(k, np, s, d);
    CHECK(check_graph(&c, "wheel") == k - 1 && cover_h(&c) == k - 1, "W%lld", (long long)k);
    release(&c);
    free(s);
    free(d);
  }
  for (int64_t k = 4; k <= 9; ++k) { /* cycles */
    int32_t s[16], d[16];
    for (int64_t i = 0; i < k; ++i) s[i] = (int32_t)i, d[i] = (int32_t)((i + 1) % k);
    Csr c = build(k, k, s, d);
    CHECK(check_graph(&c, "cycle") == 0 && cover_h(&c) == (k & 1), "C%lld", (long long)k);
    release(&c);
  }
  /* generators */
  {
    const int scale = 9;
    const int64_t n = 1 << scale, np = 16 * n;
    const double two53 = 9007199254740992.0;
    int32_t* s = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)np);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    gg_rmat(scale, np, (uint64_t)(0.57 * two53), (uint64_t)(0.76 * two53), (uint64_t)(0.95 * two53), 7, s, d);
    gg_permutation(n, 7, perm);
    gg_relabel(np, perm, s, d);
    Csr c = build(n, np, s, d);
    CHECK(check_graph(&c, "rmat") > 0, "R-MAT has triangles");
    /* validation codes of mutated copies */
    int32_t* m = (int32_t*)malloc(sizeof(int32_t) * (size_t)c.nnz);
    int64_t row = 0;
    while (c.off[row + 1] - c.off[row] < 3) ++row;
    const int64_t a = c.off[row];
    memcpy(m, c.cols, sizeof(int32_t) * (size_t)c.nnz);
    m[a + 1] = m[a];
    CHECK(oracle_validate_csr(n, c.off, m) == -6, "duplicate");
    memcpy(m, c.cols, sizeof(int32_t) * (size_t)c.nnz);
    int32_t t = m[a];
    m[a] = m[a + 1];
    m[a + 1] = t;
    CHECK(oracle_validate_csr(n, c.off, m) == -5, "unsorted");
    memcpy(m, c.cols, sizeof(int32_t) * (size_t)c.nnz);
    m[a] = (int32_t)n;
    CHECK(oracle_validate_csr(n, c.off, m) == -4, "out of range");
    free(m);
    int32_t bad_s = 0, bad_d = (int32_t)n;
    int64_t nnz = 0;
    CHECK(oracle_build_csr(n, 1, &bad_s, &bad_d, c.off, c.cols, &nnz) == -4, "build rejects an id out of range");
    release(&c);
    free(s);
    free(d);
    free(perm);
  }
  {
    const int64_t n = 600, cap = 60000;
    int32_t* s = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t k = gg_er(n, 0.05, 11, s, d, cap);
    CHECK(k > 0, "ER pairs");
    Csr c = build(n, k, s, d);
    check_graph(&c, "er");
    release(&c);
    k = gg_ba(n, 6, 12, s, d);
    Csr b = build(n, k, s, d);
    check_graph(&b, "ba");
    release(&b);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) w[i] = 40.0 / (1.0 + 0.05 * (double)i);
    k = gg_chung_lu(n, w, 13, s, d, cap);
    CHECK(k > 0, "Chung-Lu pairs");
    Csr l = build(n, k, s, d);
    check_graph(&l, "chung_lu");
    release(&l);
    free(w);
    free(s);
    free(d);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitize ok\n");
  return 0;
}
