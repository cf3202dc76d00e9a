/*
 * graphgen.c -- seeded synthetic graph generators (edge-pair lists).
 *
 * This module only produces inputs.  It holds none of the triangle-counting
 * arithmetic; both the CPU oracle and the HIP library consume its output, and
 * each side cleans the pairs up (symmetrise, drop loops and duplicates, sort)
 * with its own code.
 *
 * Randomness: one counter-based stream per (seed, stream id), built from the
 * SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014; constants from Vigna's public
 * domain splitmix64.c).  Draw i of a stream is mix(key + (i+1)*gamma), so any
 * draw can be computed independently and OpenMP threads give the same output
 * as one thread.
 *
 * Families:
 *   R-MAT (Chakrabarti, Zhan and Faloutsos 2004), Graph500 quadrant recursion;
 *   Erdos-Renyi G(n,p) by geometric skipping (Batagelj and Brandes 2005);
 *   Barabasi-Albert by the Batagelj-Brandes endpoint-array method;
 *   Chung-Lu by the Miller-Hagberg skipping method (2011);
 *   a seeded Fisher-Yates permutation to relabel vertex ids.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of stream `stream` under `seed`. */
uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
  return gg_mix(gg_mix(seed + GG_GAMMA) ^ (stream * 0xD1B54A32D192ED03ULL + 0x8CB92BA72F3D8DD7ULL));
}

/* Draw number `ctr` of the stream with key `key`. */
uint64_t gg_draw(uint64_t key, uint64_t ctr) { return gg_mix(key + (ctr + 1) * GG_GAMMA); }

/* Uniform double in (0, 1): 53 random bits, offset by half an ulp so that
 * log() never sees 0. */
static inline double gg_unit(uint64_t key, uint64_t ctr) {
  return ((double)(gg_draw(key, ctr) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, bound) by a 128-bit multiply (bias < 2^-64*bound). */
static inline uint64_t gg_below(uint64_t key, uint64_t ctr, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)gg_draw(key, ctr) * bound) >> 64);
}

/* ------------------------------------------------------------------ R-MAT */
/* Each of the `scale` bit levels draws one 53-bit integer r and picks a
 * quadrant: r < ta -> (0,0); r < tab -> (0,1); r < tabc -> (1,0); else (1,1).
 * The row bit is set for quadrants c and d, the column bit for b and d.
 * Thresholds are floor(cumulative probability * 2^53), integers, so the output
 * does not depend on floating-point evaluation. */
void gg_rmat(int scale, int64_t num_edges, uint64_t ta, uint64_t tab, uint64_t tabc,
             uint64_t seed, int32_t* src, int32_t* dst) {
  const uint64_t key = gg_stream_key(seed, 0x524D4154ULL);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < num_edges; ++e) {
    uint32_t r = 0, c = 0;
    for (int b = 0; b < scale; ++b) {
      uint64_t x = gg_draw(key, (uint64_t)e * (uint64_t)scale + (uint64_t)b) >> 11;
      uint32_t rb, cb;
      if (x < ta) { rb = 0; cb = 0; }
      else if (x < tab) { rb = 0; cb = 1; }
      else if (x < tabc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      r = (r << 1) | rb;
      c = (c << 1) | cb;
    }
    src[e] = (int32_t)r;
    dst[e] = (int32_t)c;
  }
}

/* --------------------------------------------------------- permutation */
/* perm[i] = new id of vertex i; Fisher-Yates from the top, swap index drawn
 * from a stream of its own. */
void gg_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  const uint64_t key = gg_stream_key(seed, 0x5045524DULL);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)gg_below(key, (uint64_t)i, (uint64_t)(i + 1));
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* In-place relabel of both endpoint arrays. */
void gg_relabel(int64_t num_pairs, const int32_t* perm, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < num_pairs; ++e) {
    src[e] = perm[src[e]];
    dst[e] = perm[dst[e]];
  }
}

/* ------------------------------------------------------ Erdos-Renyi G(n,p) */
/* Row v (v >= 1) holds the pairs (v, w) with w < v.  Within a row the gaps
 * between kept pairs are geometric: skip = floor(log(1-u)/log(1-p)).  Each row
 * has its own stream so rows are independent.  Two passes (count, fill) use
 * identical draws.  Returns the number of pairs, or -needed when cap is too
 * small (nothing is written past cap). */
static inline uint64_t gg_row_key(uint64_t key, int64_t row) {
  return gg_mix(key + (uint64_t)row * 0xD1B54A32D192ED03ULL);
}

static int64_t er_row(uint64_t key, int64_t v, double lq, int32_t* s, int32_t* d, int64_t cap) {
  const uint64_t rk = gg_row_key(key, v);
  int64_t cnt = 0;
  int64_t w = -1;
  uint64_t ctr = 0;
  for (;;) {
    double u = gg_unit(rk, ctr);
    ++ctr;
    double sk = floor(log(u) / lq);
    if (sk > (double)v) break;
    w += 1 + (int64_t)sk;
    if (w >= v) break;
    if (s && cnt < cap) { s[cnt] = (int32_t)v; d[cnt] = (int32_t)w; }
    ++cnt;
  }
  return cnt;
}

int64_t gg_er(int64_t n, double p, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap) {
  if (n < 2 || p <= 0.0) return 0;
  if (p >= 1.0) {
    int64_t need = n * (n - 1) / 2;
    if (need > cap) return -need;
    int64_t k = 0;
    for (int64_t v = 1; v < n; ++v)
      for (int64_t w = 0; w < v; ++w) { src[k] = (int32_t)v; dst[k] = (int32_t)w; ++k; }
    return k;
  }
  const uint64_t key = gg_stream_key(seed, 0x45520000ULL);
  const double lq = log(1.0 - p);
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return 0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t v = 1; v < n; ++v) cnt[v + 1] = er_row(key, v, lq, NULL, NULL, 0);
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int64_t total = cnt[n];
  if (total > cap) { free(cnt); return -total; }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t v = 1; v < n; ++v)
    er_row(key, v, lq, src + cnt[v], dst + cnt[v], cnt[v + 1] - cnt[v]);
  free(cnt);
  return total;
}

/* -------------------------------------------------- Barabasi-Albert (m) */
/* Endpoint array M of length 2*n*m: for new vertex v and its i-th edge,
 * M[2k] = v and M[2k+1] = M[r] with r uniform in [0, 2k] (k = v*m + i).
 * The pairs (M[2k], M[2k+1]) are the edges; the first ones are self loops and
 * some repeat, which the consumer's cleanup removes.  Sequential by nature. */
int64_t gg_ba(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  const uint64_t key = gg_stream_key(seed, 0x42410000ULL);
  const int64_t total = n * m;
  int32_t* M = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * total));
  if (!M) return 0;
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t i = 0; i < m; ++i) {
      int64_t k = v * m + i;
      M[2 * k] = (int32_t)v;
      int64_t r = (int64_t)gg_below(key, (uint64_t)k, (uint64_t)(2 * k + 1));
      M[2 * k + 1] = M[r];
    }
  }
  for (int64_t k = 0; k < total; ++k) { src[k] = M[2 * k]; dst[k] = M[2 * k + 1]; }
  free(M);
  return total;
}

/* ------------------------------------------------------------ Chung-Lu */
/* Weights w[0] >= w[1] >= ... (caller sorts them), S = sum w.
 * p_uv = min(1, w_u w_v / S).  For each u, candidates v > u are visited by
 * geometric skips under the current upper bound p and accepted with
 * probability q/p (Miller and Hagberg).  One stream per u; two passes. */
static int64_t cl_row(uint64_t key, int64_t u, int64_t n, const double* w, double S,
                      int32_t* s, int32_t* d, int64_t cap) {
  const uint64_t rk = gg_row_key(key, u);
  int64_t cnt = 0;
  uint64_t ctr = 0;
  int64_t v = u + 1;
  double p = w[u] * w[v] / S;
  if (p > 1.0) p = 1.0;
  while (v < n && p > 0.0) {
    if (p != 1.0) {
      double r = gg_unit(rk, ctr);
      ++ctr;
      double sk = floor(log(r) / log(1.0 - p));
      if (sk > (double)n) break;
      v += (int64_t)sk;
    }
    if (v < n) {
      double q = w[u] * w[v] / S;
      if (q > 1.0) q = 1.0;
      double r = gg_unit(rk, ctr);
      ++ctr;
      if (r < q / p) {
        if (s && cnt < cap) { s[cnt] = (int32_t)u; d[cnt] = (int32_t)v; }
        ++cnt;
      }
      p = q;
      v += 1;
    }
  }
  return cnt;
}

int64_t gg_chung_lu(int64_t n, const double* w, uint64_t seed, int32_t* src, int32_t* dst, int64_t cap) {
  if (n < 2) return 0;
  const uint64_t key = gg_stream_key(seed, 0x434C0000ULL);
  double S = 0.0;
  for (int64_t i = 0; i < n; ++i) S += w[i];
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return 0;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t u = 0; u < n - 1; ++u) cnt[u + 1] = cl_row(key, u, n, w, S, NULL, NULL, 0);
  for (int64_t u = 0; u < n; ++u) cnt[u + 1] += cnt[u];
  int64_t total = cnt[n];
  if (total > cap) { free(cnt); return -total; }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t u = 0; u < n - 1; ++u)
    cl_row(key, u, n, w, S, src + cnt[u], dst + cnt[u], cnt[u + 1] - cnt[u]);
  free(cnt);
  return total;
}
