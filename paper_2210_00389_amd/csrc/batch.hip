// batch.hip -- tc_count_batch: Alg. 1 on many small graphs (n <= 65536 each)
// in two kernels that issue no host synchronisation and no memset, so a
// caller can capture the whole call in one hipGraph.
//
// Kernel 1 (one block per graph): BFS levels of Alg. 1 with the level array
// resident in LDS as uint16 (128 KB for 65536 vertices).  The first root is
// the highest-degree vertex (smallest id on ties); every other component is
// then searched from its smallest unvisited id, as in the scan order of
// Alg. 1, and isolated vertices get level 0.  Each level is one pass over the
// vertices: top-down from the frontier (vertices of degree above kBigDeg are
// expanded by a whole wave) or, when the last level was large, bottom-up.
// The block writes the level parity as a bit array (Lemma 1: for adjacent
// vertices L(x) = L(y) iff their parities agree, so the parity is all the
// count needs), the optional int32 levels, and the graph's work pieces:
// piece p is the range [p * piece, (p + 1) * piece) of the graph's CSR
// entries, so a vertex of large degree is spread over several pieces.
//
// Kernel 2 (persistent blocks of 256 or 512 threads claiming pieces from a
// counter, or one 64-thread block per piece): a wave takes one
// vertex u of the piece at a time, sets the bits of N(u) in its own
// 65536-bit LDS bitmap, and for every cover edge (u, v), v > u with equal
// parity, whose entry v of N(u) lies in the piece, streams N(v) in
// chunks of kBChunk consecutive entries per lane (the stream of a lane's
// chunk comes from a 64-bit mask of stream starts, no search) and counts the
// w whose bit is set and that pass the test of Alg. 1 (parity of w differs
// from u's, or w > v).  Counts and
// |H| are reduced per block and added to the graph's outputs.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kBfsThreads = 1024;
constexpr uint16_t kUnvisited = 0xFFFF;
constexpr int kBigDeg = 64;      // frontier vertices above this degree are expanded by a wave
constexpr int kBigCap = 1024;    // LDS list of such vertices per pass (overflow: expanded by the thread)
constexpr int kRowLoads = 8;     // row entries a thread loads at once in the level passes
constexpr int kBitmapWords = TC_BATCH_MAX_N / 32;
constexpr int kPieceMin = 1024;  // smallest piece size accepted (sizes the piece slots)
constexpr int kSmallPieceMin = 16;  // the same for the one-graph path of tc_count
constexpr int kClaim = 2;        // pieces a block of 256 or 512 threads claims at once

// Piece slots of graph g start at row_offsets[vbase[g]] / piece + g, parity
// words at vbase[g] / 32 + g: both leave room for ceil(size / unit) entries.
__device__ __forceinline__ int64_t piece_base(int64_t e0, int piece, int g) { return e0 / piece + g; }
__device__ __forceinline__ int64_t parity_base(int64_t v0, int g) { return v0 / 32 + g; }

__device__ __forceinline__ int64_t block_max_i64(int64_t v, int64_t* sh) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (lane() == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t m = sh[0];
    for (int i = 1; i < nw; ++i) m = sh[i] > m ? sh[i] : m;
    sh[nw] = m;
  }
  __syncthreads();
  const int64_t r = sh[nw];
  __syncthreads();
  return r;
}

// Level-synchronous BFS over the vertices already set to level `base`
// (the roots), with L resident in LDS.
__device__ void bfs_levels_lds(uint16_t* L, const int64_t* rows, const int32_t* cols, int n, int* s_cnt,
                               int32_t* s_big, int* s_nbig, int roots) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wv = tid / kWave, nw = nt / kWave, ln = lane();
  int level = 0;
  int last = roots;  // vertices found at the previous level
  for (;;) {
    const bool bottom_up = last > n / 32;
    if (tid == 0) {
      *s_cnt = 0;
      *s_nbig = 0;
    }
    __syncthreads();
    int found = 0;
    const uint16_t cur = static_cast<uint16_t>(level), nxt = static_cast<uint16_t>(level + 1);
    // rows are read kRowLoads entries at a time (independent loads in
    // flight together); a bottom-up scan stops after the group holding the
    // first parent
    if (bottom_up) {
      for (int i = tid; i < n; i += nt) {
        if (L[i] != kUnvisited) continue;
        const int64_t e = rows[i + 1];
        for (int64_t k = rows[i]; k < e; k += kRowLoads) {
          int32_t w[kRowLoads];
#pragma unroll
          for (int q = 0; q < kRowLoads; ++q) w[q] = k + q < e ? cols[k + q] : -1;
          bool hit = false;
#pragma unroll
          for (int q = 0; q < kRowLoads; ++q) hit |= w[q] >= 0 && L[w[q]] == cur;
          if (hit) {
            L[i] = nxt;
            ++found;
            break;
          }
        }
      }
    } else {
      for (int i = tid; i < n; i += nt) {
        if (L[i] != cur) continue;
        const int64_t b = rows[i], e = rows[i + 1];
        if (e - b > kBigDeg) {
          const int q = atomicAdd(s_nbig, 1);
          if (q < kBigCap) {
            s_big[q] = i;
            continue;
          }
        }
        for (int64_t k = b; k < e; k += kRowLoads) {
          int32_t w[kRowLoads];
#pragma unroll
          for (int q = 0; q < kRowLoads; ++q) w[q] = k + q < e ? cols[k + q] : -1;
#pragma unroll
          for (int q = 0; q < kRowLoads; ++q)
            if (w[q] >= 0 && L[w[q]] == kUnvisited) {
              L[w[q]] = nxt;
              ++found;
            }
        }
      }
      __syncthreads();
      const int nbig = min(*s_nbig, kBigCap);
      // a listed row is expanded by one wave, kRowLoads entries a lane at a
      // time (independent loads in flight)
      for (int q = wv; q < nbig; q += nw) {
        const int i = s_big[q];
        const int64_t e = rows[i + 1];
        for (int64_t k0 = rows[i] + ln; k0 < e; k0 += static_cast<int64_t>(kWave) * kRowLoads) {
          int32_t w[kRowLoads];
#pragma unroll
          for (int u = 0; u < kRowLoads; ++u) {
            const int64_t k = k0 + static_cast<int64_t>(u) * kWave;
            w[u] = k < e ? cols[k] : -1;
          }
#pragma unroll
          for (int u = 0; u < kRowLoads; ++u)
            if (w[u] >= 0 && L[w[u]] == kUnvisited) {
              L[w[u]] = nxt;
              ++found;
            }
        }
      }
    }
    // `found` may count a vertex more than once in the top-down pass (two
    // parents in one level); it only steers the direction and the stop test
    found = wave_sum(found);
    if (ln == 0 && found) atomicAdd(s_cnt, found);
    __syncthreads();
    last = *s_cnt;
    __syncthreads();
    if (last == 0) break;
    ++level;
  }
}

// root0 >= 0 replaces the default root of graph 0 (the one-graph path of
// tc_count); batches pass -1.
__global__ __launch_bounds__(kBfsThreads) void batch_bfs_kernel(const int64_t* vbase, const int64_t* row_offsets,
                                                                const int32_t* cols, int piece, int32_t* levels,
                                                                uint32_t* parity, int4* pieces, int64_t* T,
                                                                int64_t* H, int32_t root0) {
  __shared__ uint16_t L[TC_BATCH_MAX_N];
  __shared__ int32_t s_big[kBigCap];
  __shared__ int64_t sh[kBfsThreads / kWave + 1];
  __shared__ int s_cnt, s_nbig;
  const int g = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t v0 = vbase[g];
  const int n = static_cast<int>(vbase[g + 1] - v0);
  const int64_t* rows = row_offsets + v0;  // rows[i] = global position of local row i
  const int64_t e0 = rows[0];
  // a graph beyond the on-chip level array is skipped and flagged with -1
  // (the host rejects it first when validation is on); it gets no pieces
  const bool too_big = n > TC_BATCH_MAX_N;
  if (tid == 0) {
    T[g] = too_big ? -1 : 0;
    if (H) H[g] = too_big ? -1 : 0;
  }
  if (n <= 0 || too_big) return;
  // root: highest degree, smallest id on ties; isolated vertices get level 0
  int64_t key = -1;
  for (int i = tid; i < n; i += nt) {
    const int64_t d = rows[i + 1] - rows[i];
    L[i] = d == 0 ? 0 : kUnvisited;
    const int64_t k = (d << 32) | static_cast<int64_t>(0xFFFFFFFFu - static_cast<uint32_t>(i));
    key = k > key ? k : key;
  }
  key = block_max_i64(key, sh);
  const int root = (g == 0 && root0 >= 0 && root0 < n)
                       ? root0
                       : static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFF));
  __syncthreads();
  if (tid == 0) L[root] = 0;  // a given root of degree 0 is level 0 already
  __syncthreads();
  bfs_levels_lds(L, rows, cols, n, &s_cnt, s_big, &s_nbig, 1);
  // remaining components, each from its smallest unvisited id; every id
  // below the last such root is visited, so each scan starts there
  int from = 0;
  for (;;) {
    int64_t cand = -1;  // max of (n - i) over unvisited i = smallest i
    for (int i = from + tid; i < n; i += nt)
      if (L[i] == kUnvisited) {
        cand = n - i;
        break;
      }
    cand = block_max_i64(cand, sh);
    if (cand < 0) break;
    from = static_cast<int>(n - cand);
    if (tid == 0) L[from] = 0;
    __syncthreads();
    bfs_levels_lds(L, rows, cols, n, &s_cnt, s_big, &s_nbig, 1);
  }
  // outputs: parity bits, levels, pieces
  uint32_t* par = parity + parity_base(v0, g);
  const int words = (n + 31) / 32;
  for (int wi = tid; wi < words; wi += nt) {
    uint32_t b = 0;
    for (int j = 0; j < 32; ++j) {
      const int i = wi * 32 + j;
      if (i < n) b |= static_cast<uint32_t>(L[i] & 1) << j;
    }
    par[wi] = b;
  }
  if (levels)
    for (int i = tid; i < n; i += nt) levels[v0 + i] = L[i];
  const int64_t nnz = rows[n] - e0;
  const int64_t np = (nnz + piece - 1) / piece;
  int4* pc = pieces + piece_base(e0, piece, g);
  for (int64_t p = tid; p < np; p += nt) {
    // piece p holds the entries [ps, ps + piece): its vertices run from the
    // one whose row holds entry ps (the last row starting at or before it;
    // rows[n] > ps, so that row is not empty) up to the last row starting
    // before ps + piece (ve: the first row starting at or after it, or n)
    const int64_t ps = e0 + p * piece;
    const int vb = static_cast<int>(upper_bound_dev(rows, 0, static_cast<int64_t>(n) + 1, ps)) - 1;
    const int ve = static_cast<int>(lower_bound_dev(rows, 0, static_cast<int64_t>(n), ps + piece));
    pc[p] = make_int4(g, vb, ve, static_cast<int>(p));
  }
}

__device__ __forceinline__ uint32_t par_bit(const uint32_t* p, int32_t i) { return (p[i >> 5] >> (i & 31)) & 1u; }

constexpr int kBChunk = 8;  // consecutive list entries a lane takes at once

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
  uint32_t lo = static_cast<uint32_t>(x), hi = static_cast<uint32_t>(x >> 32);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    lo |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(lo), d, kWave));
    hi |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(hi), d, kWave));
  }
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// One chunk of up to 64 neighbours v = N(u)[base + lane], kept when base +
// lane lies in [klo, khi), of vertex u, in one
// wave: the cover edges (u, v), v > u with u's parity, are compacted into
// this wave's LDS lists (s_beg / s_v / s_off / s_len) and their lists N(v)
// streamed in chunks of kBChunk entries per lane, each entry w counted when
// its bit is set in the wave's bitmap of N(u) and it passes the test of
// Alg. 1 (parity of w differs from u's, or w > v).  A short row (du <= 64)
// passes its neighbours in registers (nbr, one per lane).
__device__ __forceinline__ void count_chunk(int u, int64_t ru, int64_t klo, int64_t khi, int64_t base, bool shortrow,
                                            int32_t nbr,
                                            uint32_t pu, const int64_t* rows, const int32_t* cols,
                                            const uint32_t* s_par, const uint32_t* bm, int64_t* s_beg, int32_t* s_v,
                                            int32_t* s_off, int32_t* s_len, int64_t& cnt, int64_t& hc) {
  const int ln = lane();
  const int64_t k = base + ln;
  int32_t v = -1;
  int len = 0;
  int64_t vb = 0;
  if (k >= klo && k < khi) {
    v = shortrow ? nbr : cols[ru + k];
    if (v > u && par_bit(s_par, v) == pu) {
      vb = rows[v];
      len = static_cast<int>(rows[v + 1] - vb);
      ++hc;
    }
  }
  // N(v) of these edges in chunks of kBChunk consecutive entries; the
  // non-empty streams are compacted in LDS with their first chunk
  const int nch = (len + kBChunk - 1) / kBChunk;
  const uint64_t ne = __ballot(nch > 0);
  const int incl = wave_incl_scan(nch);
  const int cst = incl - nch;
  const int C = __shfl(incl, kWave - 1, kWave);
  if (nch > 0) {
    const int r = __popcll(ne & lanemask_lt());
    s_beg[r] = vb;
    s_v[r] = v;
    s_off[r] = cst;
    s_len[r] = len;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int t0 = 0; t0 < C; t0 += kWave) {
    // streams whose first chunk lies in [t0, t0 + 64): a 64-bit mask of
    // those first chunks, and the number of streams begun before t0; lane
    // i's chunk t0 + i then belongs to stream before + |{starts <= i}| - 1
    const bool starts_here = nch > 0 && cst >= t0 && cst < t0 + kWave;
    const uint64_t M = wave_or_u64(starts_here ? (1ull << (cst - t0)) : 0ull);
    const int before = __popcll(__ballot(nch > 0 && cst < t0));
    const int c = t0 + ln;
    if (c < C) {
      const int j = before + __popcll(M & ((2ull << ln) - 1ull)) - 1;
      const int kk = c - s_off[j];
      const int64_t p0 = s_beg[j] + static_cast<int64_t>(kk) * kBChunk;
      const int rem = s_len[j] - kk * kBChunk;
      const int32_t vv = s_v[j];
      int32_t w[kBChunk];
#pragma unroll
      for (int q = 0; q < kBChunk; ++q) w[q] = q < rem ? cols[p0 + q] : -1;
#pragma unroll
      for (int q = 0; q < kBChunk; ++q)
        if (w[q] >= 0 && ((bm[w[q] >> 5] >> (w[q] & 31)) & 1u) && (par_bit(s_par, w[q]) != pu || w[q] > vv))
          ++cnt;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Vertices with more than kLongDeg neighbours inside the piece are left to
// a phase at the end of the piece in which every wave of the block takes a
// share of their 64-neighbour chunks (each wave with its own bitmap of
// N(u)), so one hub does not keep a single wave busy while the others wait.
constexpr int kLongDeg = 4 * kWave;
constexpr int kLongCap = 64;  // deferred vertices per piece (more: counted by the claiming wave)

template <int THREADS>
__global__ __launch_bounds__(THREADS) void batch_count_kernel(const int64_t* vbase, const int64_t* row_offsets,
                                                              const int32_t* cols, const uint32_t* parity,
                                                              const int4* pieces, int64_t nslots, int piece,
                                                              int claim_n, unsigned long long* ctr, int64_t* T,
                                                              int64_t* H) {
  constexpr int NW = THREADS / kWave;
  __shared__ uint32_t s_bm[NW][kBitmapWords];
  __shared__ int32_t s_off[NW][kWave];  // first chunk of each compacted stream
  __shared__ int32_t s_len[NW][kWave];
  __shared__ int64_t s_beg[NW][kWave];
  __shared__ int32_t s_v[NW][kWave];
  __shared__ int64_t sh[NW + 1];
  __shared__ int32_t s_long[kLongCap];
  __shared__ unsigned long long s_claim;
  __shared__ int s_next, s_nlong;
  const int tid = threadIdx.x, wv = tid / kWave, ln = lane();
  uint32_t* bm = s_bm[wv];
  for (int i = ln; i < kBitmapWords; i += kWave) bm[i] = 0u;
  // claim_n > 0: persistent blocks claim claim_n slots at a time from the
  // counter; claim_n = 0: block b takes slot b alone (one block per slot,
  // no shared counter for a single small graph's many one-wave blocks)
  if (tid == 0)
    s_claim = claim_n > 0 ? atomicAdd(ctr, static_cast<unsigned long long>(claim_n))
                          : static_cast<unsigned long long>(blockIdx.x);
  __syncthreads();
  unsigned long long claim = s_claim;
  while (claim < static_cast<unsigned long long>(nslots)) {
    unsigned long long next = 0;
    if (tid == 0)
      next = claim_n > 0 ? atomicAdd(ctr, static_cast<unsigned long long>(claim_n))
                         : static_cast<unsigned long long>(nslots);
    const unsigned long long cend =
        min(claim + static_cast<unsigned long long>(claim_n > 0 ? claim_n : 1), static_cast<unsigned long long>(nslots));
    for (unsigned long long sl = claim; sl < cend; ++sl) {
      const int4 pc = pieces[sl];
      if (pc.x < 0 || pc.y >= pc.z) continue;  // empty slot (block-uniform)
      const int g = pc.x;
      const int64_t v0 = vbase[g];
      const int64_t* rows = row_offsets + v0;
      // the graph's parity bits stay in global memory (at most 8 KB, cached):
      // keeping them out of LDS leaves room for more blocks per CU
      const uint32_t* s_par = parity + parity_base(v0, g);
      // the piece's entries [ps, ps + piece): vertex u takes the neighbours
      // N(u)[k] with ru + k inside them (its whole row sets the bitmap)
      const int64_t ps = rows[0] + static_cast<int64_t>(pc.w) * piece;
      if (tid == 0) {
        s_next = pc.y;
        s_nlong = 0;
      }
      __syncthreads();
      int64_t cnt = 0, hc = 0;
      // one vertex ahead: the next vertex's row bounds, and for a row of at
      // most 64 entries its neighbours, are loaded while the current vertex
      // is counted; a short row's neighbours stay in registers (one a lane)
      int u = 0;
      if (ln == 0) u = atomicAdd(&s_next, 1);
      u = __shfl(u, 0, kWave);
      int64_t ru = 0, du = 0;
      int32_t nbr = -1;
      if (u < pc.z) {
        ru = rows[u];
        du = rows[u + 1] - ru;
        if (du <= kWave && ln < du) nbr = cols[ru + ln];
      }
      while (u < pc.z) {
        int un = 0;
        if (ln == 0) un = atomicAdd(&s_next, 1);
        un = __shfl(un, 0, kWave);
        int64_t run = 0, dun = 0;
        if (un < pc.z) {
          run = rows[un];
          dun = rows[un + 1] - run;
        }
        const int64_t klo = ps > ru ? ps - ru : 0;
        const int64_t khi = ps + piece - ru < du ? ps + piece - ru : du;
        int deferred = 0;
        if (khi - klo > kLongDeg) {
          if (ln == 0) {
            const int q = atomicAdd(&s_nlong, 1);
            if (q < kLongCap) {
              s_long[q] = u;
              deferred = 1;
            }
          }
          deferred = __shfl(deferred, 0, kWave);
        }
        if (!deferred) {
          const uint32_t pu = par_bit(s_par, u);
          const bool shortrow = du <= kWave;
          if (shortrow) {
            if (nbr >= 0) atomicOr(&bm[nbr >> 5], 1u << (nbr & 31));
          } else {
            for (int64_t k = ln; k < du; k += kWave) {
              const int32_t w = cols[ru + k];
              atomicOr(&bm[w >> 5], 1u << (w & 31));
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          // a short row's neighbours sit in lanes 0 .. du - 1 (one chunk
          // from 0); a long row's chunks start at klo
          for (int64_t base = shortrow ? 0 : klo; base < khi; base += kWave)
            count_chunk(u, ru, klo, khi, base, shortrow, nbr, pu, rows, cols, s_par, bm, s_beg[wv], s_v[wv],
                        s_off[wv], s_len[wv], cnt, hc);
          if (shortrow) {
            if (nbr >= 0) bm[nbr >> 5] = 0u;
          } else {
            for (int64_t k = ln; k < du; k += kWave) bm[cols[ru + k] >> 5] = 0u;
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        // the next vertex's neighbours (short rows) for the next round
        int32_t nbn = -1;
        if (un < pc.z && dun <= kWave && ln < dun) nbn = cols[run + ln];
        u = un;
        ru = run;
        du = dun;
        nbr = nbn;
      }
      // the deferred long rows: every wave sets N(u) in its own bitmap and
      // takes the chunks wv, wv + NW, ... of N(u)
      __syncthreads();
      const int nlong = min(s_nlong, kLongCap);
      for (int j = 0; j < nlong; ++j) {
        const int lu = s_long[j];
        const int64_t lr = rows[lu], ld = rows[lu + 1] - lr;
        const int64_t klo = ps > lr ? ps - lr : 0;
        const int64_t khi = ps + piece - lr < ld ? ps + piece - lr : ld;
        const uint32_t pu = par_bit(s_par, lu);
        for (int64_t k = ln; k < ld; k += kWave) {
          const int32_t w = cols[lr + k];
          atomicOr(&bm[w >> 5], 1u << (w & 31));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int64_t base = klo + static_cast<int64_t>(wv) * kWave; base < khi;
             base += static_cast<int64_t>(NW) * kWave)
          count_chunk(lu, lr, klo, khi, base, false, -1, pu, rows, cols, s_par, bm, s_beg[wv], s_v[wv], s_off[wv],
                      s_len[wv], cnt, hc);
        for (int64_t k = ln; k < ld; k += kWave) bm[cols[lr + k] >> 5] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      cnt = block_sum(cnt, sh);
      hc = block_sum(hc, sh);
      if (tid == 0) {
        if (cnt) atomicAdd(reinterpret_cast<unsigned long long*>(&T[g]), static_cast<unsigned long long>(cnt));
        if (hc && H) atomicAdd(reinterpret_cast<unsigned long long*>(&H[g]), static_cast<unsigned long long>(hc));
      }
    }
    __syncthreads();
    if (tid == 0) s_claim = next;
    __syncthreads();
    claim = s_claim;
  }
}

// Clears the claim counters and marks every piece slot empty, in one launch;
// the one-graph path of tc_count also has its vertex bases {0, n} written
// here (vbase not null).
__global__ void batch_prep_kernel(unsigned long long* ctr, int4* pieces, int64_t nslots, int64_t* vbase,
                                  int64_t one_n) {
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t0 < 4) ctr[t0] = 0ull;
  if (vbase && t0 == 0) {
    vbase[0] = 0;
    vbase[1] = one_n;
  }
  for (int64_t i = t0; i < nslots; i += (int64_t)gridDim.x * blockDim.x) pieces[i] = make_int4(-1, 0, 0, 0);
}

struct BatchPlan {
  uint32_t* parity;
  int4* pieces;
  unsigned long long* ctr;
  int64_t nslots_cap;
  size_t bytes;
};

BatchPlan plan_batch(void* base, int64_t total_n, int64_t total_nnz, int32_t G, int piece_min = kPieceMin) {
  BatchPlan p;
  Carver c(base);
  p.ctr = c.take<unsigned long long>(4);
  p.parity = c.take<uint32_t>(total_n / 32 + G + 2);
  p.nslots_cap = total_nnz / piece_min + G + 2;
  p.pieces = c.take<int4>(p.nslots_cap);
  p.bytes = c.used();
  return p;
}

template <int THREADS>
int launch_count(const tc_batch* b, const BatchPlan& p, int64_t nslots, int piece, int blocks_per_cu, int64_t* T,
                 int64_t* H, hipStream_t s) {
  // persistent blocks, no more than there are piece slots to claim; or,
  // for one-wave blocks, one block per slot with no shared counter (the
  // pieces of a single small graph then spread over as many waves as there
  // are pieces, and no claim waits on thousands of others) while that grid
  // stays far below 2^32 work-items
  const int claim_n = THREADS == kWave && nslots <= (int64_t(1) << 24) ? 0 : kClaim;
  const int64_t full = static_cast<int64_t>(num_cus()) * blocks_per_cu;
  const int64_t want = claim_n > 0 ? (nslots + claim_n - 1) / claim_n : nslots;
  const int64_t blocks = claim_n == 0 || want < full ? want : full;
  batch_count_kernel<THREADS><<<static_cast<unsigned>(blocks), THREADS, 0, s>>>(
      b->vbase, b->row_offsets, b->cols, p.parity, p.pieces, nslots, piece, claim_n, p.ctr, T, H);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace

size_t batch_ws_bytes(int64_t total_n, int64_t total_nnz, int32_t num_graphs, int piece_min) {
  return plan_batch(nullptr, total_n, total_nnz, num_graphs, piece_min).bytes;
}

namespace {

// The launches of a batch (tuning checked here, validation done by the
// caller); one_vbase: the one-graph path's vertex bases, written first.
int batch_launch(const tc_batch* b, const tc_tuning* t, int64_t* triangles, int64_t* h_count, int32_t* levels,
                 void* ws, size_t ws_bytes, hipStream_t s, int32_t root0, int piece_min, int64_t* one_vbase) {
  const int G = b->num_graphs;
  int threads = 256, piece = 16384, bpc = 0;
  if (t) {
    if (t->batch_block) threads = t->batch_block;
    if (t->batch_piece) piece = t->batch_piece;
    bpc = t->batch_blocks_per_cu;
  }
  if (threads != kWave && threads != 256 && threads != 512)
    return fail(TC_ERR_INVALID_ARG, "tc_count_batch: batch_block must be 64, 256 or 512 (got %d)", threads);
  if (piece < piece_min) return fail(TC_ERR_INVALID_ARG, "tc_count_batch: batch_piece must be >= %d", piece_min);
  // LDS per block: one bitmap per wave of 8 KB, plus staging
  const int max_bpc = threads == kWave ? 16 : (threads == 256 ? 4 : 2);  // blocks that fit a CU's LDS
  if (bpc <= 0 || bpc > max_bpc) bpc = max_bpc;
  BatchPlan p = plan_batch(ws, b->total_vertices, b->total_nnz, G, piece_min);
  if (ws_bytes < p.bytes) return fail(TC_ERR_WORKSPACE, "tc_count_batch: workspace %zu < %zu", ws_bytes, p.bytes);
  const int64_t nslots = b->total_nnz / piece + G + 2;
  prof_stage("batch_bfs");
  batch_prep_kernel<<<grid_for(nslots, 256, 8192), 256, 0, s>>>(p.ctr, p.pieces, nslots, one_vbase,
                                                                 b->total_vertices);
  TC_HIP(hipGetLastError());
  batch_bfs_kernel<<<static_cast<unsigned>(G), kBfsThreads, 0, s>>>(b->vbase, b->row_offsets, b->cols, piece, levels,
                                                                    p.parity, p.pieces, triangles, h_count, root0);
  TC_HIP(hipGetLastError());
  prof_stage("batch_count");
  if (threads == kWave) TC_TRY(launch_count<kWave>(b, p, nslots, piece, bpc, triangles, h_count, s));
  else if (threads == 256) TC_TRY(launch_count<256>(b, p, nslots, piece, bpc, triangles, h_count, s));
  else TC_TRY(launch_count<512>(b, p, nslots, piece, bpc, triangles, h_count, s));
  return TC_OK;
}

}  // namespace

int batch_run(const tc_batch* b, const tc_tuning* t, uint32_t flags, int64_t* triangles, int64_t* h_count,
              int32_t* levels, void* ws, size_t ws_bytes, hipStream_t s, int32_t root0, int piece_min) {
  if (b->num_graphs == 0) return TC_OK;
  if (flags & TC_VALIDATE) TC_TRY(validate_batch_run(b, ws, s));
  return batch_launch(b, t, triangles, h_count, levels, ws, ws_bytes, s, root0, piece_min, nullptr);
}

namespace {

__global__ void small_stats_kernel(int64_t* stats, int64_t n, int64_t nnz, const int64_t* H) {
  for (int i = 0; i < 24; ++i) stats[i] = 0;
  stats[0] = n;
  stats[1] = nnz;
  stats[2] = *H;
}

struct SmallPlan {
  int64_t* stats;  // the tc_stats mirror, first in the workspace like the count plan's
  int64_t* vbase;  // {0, n}
  int64_t* h;      // |H| when the caller passes no h_count
  char* batch;
  size_t bytes;
};

SmallPlan plan_small(void* base, int64_t n, int64_t nnz) {
  SmallPlan p;
  Carver c(base);
  p.stats = c.take<int64_t>(24);
  p.vbase = c.take<int64_t>(2);
  p.h = c.take<int64_t>(1);
  p.batch = c.take<char>(0);
  p.bytes = c.used() + batch_ws_bytes(n, nnz, 1, kSmallPieceMin);
  return p;
}

}  // namespace

size_t small_ws_bytes(int64_t n, int64_t nnz) { return plan_small(nullptr, n, nnz).bytes; }

bool small_path_fits(int64_t n, int64_t nnz, int64_t max_n, int64_t max_nnz) {
  return n > 0 && n <= TC_BATCH_MAX_N && n <= max_n && nnz <= max_nnz;
}

int small_count_run(const tc_csr* g, int64_t root, int64_t* triangles, int64_t* h_count, int32_t* levels, void* ws,
                    size_t ws_bytes, hipStream_t s) {
  SmallPlan p = plan_small(ws, g->n, g->nnz);
  if (ws_bytes < p.bytes) return fail(TC_ERR_WORKSPACE, "tc_count: workspace %zu < %zu", ws_bytes, p.bytes);
  int64_t* H = h_count ? h_count : p.h;
  prof_stage("small_count");
  tc_batch b;
  b.num_graphs = 1;
  b.total_vertices = g->n;
  b.total_nnz = g->nnz;
  b.vbase = p.vbase;
  b.row_offsets = g->row_offsets;
  b.cols = g->cols;
  b.max_graph_vertices = static_cast<int32_t>(g->n);
  // one-wave counting blocks (sixteen per CU), each taking one piece at a
  // time, and pieces of one such block's share of the CSR entries (at least
  // kSmallPieceMin): a graph's vertices of large degree are cut across many
  // waves instead of keeping one block busy
  tc_tuning t{};
  t.batch_block = kWave;
  const int64_t share = g->nnz / (16 * static_cast<int64_t>(num_cus()));
  t.batch_piece = static_cast<int32_t>(share < kSmallPieceMin ? kSmallPieceMin : (share > 16384 ? 16384 : share));
  TC_TRY(batch_launch(&b, &t, triangles, H, levels, p.batch, p.bytes - (p.batch - static_cast<char*>(ws)), s,
                      static_cast<int32_t>(root), kSmallPieceMin, p.vbase));
  small_stats_kernel<<<1, 1, 0, s>>>(p.stats, g->n, g->nnz, H);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
