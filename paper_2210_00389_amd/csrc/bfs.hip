// bfs.hip -- BFS levels L(v) of Def. 2 with the root rule of Alg. 1:
// a BFS from r0 (given, or the largest-degree vertex with the smallest id on
// ties), then every component not reached is levelled from its smallest id.
//
// GPU structure (frontiers are bitmaps; three rotate so that the bitmap of
// the level after next is cleared while the current one is read):
//   * a top-down step lets every frontier vertex expand its row; rows above
//     kBig entries are listed and expanded edge-balanced by a second kernel
//     (flat edge index over the listed rows, so a hub's row is spread over
//     the whole grid); new vertices are claimed with an atomic OR on the
//     visited bitmap;
//   * a bottom-up step (Beamer et al.'s direction optimisation) lets every
//     unvisited vertex look for a neighbour in the frontier and stop at the
//     first hit; a wave composes its 64 vertices' bits with ballots;
//   * per-block counts (new vertices, their edges) go to an array that a
//     one-block kernel sums to decide the next direction (alpha 14, beta 24)
//     and the stop, all on the device; the host launches levels in groups
//     of kLevelsPerSync and reads the state once per group;
//   * the state counts the row entries of the vertices not yet reached; when
//     the BFS from r0 ends with none, every vertex left is isolated and takes
//     level 0 in one pass;
//   * otherwise the remaining components: union-find over the unreached vertices where
//     a root is always hooked under the smaller root, so every component's
//     final root is its smallest id; those roots then start one multi-source
//     BFS (components are disjoint, so the per-component distances are
//     exactly those of separate BFS runs).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t row_deg(const int64_t* off, int64_t v) { return off[v + 1] - off[v]; }

__global__ void root_key_kernel(const int64_t* off, int64_t n, unsigned long long* key) {
  unsigned long long best = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long d = static_cast<unsigned long long>(row_deg(off, v));
    // larger degree first, then smaller id
    unsigned long long k = (d << 32) | (0xFFFFFFFFull - static_cast<unsigned long long>(v));
    best = k > best ? k : best;
  }
  __shared__ unsigned long long sm[kThreads / kWave];
  best = wave_max(best);
  if (lane() == 0) sm[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kThreads / kWave; ++i) best = sm[i] > best ? sm[i] : best;
    if (best) atomicMax(key, best);
  }
}


// frontier rows above this length are expanded edge-balanced over the grid
// (a row below it is expanded by one wave: R-MAT S14's root, 3644 entries,
// took 0.12 ms that way under a bound of 4096, against 5 us listed)
constexpr int kBig = 1024;
constexpr int kBigCap = 4096;      // listed rows per level (more: expanded by their thread)
constexpr int kMaxParts = 4096;    // blocks of the step kernels (partials per kernel)
// levels launched between two reads of the state: six covers a small-world
// graph searched from a hub (R-MAT S10-S20 take 5-6; deeper graphs read the
// state again after six, and the levels past the stop cost a no-op launch each)
constexpr int kLevelsPerSync = 6;
constexpr int kLevelsPerSyncRest = 4;

// Device-side state of one BFS (see BfsWs::st).
struct BfsState {
  int64_t f, ef;         // frontier size and its row entries
  int64_t unexplored;    // row entries not yet in any frontier
  int64_t nbig;          // listed big rows of the current level
  int32_t level;         // level of the current frontier
  int32_t bottom_up;     // direction of the step that expands it
  int32_t prev_bu;       // direction of the previous step
  int32_t done;          // the frontier is empty
  int32_t num_levels;    // deepest level + 1 once done
  int32_t pad;
};

__device__ __forceinline__ uint32_t* bm_at(uint32_t* base, int64_t words, int32_t level, int k) {
  return base + static_cast<int64_t>((level + k) % 3) * words;
}

// Block sums of (new vertices, their entries) -> part[2 * blockIdx.x + 0/1].
__device__ __forceinline__ void block_partial(int64_t cnt, int64_t edg, int64_t* part, int64_t* sh) {
  cnt = block_sum(cnt, sh);
  edg = block_sum(edg, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = cnt;
    part[2 * blockIdx.x + 1] = edg;
  }
}

__global__ __launch_bounds__(kThreads) void step_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                                                        BfsState* st, int32_t* L, uint32_t* vis, uint32_t* bms,
                                                        int32_t* big, int64_t* part) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  __shared__ int32_t s_off[kThreads / kWave][kWave + 1];
  __shared__ int64_t s_beg[kThreads / kWave][kWave];
  const int64_t words = (n + 31) / 32 + 1;
  const int32_t level = st->level;
  int64_t cnt = 0, edg = 0;
  if (!st->done) {
    const uint32_t* cur = bm_at(bms, words, level, 0);
    uint32_t* nxt = bm_at(bms, words, level, 1);
    uint32_t* old = bm_at(bms, words, level, 2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < words; i += stride) old[i] = 0u;  // the bitmap of the level after next
    const int32_t nl = level + 1;
    if (st->bottom_up) {
      // 64 consecutive vertices per wave and round: words 2k, 2k+1 are this wave's
      for (int64_t v0 = (t0 / kWave) * kWave; v0 < n; v0 += stride) {
        const int64_t v = v0 + lane();
        bool take = false;
        if (v < n && !((vis[v >> 5] >> (v & 31)) & 1u)) {
          const int64_t b = off[v], e = off[v + 1];
          for (int64_t j = b; j < e; ++j) {
            const int32_t w = cols[j];
            if ((cur[w >> 5] >> (w & 31)) & 1u) {
              take = true;
              break;
            }
          }
          if (take) {
            L[v] = nl;
            ++cnt;
            edg += e - b;
          }
        }
        const uint64_t m = __ballot(take);
        if (m && (lane() & 31) == 0) {
          const uint32_t word = static_cast<uint32_t>(m >> lane());
          if (word) {
            nxt[v >> 5] |= word;
            vis[v >> 5] |= word;
          }
        }
      }
    } else {
      // 64 consecutive vertices per wave and round; the rows of the group's
      // frontier vertices are flattened across the lanes
      const int wv = threadIdx.x / kWave;
      for (int64_t v0 = (t0 / kWave) * kWave; v0 < n; v0 += stride) {
        const uint64_t fw = static_cast<uint64_t>(cur[v0 >> 5]) | (static_cast<uint64_t>(cur[(v0 >> 5) + 1]) << 32);
        if (fw == 0) continue;  // uniform per wave
        const int64_t v = v0 + lane();
        int64_t b = 0;
        int d = 0;
        if (((fw >> lane()) & 1ull) && v < n) {
          b = off[v];
          const int64_t e = off[v + 1];
          if (e - b > kBig) {
            const unsigned long long q = atomicAdd(reinterpret_cast<unsigned long long*>(&st->nbig), 1ull);
            if (q < static_cast<unsigned long long>(kBigCap)) big[q] = static_cast<int32_t>(v);
            else d = static_cast<int>(e - b);  // list full: flattened here
          } else {
            d = static_cast<int>(e - b);
          }
        }
        const int incl = wave_incl_scan(d);
        const int total = __shfl(incl, kWave - 1, kWave);
        s_off[wv][lane()] = incl - d;
        s_beg[wv][lane()] = b;
        if (lane() == 0) s_off[wv][kWave] = total;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int k = lane(); k < total; k += kWave) {
          int lo = 0, hi = kWave;  // last j with s_off[j] <= k
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[wv][mid] <= k) lo = mid;
            else hi = mid;
          }
          const int32_t w = cols[s_beg[wv][lo] + (k - s_off[wv][lo])];
          const uint32_t bit = 1u << (w & 31);
          if (load_relaxed(&vis[w >> 5]) & bit) continue;
          if (atomicOr(&vis[w >> 5], bit) & bit) continue;
          atomicOr(&nxt[w >> 5], bit);
          L[w] = nl;
          ++cnt;
          edg += off[w + 1] - off[w];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
  }
  block_partial(cnt, edg, part, sh);
}

// Top-down expansion of the listed big rows: flat entry index over them.
__global__ __launch_bounds__(kThreads) void big_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                                                       BfsState* st, int32_t* L, uint32_t* vis, uint32_t* bms,
                                                       const int32_t* big, int64_t* part) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  __shared__ int64_t s_pre[kBigCap + 1];
  const int64_t words = (n + 31) / 32 + 1;
  int64_t cnt = 0, edg = 0;
  const int64_t nb = min(st->nbig, static_cast<int64_t>(kBigCap));
  if (!st->done && !st->bottom_up && nb > 0) {
    uint32_t* nxt = bm_at(bms, words, st->level, 1);
    const int32_t nl = st->level + 1;
    // prefix of the listed rows' lengths (each block computes it)
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
      const int64_t i = b0 + threadIdx.x;
      const int64_t d = i < nb ? off[big[i] + 1] - off[big[i]] : 0;
      int64_t tot;
      const int64_t ex = block_excl_scan(d, sh, &tot);
      if (i < nb) s_pre[i] = run + ex;
      run += tot;
    }
    if (threadIdx.x == 0) s_pre[nb] = run;
    __syncthreads();
    const int64_t total = run;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
      int64_t lo = 0, hi = nb;  // last row with s_pre <= k
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (s_pre[mid] <= k) lo = mid;
        else hi = mid;
      }
      const int32_t v = big[lo];
      const int32_t w = cols[off[v] + (k - s_pre[lo])];
      const uint32_t bit = 1u << (w & 31);
      if (load_relaxed(&vis[w >> 5]) & bit) continue;
      if (atomicOr(&vis[w >> 5], bit) & bit) continue;
      atomicOr(&nxt[w >> 5], bit);
      L[w] = nl;
      ++cnt;
      edg += off[w + 1] - off[w];
    }
  }
  block_partial(cnt, edg, part, sh);
}

// Sums the partials of both kernels, decides the next step, advances.
__global__ __launch_bounds__(kThreads) void decide_kernel(int64_t n, BfsState* st, const int64_t* part,
                                                          int nparts) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  if (st->done) return;  // uniform
  int64_t cnt = 0, edg = 0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) {
    cnt += part[2 * i];
    edg += part[2 * i + 1];
  }
  cnt = block_sum(cnt, sh);
  edg = block_sum(edg, sh);
  if (threadIdx.x == 0) {
    const int64_t alpha = 14, beta = 24;
    st->prev_bu = st->bottom_up;
    st->nbig = 0;
    if (cnt == 0) {
      st->done = 1;
      st->num_levels = st->level + 1;
      st->f = 0;
      st->ef = 0;
      return;
    }
    st->level += 1;
    st->f = cnt;
    st->ef = edg;
    st->unexplored -= edg;
    // Beamer's rule on the new frontier
    st->bottom_up = !st->prev_bu ? (edg > st->unexplored / alpha && cnt > n / 256) : (cnt >= n / beta);
  }
}

// Initial state of a BFS whose level-0 frontier is already in the bitmap of
// level 0 (start_kernel or the component roots); counts from part.
__global__ __launch_bounds__(kThreads) void init_state_kernel(int64_t n, BfsState* st, const int64_t* part,
                                                              int nparts, int64_t unexplored) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t cnt = 0, edg = 0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) {
    cnt += part[2 * i];
    edg += part[2 * i + 1];
  }
  cnt = block_sum(cnt, sh);
  edg = block_sum(edg, sh);
  if (threadIdx.x == 0) {
    st->f = cnt;
    st->ef = edg;
    st->unexplored = (unexplored < 0 ? st->unexplored : unexplored) - edg;
    st->nbig = 0;
    st->level = 0;
    st->prev_bu = 0;
    st->bottom_up = edg > st->unexplored / 14 && cnt > n / 256;
    st->done = cnt == 0;
    st->num_levels = cnt == 0 ? 0 : 1;
  }
}

__global__ void copy_words_kernel(const uint32_t* src, uint32_t* dst, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Clears the state of a BFS in one launch: levels to -1, the visited and
// frontier bitmaps, the root key and the step kernels' partials.
__global__ void clear_state_kernel(int32_t* L, int64_t n, uint32_t* vis, int64_t words, uint32_t* bms,
                                   unsigned long long* key, int64_t* part, int64_t nparts) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n || i < 3 * words || i < nparts;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) L[i] = -1;
    if (i < words) vis[i] = 0u;
    if (i < 3 * words) bms[i] = 0u;
    if (i < nparts) part[i] = 0;
    if (i == 0) *key = 0ull;
  }
}

// Starts the BFS from one root (either the argmax key or a given root).
// The partials must be zero beforehand.
__global__ void start_kernel(const int64_t* off, const unsigned long long* key, int64_t given_root, int32_t* L,
                             uint32_t* vis, uint32_t* bm0, int64_t* part, int64_t* root_out) {
  int64_t r = given_root;
  if (r < 0) r = static_cast<int64_t>(0xFFFFFFFFull - (*key & 0xFFFFFFFFull));
  L[r] = 0;
  vis[r >> 5] |= 1u << (r & 31);
  bm0[r >> 5] |= 1u << (r & 31);
  part[0] = 1;
  part[1] = row_deg(off, r);
  *root_out = r;
}

// ------------------------------------------------- remaining components
// When the first BFS has reached every vertex with an edge, each vertex left
// is isolated and its own one-vertex BFS gives it level 0.
__global__ void isolated_kernel(const uint32_t* vis, int64_t n, int32_t* L) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (!((vis[v >> 5] >> (v & 31)) & 1u)) L[v] = 0;
}

__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    int32_t p = load_relaxed(&parent[x]);
    if (p == x) return x;
    int32_t gp = load_relaxed(&parent[p]);
    if (gp != p) __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
  }
}

// Hooks the larger root under the smaller, so parent[x] <= x always holds
// and the root of a finished component is its smallest vertex.
__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    int32_t old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
    b = old;  // b was hooked meanwhile: retry from its new parent
  }
}

__global__ void uf_init_kernel(int32_t* parent, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = static_cast<int32_t>(v);
}

__global__ void uf_hook_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                               const uint32_t* vis, int32_t* parent) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (vis[v >> 5] & (1u << (v & 31))) continue;
    for (int64_t j = off[v], e = off[v + 1]; j < e; ++j) {
      int32_t w = cols[j];
      if (w < v) uf_union(parent, static_cast<int32_t>(v), w);
    }
  }
}

// Roots of the unreached components start the multi-source BFS at level 0
// (bits in the level-0 frontier bitmap); isolated vertices get level 0 and
// need no expansion.  Per-block counts go to part.  A wave takes 64
// consecutive vertices from a multiple of 64, i.e. two whole bitmap words
// that no other wave of this kernel touches: its roots are gathered by
// ballot and one lane updates each word, with no atomics.
__global__ __launch_bounds__(kThreads) void uf_roots_kernel(const int64_t* off, int64_t n, int32_t* parent,
                                                            int32_t* L, uint32_t* vis, uint32_t* bm0,
                                                            int64_t* part) {
  static_assert(kThreads % kWave == 0, "waves start at multiples of 64 vertices");
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t cnt = 0, edg = 0;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = v0 + threadIdx.x;
    bool root = false, expand = false;
    if (v < n && !((vis[v >> 5] >> (v & 31)) & 1u) && uf_find(parent, static_cast<int32_t>(v)) == v) {
      root = true;
      L[v] = 0;
      const int64_t d = row_deg(off, v);
      if (d > 0) {
        expand = true;
        ++cnt;
        edg += d;
      }
    }
    const uint64_t rm = __ballot(root), em = __ballot(expand);
    if (lane() == 0 && rm) {
      const int64_t w = (v - lane()) >> 5;  // the wave's first word
      if (static_cast<uint32_t>(rm)) vis[w] |= static_cast<uint32_t>(rm);
      if (rm >> 32) vis[w + 1] |= static_cast<uint32_t>(rm >> 32);
      if (static_cast<uint32_t>(em)) bm0[w] |= static_cast<uint32_t>(em);
      if (em >> 32) bm0[w + 1] |= static_cast<uint32_t>(em >> 32);
    }
  }
  block_partial(cnt, edg, part, sh);
}

}  // namespace

BfsWs bfs_reserve(Carver& c, int64_t n) {
  BfsWs w;
  const int64_t words = (n + 31) / 32 + 1;
  w.vis = c.take<uint32_t>(words);
  w.bms = c.take<uint32_t>(3 * words);
  w.big = c.take<int32_t>(kBigCap);
  w.parent = c.take<int32_t>(n + 1);
  w.part = c.take<int64_t>(4 * kMaxParts);  // step and big kernels, (count, entries) each
  w.st = c.take<char>(sizeof(BfsState));
  w.key = c.take<unsigned long long>(1);
  w.root = c.take<int64_t>(1);
  w.comp0 = nullptr;
  return w;
}

namespace {

// Blocks of the level kernels: one per 256 vertices (each thread then takes
// one vertex or one 64-vertex wave group per level), at most eight per CU,
// so that a small graph's levels launch only the blocks they can use.
unsigned step_grid(int64_t n) {
  int64_t g = num_cus() * 8;
  if (g > kMaxParts) g = kMaxParts;
  const int64_t want = (n + kThreads - 1) / kThreads;
  if (want < g) g = want;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// Pinned host copy of the BFS state, one per host thread (allocated on
// first use, kept until the process ends; null if it cannot be had, and the
// state is then read into pageable memory): a readback into pageable memory
// goes through a staging copy and took about 13 us more per level group
// (R-MAT S14 BFS 0.26 -> 0.24 ms, S20 0.31 -> 0.28 ms).
BfsState* pinned_state() {
  thread_local BfsState* p = nullptr;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void* q = nullptr;
    if (hipHostMalloc(&q, sizeof(BfsState), hipHostMallocDefault) == hipSuccess) p = static_cast<BfsState*>(q);
    else (void)hipGetLastError();  // the fallback needs no error left behind
  }
  return p;
}

// Runs the levels of the BFS whose state and level-0 bitmap are set, in
// groups of kLevelsPerSync, until the frontier is empty.  Returns its level
// count and, in *rest_out (nullable), the row entries of the vertices it
// left unvisited.
int bfs_levels_loop(const tc_csr* g, int32_t* L, BfsWs& w, int group, int32_t* levels_out, hipStream_t s,
                    int64_t* rest_out = nullptr) {
  BfsState* st = reinterpret_cast<BfsState*>(w.st);
  const unsigned gs = step_grid(g->n);
  // the big-row kernel runs every level but has work only where a frontier
  // row exceeds kBig entries; two blocks per CU expand those rows and keep
  // the launch cheap where there are none (its partials past this grid stay
  // zero from the clear at the start of the BFS)
  const unsigned gb = gs < static_cast<unsigned>(num_cus() * 2) ? gs : static_cast<unsigned>(num_cus() * 2);
  for (;;) {
    for (int k = 0; k < group; ++k) {
      step_kernel<<<gs, kThreads, 0, s>>>(g->row_offsets, g->cols, g->n, st, L, w.vis, w.bms, w.big, w.part);
      big_kernel<<<gb, kThreads, 0, s>>>(g->row_offsets, g->cols, g->n, st, L, w.vis, w.bms, w.big,
                                         w.part + 2 * gs);
      decide_kernel<<<1, kThreads, 0, s>>>(g->n, st, w.part, static_cast<int>(2 * gs));
    }
    TC_HIP(hipGetLastError());
    BfsState* pin = pinned_state();
    BfsState local;
    BfsState* dst = pin ? pin : &local;
    TC_HIP(hipMemcpyAsync(dst, st, sizeof(BfsState), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const BfsState h = *dst;
    if (h.done) {
      *levels_out = h.num_levels;
      if (rest_out) *rest_out = h.unexplored;
      return TC_OK;
    }
  }
}

}  // namespace

int bfs_run(const tc_csr* g, int64_t root, int32_t* L, int32_t* num_levels, BfsWs& w,
            hipStream_t s, int32_t* first_levels) {
  const int64_t n = g->n;
  if (n == 0) {
    if (num_levels) *num_levels = 0;
    if (first_levels) *first_levels = 0;
    return TC_OK;
  }
  const int64_t words = (n + 31) / 32 + 1;
  BfsState* st = reinterpret_cast<BfsState*>(w.st);
  const unsigned gs = step_grid(g->n);
  const int64_t clear = n > 3 * words ? n : 3 * words;
  clear_state_kernel<<<grid_for(clear, kThreads, 16384), kThreads, 0, s>>>(L, n, w.vis, words, w.bms, w.key,
                                                                         w.part, 4 * static_cast<int64_t>(gs));
  TC_HIP(hipGetLastError());
  if (root < 0) {
    root_key_kernel<<<grid_for(n, kThreads, static_cast<unsigned>(num_cus() * 2)), kThreads, 0, s>>>(
        g->row_offsets, n, w.key);
    TC_HIP(hipGetLastError());
  }
  start_kernel<<<1, 1, 0, s>>>(g->row_offsets, w.key, root, L, w.vis, w.bms, w.part, w.root);
  init_state_kernel<<<1, kThreads, 0, s>>>(n, st, w.part, static_cast<int>(2 * gs), g->nnz);
  TC_HIP(hipGetLastError());
  int32_t lv0 = 0;
  int64_t rest = 0;
  TC_TRY(bfs_levels_loop(g, L, w, kLevelsPerSync, &lv0, s, &rest));
  if (first_levels) *first_levels = lv0;
  if (w.comp0) {
    copy_words_kernel<<<grid_for(words, kThreads, 16384), kThreads, 0, s>>>(w.vis, w.comp0, words);
    TC_HIP(hipGetLastError());
  }
  if (rest == 0) {
    // no unreached vertex has an edge: no other component to level
    isolated_kernel<<<grid_for(n, kThreads, 16384), kThreads, 0, s>>>(w.vis, n, L);
    TC_HIP(hipGetLastError());
    if (num_levels) *num_levels = lv0;
    return TC_OK;
  }
  // Remaining components (Alg. 1 rescans for unvisited vertices): one
  // union-find pass over the unreached vertices gives each component its
  // smallest id as root.
  uf_init_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(w.parent, n);
  uf_hook_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(g->row_offsets, g->cols, n, w.vis, w.parent);
  TC_TRY(fill_i32(reinterpret_cast<int32_t*>(w.bms), 0, 3 * words, s));
  uf_roots_kernel<<<gs, kThreads, 0, s>>>(g->row_offsets, n, w.parent, L, w.vis, w.bms, w.part);
  init_state_kernel<<<1, kThreads, 0, s>>>(n, st, w.part, static_cast<int>(gs), -1);
  TC_HIP(hipGetLastError());
  int32_t lv1 = 0;
  // the remaining components are usually shallow: shorter groups
  TC_TRY(bfs_levels_loop(g, L, w, kLevelsPerSyncRest, &lv1, s));
  if (num_levels) *num_levels = lv0 > lv1 ? lv0 : lv1;
  return TC_OK;
}

}  // namespace tc
