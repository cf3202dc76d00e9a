// bfs.hip -- BFS levels L(v) of Def. 2 with the root rule of Alg. 1:
// a BFS from r0 (given, or the largest-degree vertex with the smallest id on
// ties), then every component not reached is levelled from its smallest id.
//
// GPU structure:
//   * top-down steps expand a frontier queue edge-balanced: the frontier's
//     degree prefix maps a flat edge index to (frontier vertex, offset), so a
//     hub row is spread over many waves and every read of cols is coalesced;
//     new vertices are claimed with an atomic OR on a visited bitmap (n bits,
//     L2-resident) and appended with one atomic per wave;
//   * bottom-up steps (Beamer et al.'s direction optimisation) let every
//     unvisited vertex look for a neighbour in the frontier bitmap and stop
//     at the first hit; they run when the frontier's edges outnumber the
//     unexplored edges / alpha;
//   * the remaining components: union-find over the unreached vertices where
//     a root is always hooked under the smaller root, so every component's
//     final root is its smallest id; those roots then start one multi-source
//     BFS (components are disjoint, so the per-component distances are
//     exactly those of separate BFS runs).
// The host reads two counters per level (frontier size and its edge count).
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

// Starts the BFS from one root (either the argmax key or a given root):
// level 0, visited, first queue entry, counters.
__global__ void start_kernel(const int64_t* off, const unsigned long long* key, int64_t given_root,
                             int32_t* L, uint32_t* vis, int32_t* q, int64_t* ctr, int64_t* root_out) {
  int64_t r = given_root;
  if (r < 0) r = static_cast<int64_t>(0xFFFFFFFFull - (*key & 0xFFFFFFFFull));
  L[r] = 0;
  vis[r >> 5] |= 1u << (r & 31);
  q[0] = static_cast<int32_t>(r);
  ctr[0] = 1;
  ctr[1] = row_deg(off, r);
  *root_out = r;
}

__global__ void zero_ctr_kernel(int64_t* ctr) {
  if (threadIdx.x < 4) ctr[threadIdx.x] = 0;
}

__global__ void frontier_deg_kernel(const int64_t* off, const int32_t* q, int64_t f, int64_t* fdeg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < f;
       i += (int64_t)gridDim.x * blockDim.x)
    fdeg[i] = row_deg(off, q[i]);
}

// Block-aggregated append: the lanes with `take` set write `item` to the
// queue q at consecutive slots reserved with one atomic per block on
// ctr[slot]; ctr[1] accumulates their `weight` (edge counts).  Every thread
// of the block must call it (it synchronises).
struct AppendLds {
  int64_t cnt[kThreads / kWave];
  int64_t edg[kThreads / kWave];
  int64_t base;
};

__device__ __forceinline__ void block_append(bool take, int32_t item, int64_t weight, int32_t* q, int64_t* ctr,
                                             int slot, AppendLds& L) {
  const int w = threadIdx.x / kWave;
  const uint64_t m = __ballot(take);
  const int64_t we = wave_sum(take ? weight : int64_t(0));
  if (lane() == 0) {
    L.cnt[w] = __popcll(m);
    L.edg[w] = we;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t tc = 0, te = 0;
    for (int i = 0; i < kThreads / kWave; ++i) {
      const int64_t c = L.cnt[i];
      L.cnt[i] = tc;
      tc += c;
      te += L.edg[i];
    }
    L.base = tc ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[slot]),
                                                 static_cast<unsigned long long>(tc)))
                : 0;
    if (te) atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[1]), static_cast<unsigned long long>(te));
  }
  __syncthreads();
  if (take && q) q[L.base + L.cnt[w] + __popcll(m & lanemask_lt())] = item;
  __syncthreads();
}

// Top-down: flat edge index k in [0, ef) -> frontier slot i with
// pre[i] <= k < pre[i+1].
__global__ __launch_bounds__(kThreads) void topdown_kernel(const int64_t* off, const int32_t* cols,
                                                           const int32_t* q, int64_t f,
                                                           const int64_t* pre, int64_t ef,
                                                           int32_t next_level, int32_t* L,
                                                           uint32_t* vis, int32_t* qn, int64_t* ctr) {
  __shared__ AppendLds lds;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k0 = blockIdx.x * (int64_t)blockDim.x; k0 < ef; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    bool take = false;
    int32_t w = 0;
    int64_t dw = 0;
    if (k < ef) {
      int64_t i = upper_bound_dev(pre, 0, f + 1, k) - 1;
      int32_t v = q[i];
      w = cols[off[v] + (k - pre[i])];
      uint32_t bit = 1u << (w & 31);
      if (!(load_relaxed(&vis[w >> 5]) & bit)) {
        uint32_t old = atomicOr(&vis[w >> 5], bit);
        if (!(old & bit)) {
          take = true;
          L[w] = next_level;
          dw = row_deg(off, w);
        }
      }
    }
    block_append(take, w, dw, qn, ctr, 0, lds);
  }
}

// Frontier queue -> frontier bitmap (bits must be clear beforehand).
__global__ void queue_to_bits_kernel(const int32_t* q, int64_t f, uint32_t* bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < f;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = q[i];
    atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
}

// Bottom-up: every unvisited vertex scans its row for a frontier neighbour.
__global__ __launch_bounds__(kThreads) void bottomup_kernel(const int64_t* off, const int32_t* cols,
                                                            int64_t n, const uint32_t* fbits,
                                                            int32_t next_level, int32_t* L,
                                                            uint32_t* vis, uint32_t* nbits,
                                                            int64_t* ctr) {
  __shared__ AppendLds lds;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    bool take = false;
    int64_t dv = 0;
    if (v < n && !(vis[v >> 5] & (1u << (v & 31)))) {
      const int64_t b = off[v], e = off[v + 1];
      for (int64_t j = b; j < e; ++j) {
        int32_t w = cols[j];
        if (fbits[w >> 5] & (1u << (w & 31))) {
          take = true;
          break;
        }
      }
      if (take) {
        L[v] = next_level;
        dv = e - b;
        atomicOr(&nbits[v >> 5], 1u << (v & 31));
        atomicOr(&vis[v >> 5], 1u << (v & 31));
      }
    }
    block_append(take, 0, dv, nullptr, ctr, 0, lds);
  }
}

// Bitmap -> queue (order within the queue is irrelevant).
__global__ void bits_to_queue_kernel(const uint32_t* bits, int64_t n, int32_t* q, int64_t* ctr) {
  __shared__ AppendLds lds;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    const bool take = v < n && (bits[v >> 5] & (1u << (v & 31)));
    block_append(take, static_cast<int32_t>(v), 0, q, ctr, 2, lds);
  }
}

// ------------------------------------------------- remaining components
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

// Roots of the unreached components start the multi-source BFS at level 0;
// isolated vertices get level 0 and need no expansion.
__global__ void uf_roots_kernel(const int64_t* off, int64_t n, int32_t* parent, int32_t* L,
                                uint32_t* vis, int32_t* q, int64_t* ctr) {
  __shared__ AppendLds lds;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    bool take = false;
    int64_t dv = 0;
    if (v < n && !(vis[v >> 5] & (1u << (v & 31)))) {
      if (uf_find(parent, static_cast<int32_t>(v)) == v) {
        L[v] = 0;
        atomicOr(&vis[v >> 5], 1u << (v & 31));
        dv = row_deg(off, v);
        take = dv > 0;
      }
    }
    block_append(take, static_cast<int32_t>(v), dv, q, ctr, 0, lds);
  }
}

}  // namespace

BfsWs bfs_reserve(Carver& c, int64_t n) {
  BfsWs w;
  const int64_t words = (n + 31) / 32 + 1;
  w.vis = c.take<uint32_t>(words);
  w.fbits = c.take<uint32_t>(words);
  w.nbits = c.take<uint32_t>(words);
  w.q0 = c.take<int32_t>(n + 1);
  w.q1 = c.take<int32_t>(n + 1);
  w.fdeg = c.take<int64_t>(n + 1);
  w.pre = c.take<int64_t>(n + 2);
  w.parent = c.take<int32_t>(n + 1);
  w.ctr = c.take<int64_t>(8);
  w.key = c.take<unsigned long long>(1);
  w.root = c.take<int64_t>(1);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1));
  w.scratch_bytes = scan_ws_bytes(n + 1);
  w.comp0 = nullptr;
  return w;
}

// Runs one level-synchronous BFS from the queue currently in w.q0 (ctr[0] =
// size, ctr[1] = its edges, already read into f / ef).  Returns the number
// of levels (deepest level + 1).
static int bfs_loop(const tc_csr* g, int32_t* L, BfsWs& w, int64_t f, int64_t ef,
                    int64_t& unexplored_edges, int32_t* levels_out, hipStream_t s) {
  const int64_t n = g->n;
  const int64_t words = (n + 31) / 32 + 1;
  int32_t* q = w.q0;
  int32_t* qn = w.q1;
  bool bottom_up = false;   // direction of the previous step
  bool queue_valid = true;  // q holds the frontier (else only fbits does)
  int32_t level = 0;
  int64_t host[4];
  const int64_t alpha = 14, beta = 24;
  while (f > 0) {
    unexplored_edges -= ef;
    bool go_bottom_up;
    if (!bottom_up) go_bottom_up = ef > unexplored_edges / alpha && f > n / 256;
    else go_bottom_up = f >= n / beta;
    zero_ctr_kernel<<<1, 64, 0, s>>>(w.ctr);
    if (go_bottom_up) {
      if (!bottom_up) {  // frontier bitmap from the queue
        TC_TRY(fill_i32(reinterpret_cast<int32_t*>(w.fbits), 0, words, s));
        queue_to_bits_kernel<<<grid_for(f, kThreads, 65536), kThreads, 0, s>>>(q, f, w.fbits);
      }
      TC_TRY(fill_i32(reinterpret_cast<int32_t*>(w.nbits), 0, words, s));
      bottomup_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(
          g->row_offsets, g->cols, n, w.fbits, level + 1, L, w.vis, w.nbits, w.ctr);
      TC_HIP(hipGetLastError());
      // the new frontier's bitmap becomes the current one
      uint32_t* t = w.fbits;
      w.fbits = w.nbits;
      w.nbits = t;
      queue_valid = false;
    } else {
      if (!queue_valid) {  // rebuild the queue from the frontier bitmap
        bits_to_queue_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(w.fbits, n, q, w.ctr);
        TC_HIP(hipGetLastError());
        zero_ctr_kernel<<<1, 64, 0, s>>>(w.ctr);
      }
      frontier_deg_kernel<<<grid_for(f, kThreads, 65536), kThreads, 0, s>>>(g->row_offsets, q, f,
                                                                              w.fdeg);
      Carver sc(w.scratch);
      TC_TRY(scan_exclusive<int64_t>(w.fdeg, w.pre, f, sc, s));
      if (ef > 0) {
        topdown_kernel<<<grid_for(ef, kThreads, 8 * num_cus() * 8), kThreads, 0, s>>>(
            g->row_offsets, g->cols, q, f, w.pre, ef, level + 1, L, w.vis, qn, w.ctr);
        TC_HIP(hipGetLastError());
      }
      int32_t* t = q;
      q = qn;
      qn = t;
      queue_valid = true;
    }
    bottom_up = go_bottom_up;
    TC_HIP(hipMemcpyAsync(host, w.ctr, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    f = host[0];
    ef = host[1];
    if (f > 0) ++level;
  }
  if (q != w.q0) {  // keep the convention that the caller's next queue is q0
    int32_t* t = w.q0;
    w.q0 = w.q1;
    w.q1 = t;
  }
  *levels_out = level + 1;
  return TC_OK;
}

__global__ void copy_words_kernel(const uint32_t* src, uint32_t* dst, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int bfs_run(const tc_csr* g, int64_t root, int32_t* L, int32_t* num_levels, BfsWs& w,
            hipStream_t s, int32_t* first_levels) {
  const int64_t n = g->n;
  if (n == 0) {
    if (num_levels) *num_levels = 0;
    if (first_levels) *first_levels = 0;
    return TC_OK;
  }
  const int64_t words = (n + 31) / 32 + 1;
  TC_TRY(fill_i32(L, -1, n, s));
  TC_TRY(fill_i32(reinterpret_cast<int32_t*>(w.vis), 0, words, s));
  zero_ctr_kernel<<<1, 64, 0, s>>>(w.ctr);
  if (root < 0) {
    TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.key), 0, 1, s));
    root_key_kernel<<<grid_for(n, kThreads, 4096), kThreads, 0, s>>>(g->row_offsets, n, w.key);
    TC_HIP(hipGetLastError());
  }
  start_kernel<<<1, 1, 0, s>>>(g->row_offsets, w.key, root, L, w.vis, w.q0, w.ctr, w.root);
  TC_HIP(hipGetLastError());
  int64_t host[2];
  TC_HIP(hipMemcpyAsync(host, w.ctr, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  int32_t lv0 = 0;
  int64_t unexplored = g->nnz;
  TC_TRY(bfs_loop(g, L, w, host[0], host[1], unexplored, &lv0, s));
  if (first_levels) *first_levels = lv0;
  if (w.comp0) {
    copy_words_kernel<<<grid_for(words, kThreads, 16384), kThreads, 0, s>>>(w.vis, w.comp0, words);
    TC_HIP(hipGetLastError());
  }
  // Remaining components (Alg. 1 rescans for unvisited vertices): one
  // union-find pass over the unreached vertices gives each component its
  // smallest id as root.
  uf_init_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(w.parent, n);
  uf_hook_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(g->row_offsets, g->cols, n, w.vis,
                                                                   w.parent);
  zero_ctr_kernel<<<1, 64, 0, s>>>(w.ctr);
  uf_roots_kernel<<<grid_for(n, kThreads, 65536), kThreads, 0, s>>>(g->row_offsets, n, w.parent, L,
                                                                    w.vis, w.q0, w.ctr);
  TC_HIP(hipGetLastError());
  TC_HIP(hipMemcpyAsync(host, w.ctr, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  int32_t lv1 = 0;
  if (host[0] > 0) TC_TRY(bfs_loop(g, L, w, host[0], host[1], unexplored, &lv1, s));
  if (num_levels) *num_levels = lv0 > lv1 ? lv0 : lv1;
  return TC_OK;
}

}  // namespace tc
