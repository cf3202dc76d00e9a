// root_select.hip -- choice of the BFS root by the size of the cover-edge
// set.  The paper's stated goal for the cover-edge set is the smallest
// k = |H| / m, and H depends on the BFS root.  Here the candidates are the
// vertices of largest degree (smallest id first on ties); every candidate
// gets the full level assignment of Alg. 1 (its BFS, then the remaining
// components from their smallest ids) and its |H| is counted; the smallest
// |H| wins, the earlier candidate on ties.
#include "tc_internal.h"

namespace tc {

namespace {

static_assert(kMaxRootCandidates == TC_MAX_ROOT_CANDIDATES, "the header's candidate limit");
constexpr int kThreads = 256;
constexpr int kWaveRow = 64;  // rows longer than this are scanned by a whole wave

// Largest key below `*bound` (0: no bound) over (degree << 32 | ~id):
// larger degree first, then smaller id.  One atomic per block.
__global__ __launch_bounds__(kThreads) void next_key_kernel(const int64_t* off, int64_t n,
                                                            const unsigned long long* bound,
                                                            unsigned long long* key) {
  const unsigned long long lim = bound ? *bound : ~0ull;
  unsigned long long best = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long d = static_cast<unsigned long long>(off[v + 1] - off[v]);
    const unsigned long long k = (d << 32) | (0xFFFFFFFFull - static_cast<unsigned long long>(v));
    if (k < lim && k > best) best = k;
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

// |H| = |{(x, v) : v in N(x), v > x, L(v) = L(x)}|: short rows one thread,
// long rows one wave; one atomic per block.
__global__ __launch_bounds__(kThreads) void hsize_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                                                         const int32_t* L, unsigned long long* h) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += stride) {
    const int64_t b = off[x], e = off[x + 1];
    if (e - b > kWaveRow) continue;
    const int32_t lx = L[x];
    for (int64_t i = b; i < e; ++i) {
      const int32_t v = cols[i];
      c += (v > x && L[v] == lx) ? 1 : 0;
    }
  }
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  for (int64_t x = wid; x < n; x += stride / kWave) {
    const int64_t b = off[x], e = off[x + 1];
    if (e - b <= kWaveRow) continue;
    const int32_t lx = L[x];
    for (int64_t i = b + lane(); i < e; i += kWave) {
      const int32_t v = cols[i];
      c += (v > x && L[v] == lx) ? 1 : 0;
    }
  }
  c = block_sum(c, sh);
  if (threadIdx.x == 0 && c) atomicAdd(h, static_cast<unsigned long long>(c));
}

}  // namespace

struct SelectWs {
  BfsWs bfs;
  int32_t* L;
  unsigned long long* keys;  // [kMaxRootCandidates]
  unsigned long long* h;     // [kMaxRootCandidates]
};

static SelectWs select_reserve(Carver& c, int64_t n) {
  SelectWs w;
  w.bfs = bfs_reserve(c, n);
  w.L = c.take<int32_t>(n + 1);
  w.keys = c.take<unsigned long long>(kMaxRootCandidates);
  w.h = c.take<unsigned long long>(kMaxRootCandidates);
  return w;
}

size_t select_root_ws_bytes(int64_t n) {
  Carver c(nullptr);
  select_reserve(c, n);
  return c.used();
}

int select_root_run(const tc_csr* g, int num, int64_t* root_out, int64_t* cand_out, int64_t* h_out, void* ws,
                    hipStream_t s) {
  const int64_t n = g->n;
  Carver c(ws);
  SelectWs w = select_reserve(c, n);
  num = static_cast<int>(std::min<int64_t>(num, n));
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.keys), 0, kMaxRootCandidates, s));
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.h), 0, kMaxRootCandidates, s));
  const unsigned gk = grid_for(n, kThreads, static_cast<unsigned>(num_cus() * 2));
  for (int i = 0; i < num; ++i) {
    next_key_kernel<<<gk, kThreads, 0, s>>>(g->row_offsets, n, i ? w.keys + i - 1 : nullptr, w.keys + i);
    TC_HIP(hipGetLastError());
  }
  unsigned long long keys[kMaxRootCandidates] = {0};
  if (num > 0) {
    TC_HIP(hipMemcpyAsync(keys, w.keys, num * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
  }
  int64_t cand[kMaxRootCandidates];
  for (int i = 0; i < num; ++i) cand[i] = static_cast<int64_t>(0xFFFFFFFFull - (keys[i] & 0xFFFFFFFFull));
  const unsigned gh = static_cast<unsigned>(num_cus() * 4);
  for (int i = 0; i < num; ++i) {
    TC_TRY(bfs_run(g, cand[i], w.L, nullptr, w.bfs, s));
    hsize_kernel<<<gh, kThreads, 0, s>>>(g->row_offsets, g->cols, n, w.L, w.h + i);
    TC_HIP(hipGetLastError());
  }
  unsigned long long h[kMaxRootCandidates] = {0};
  if (num > 0) {
    TC_HIP(hipMemcpyAsync(h, w.h, num * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
  }
  int best = 0;
  for (int i = 1; i < num; ++i)
    if (h[i] < h[best]) best = i;
  *root_out = num > 0 ? cand[best] : -1;
  for (int i = 0; i < num; ++i) {
    if (cand_out) cand_out[i] = cand[i];
    if (h_out) h_out[i] = static_cast<int64_t>(h[i]);
  }
  return TC_OK;
}

}  // namespace tc
