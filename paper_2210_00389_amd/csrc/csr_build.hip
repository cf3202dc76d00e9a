// csr_build.hip -- raw pairs -> simple undirected CSR (the graph input of
// Sec. III, with both orientations and sorted rows).
//
// Every pair (s, d), s != d, becomes two keys (s << B) | d and (d << B) | s
// with B = bits(n - 1); loops become an all-ones sentinel that sorts last.
// An LSD radix sort (8-bit digits, ceil(2B / 8) passes) orders the keys;
// each pass is a per-tile digit histogram, a device scan of the
// digit-major histogram, and a stable scatter in which every tile ranks its
// keys with wave ballots (the peer mask of a digit is the AND of 8 ballots).
// Adjacent equal keys are then dropped, the low B bits become cols, and a
// degree histogram plus a scan gives row_offsets.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int64_t kTile = kThreads * kRounds;  // 4096 keys per tile
constexpr int kRadix = 256;
constexpr uint64_t kSentinel = ~0ull;

__global__ void range_check_kernel(const int32_t* src, const int32_t* dst, int64_t P, int64_t n, int32_t* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = src[i], d = dst[i];
    if (s < 0 || s >= n || d < 0 || d >= n) atomicOr(bad, 1);
  }
}

__global__ void make_keys_kernel(const int32_t* src, const int32_t* dst, int64_t P, int B, uint64_t* keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t s = static_cast<uint32_t>(src[i]), d = static_cast<uint32_t>(dst[i]);
    const bool loop = s == d;
    keys[2 * i] = loop ? kSentinel : ((s << B) | d);
    keys[2 * i + 1] = loop ? kSentinel : ((d << B) | s);
  }
}

__global__ __launch_bounds__(kThreads) void hist_kernel(const uint64_t* keys, int64_t N, int shift,
                                                         int64_t nblocks, int64_t* ghist) {
  __shared__ int32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * kTile;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    if (i < N) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  ghist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void scatter_kernel(const uint64_t* keys, int64_t N, int shift,
                                                            int64_t nblocks, const int64_t* gpos,
                                                            uint64_t* out) {
  constexpr int kW = kThreads / kWave;
  __shared__ int32_t run[kRadix];        // keys of each digit already placed by this tile
  __shared__ int32_t wcnt[kW][kRadix];   // per-wave digit counts of the current round
  __shared__ int64_t base_pos[kRadix];
  const int tid = threadIdx.x, w = tid / kWave;
  run[tid] = 0;
  base_pos[tid] = gpos[tid * nblocks + blockIdx.x];
  const int64_t base = blockIdx.x * kTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kRounds; ++r) {
    for (int k = tid; k < kW * kRadix; k += kThreads) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const int64_t i = base + r * kThreads + tid;
    const bool valid = i < N;
    uint64_t key = 0;
    int dig = 0;
    if (valid) {
      key = keys[i];
      dig = static_cast<int>((key >> shift) & (kRadix - 1));
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank_in_wave = __popcll(peers & lt);
    // the highest lane of each peer group publishes the group size
    if (valid && (peers >> lane()) == 1ull) wcnt[w][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int before = run[dig];
      for (int ww = 0; ww < w; ++ww) before += wcnt[ww][dig];
      out[base_pos[dig] + before + rank_in_wave] = key;
    }
    __syncthreads();
    {
      int add = 0;
      for (int ww = 0; ww < kW; ++ww) add += wcnt[ww][tid];
      run[tid] += add;
    }
    __syncthreads();
  }
}

__global__ void unique_flags_kernel(const uint64_t* keys, int64_t N, int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    flag[i] = (k != kSentinel) && (i == 0 || keys[i - 1] != k);
  }
}

__global__ void compact_kernel(const uint64_t* keys, int64_t N, const int32_t* flag, const int64_t* pos,
                               int B, int32_t* cols, int32_t* deg) {
  const uint64_t low = (1ull << B) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const uint64_t k = keys[i];
    cols[pos[i]] = static_cast<int32_t>(k & low);
    atomicAdd(&deg[k >> B], 1);
  }
}

}  // namespace

size_t radix_ws_bytes(int64_t N) {
  Carver c(nullptr);
  const int64_t nblocks = (N + kTile - 1) / kTile;
  c.take<int64_t>(kRadix * nblocks + 1);
  c.take<int64_t>(kRadix * nblocks + 2);
  c.take<char>(scan_ws_bytes(kRadix * nblocks + 1));
  return c.used();
}

int radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t N, int bit_lo, int bit_hi, char* scratch,
                   hipStream_t s, uint64_t** result) {
  *result = keys;
  if (N <= 0 || bit_hi <= bit_lo) return TC_OK;
  const int64_t nblocks = (N + kTile - 1) / kTile;
  Carver c(scratch);
  int64_t* ghist = c.take<int64_t>(kRadix * nblocks + 1);
  int64_t* gpos = c.take<int64_t>(kRadix * nblocks + 2);
  char* sc_base = c.take<char>(0);
  uint64_t* a = keys;
  uint64_t* b = tmp;
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    hist_kernel<<<(unsigned)nblocks, kThreads, 0, s>>>(a, N, shift, nblocks, ghist);
    Carver sc(sc_base);
    TC_TRY(scan_exclusive<int64_t>(ghist, gpos, kRadix * nblocks, sc, s));
    scatter_kernel<<<(unsigned)nblocks, kThreads, 0, s>>>(a, N, shift, nblocks, gpos, b);
    TC_HIP(hipGetLastError());
    uint64_t* t = a;
    a = b;
    b = t;
  }
  *result = a;
  return TC_OK;
}

static int bits_for(int64_t n) {
  int B = 1;
  while (B < 31 && (int64_t(1) << B) < n) ++B;
  return B;
}

size_t build_ws_bytes(int64_t n, int64_t num_pairs) {
  Carver c(nullptr);
  const int64_t N = 2 * num_pairs;
  const int64_t nblocks = (N + kTile - 1) / kTile;
  (void)nblocks;
  c.take<uint64_t>(N + 1);
  c.take<uint64_t>(N + 1);
  c.take<int32_t>(N + 1);
  c.take<int64_t>(N + 2);
  c.take<int32_t>(n + 1);
  c.take<int32_t>(4);
  size_t sc = scan_ws_bytes(N + 1);
  size_t sc2 = radix_ws_bytes(N);
  c.take<char>(sc > sc2 ? sc : sc2);
  return c.used();
}

int build_run(int64_t n, int64_t P, const int32_t* src, const int32_t* dst, int64_t* row_offsets,
              int32_t* cols, int64_t* nnz_out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (ws_bytes < build_ws_bytes(n, P))
    return fail(TC_ERR_WORKSPACE, "tc_build_csr: workspace %zu < %zu bytes", ws_bytes, build_ws_bytes(n, P));
  const int64_t N = 2 * P;
  Carver c(ws);
  uint64_t* ka = c.take<uint64_t>(N + 1);
  uint64_t* kb = c.take<uint64_t>(N + 1);
  int32_t* flag = c.take<int32_t>(N + 1);
  int64_t* pos = c.take<int64_t>(N + 2);
  int32_t* deg = c.take<int32_t>(n + 1);
  int32_t* bad = c.take<int32_t>(4);
  char* scratch = c.take<char>(1);
  TC_TRY(fill_i32(deg, 0, n + 1, s));
  TC_TRY(fill_i32(bad, 0, 1, s));
  if (P > 0) {
    range_check_kernel<<<grid_for(P, kThreads, 16384), kThreads, 0, s>>>(src, dst, P, n, bad);
    TC_HIP(hipGetLastError());
    int32_t hbad = 0;
    TC_HIP(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(TC_ERR_OUT_OF_RANGE, "tc_build_csr: a pair has an id outside [0, %lld)", (long long)n);
    const int B = bits_for(n);
    make_keys_kernel<<<grid_for(P, kThreads, 16384), kThreads, 0, s>>>(src, dst, P, B, ka);
    uint64_t* sorted = nullptr;
    TC_TRY(radix_sort_u64(ka, kb, N, 0, 2 * B, scratch, s, &sorted));
    ka = sorted;
    unique_flags_kernel<<<grid_for(N, kThreads, 16384), kThreads, 0, s>>>(ka, N, flag);
    Carver sc(scratch);
    TC_TRY(scan_exclusive<int32_t>(flag, pos, N, sc, s));
    compact_kernel<<<grid_for(N, kThreads, 16384), kThreads, 0, s>>>(ka, N, flag, pos, B, cols, deg);
    TC_HIP(hipGetLastError());
  }
  Carver sc(scratch);
  TC_TRY(scan_exclusive<int32_t>(deg, row_offsets, n, sc, s));
  int64_t nnz = 0;
  TC_HIP(hipMemcpyAsync(&nnz, row_offsets + n, sizeof nnz, hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  *nnz_out = nnz;
  return TC_OK;
}

}  // namespace tc
