// validate.hip -- structural checks of a CSR (the simple undirected graph the
// method assumes, Sec. II-A).  Three rounds, each only after the previous
// one passed, because later checks index with what earlier ones verify:
//   1. offsets: row_offsets[0] = 0, row_offsets[n] = nnz, never decreasing;
//   2. every id in [0, n);
//   3. per entry: no loop, strictly above its predecessor in the row (else
//      equal -> duplicate, smaller -> not sorted), and the reverse entry
//      exists (binary search in the other row).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;

__global__ void offsets_kernel(const int64_t* off, int64_t n, int64_t nnz, int32_t* flags) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (off[v + 1] < off[v]) atomicOr(flags, 1);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != nnz)) atomicOr(flags, 1);
}

__global__ void range_kernel(const int32_t* cols, int64_t nnz, int64_t n, int32_t* flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = cols[i];
    if (w < 0 || w >= n) atomicOr(flags, 2);
  }
}

// One wave per row.
__global__ void entries_kernel(const int64_t* off, const int32_t* cols, int64_t n, int32_t* flags) {
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = wid; v < n; v += nw) {
    const int64_t b = off[v], e = off[v + 1];
    int f = 0;
    for (int64_t j = b + lane(); j < e; j += kWave) {
      const int32_t w = cols[j];
      if (w == v) f |= 4;
      if (j > b) {
        const int32_t p = cols[j - 1];
        if (p == w) f |= 8;
        else if (p > w) f |= 16;
      }
      // reverse entry v in row w (only meaningful when rows are sorted;
      // a failed search on an unsorted row is reported as unsorted first)
      const int64_t wb = off[w], we = off[w + 1];
      const int64_t k = lower_bound_dev(cols, wb, we, static_cast<int32_t>(v));
      if (k >= we || cols[k] != v) f |= 32;
    }
    f = static_cast<int>(__ballot(f & 4) ? 4 : 0) | static_cast<int>(__ballot(f & 8) ? 8 : 0) |
        static_cast<int>(__ballot(f & 16) ? 16 : 0) | static_cast<int>(__ballot(f & 32) ? 32 : 0);
    if (lane() == 0 && f) atomicOr(flags, f);
  }
}

}  // namespace

size_t validate_ws_bytes(int64_t, int64_t) { return 256; }

int validate_run(const tc_csr* g, void* ws, hipStream_t s) {
  const int64_t n = g->n, nnz = g->nnz;
  int32_t* flags = static_cast<int32_t*>(ws);
  TC_TRY(fill_i32(flags, 0, 1, s));
  int32_t h = 0;
  offsets_kernel<<<grid_for(n + 1, kThreads, 16384), kThreads, 0, s>>>(g->row_offsets, n, nnz, flags);
  TC_HIP(hipGetLastError());
  TC_HIP(hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h) return fail(TC_ERR_BAD_OFFSETS, "row_offsets must start at 0, end at nnz and never decrease");
  if (nnz > 0) {
    range_kernel<<<grid_for(nnz, kThreads, 16384), kThreads, 0, s>>>(g->cols, nnz, n, flags);
    TC_HIP(hipGetLastError());
    TC_HIP(hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h) return fail(TC_ERR_OUT_OF_RANGE, "a column id is outside [0, n)");
    entries_kernel<<<static_cast<unsigned>(num_cus() * 8), kThreads, 0, s>>>(g->row_offsets, g->cols, n, flags);
    TC_HIP(hipGetLastError());
    TC_HIP(hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h & 4) return fail(TC_ERR_SELF_LOOP, "a row contains its own vertex");
    if (h & 8) return fail(TC_ERR_DUPLICATE, "a row repeats a column id");
    if (h & 16) return fail(TC_ERR_NOT_SORTED, "a row is not ascending");
    if (h & 32) return fail(TC_ERR_NOT_SYMMETRIC, "an entry (u, v) has no reverse entry (v, u)");
  }
  return TC_OK;
}

}  // namespace tc
