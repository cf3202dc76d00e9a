// validate.hip -- structural checks of a CSR (the simple undirected graph the
// method assumes, Sec. II-A).  Three rounds, each only after the previous
// one passed, because later checks index with what earlier ones verify:
//   1. offsets: row_offsets[0] = 0, row_offsets[n] = nnz, never decreasing;
//   2. every id in [0, n);
//   3. per entry: no loop, strictly above its predecessor in the row (else
//      equal -> duplicate, smaller -> not sorted), and the reverse entry
//      exists (binary search in the other row).
#include <stdlib.h>

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

// One wave per row of the concatenated batch: the row's graph g is the last
// with vbase[g] <= v; its entries must be local ids in [0, n_g), not the
// row's own local id, strictly ascending, with the reverse entry in row
// vbase[g] + w.  Ids out of range are flagged and never dereferenced.
__global__ void batch_entries_kernel(const int64_t* vbase, int32_t G, const int64_t* off, const int32_t* cols,
                                     int64_t total_n, int32_t* flags) {
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = wid; v < total_n; v += nw) {
    const int64_t g = upper_bound_dev(vbase, 0, static_cast<int64_t>(G) + 1, v) - 1;
    const int64_t v0 = vbase[g], ng = vbase[g + 1] - v0, lv = v - v0;
    const int64_t b = off[v], e = off[v + 1];
    int f = 0;
    for (int64_t j = b + lane(); j < e; j += kWave) {
      const int32_t w = cols[j];
      if (w < 0 || w >= ng) {
        f |= 2;
        continue;
      }
      if (w == lv) f |= 4;
      if (j > b) {
        const int32_t p = cols[j - 1];
        if (p == w) f |= 8;
        else if (p > w) f |= 16;
      }
      const int64_t wb = off[v0 + w], we = off[v0 + w + 1];
      const int64_t k = lower_bound_dev(cols, wb, we, static_cast<int32_t>(lv));
      if (k >= we || cols[k] != lv) f |= 32;
    }
    int any = 0;
    for (int bit = 2; bit <= 32; bit <<= 1)
      if (__ballot(f & bit)) any |= bit;
    if (lane() == 0 && any) atomicOr(flags, any);
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

int validate_batch_run(const tc_batch* b, void* ws, hipStream_t s) {
  const int32_t G = b->num_graphs;
  const int64_t total_n = b->total_vertices, nnz = b->total_nnz;
  int64_t* hv = static_cast<int64_t*>(malloc(sizeof(int64_t) * (static_cast<size_t>(G) + 1)));
  if (!hv) return fail(TC_ERR_INVALID_ARG, "tc_count_batch: no host memory for the vertex bases");
  hipError_t e = hipMemcpyAsync(hv, b->vbase, sizeof(int64_t) * (static_cast<size_t>(G) + 1),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free(hv);
    return fail(TC_ERR_HIP, "tc_count_batch: reading vbase failed: %s", hipGetErrorString(e));
  }
  int status = TC_OK;
  int64_t most = 0;
  if (hv[0] != 0 || hv[G] != total_n) status = TC_ERR_BAD_OFFSETS;
  for (int32_t g = 0; g < G && status == TC_OK; ++g) {
    const int64_t ng = hv[g + 1] - hv[g];
    if (ng < 0) status = TC_ERR_BAD_OFFSETS;
    else if (ng > most) most = ng;
  }
  free(hv);
  if (status != TC_OK) return fail(status, "tc_count_batch: vbase must rise from 0 to total_vertices");
  if (most > TC_BATCH_MAX_N)
    return fail(TC_ERR_TOO_LARGE, "tc_count_batch: a graph has %lld vertices (limit %d)", (long long)most,
                TC_BATCH_MAX_N);
  if (most > b->max_graph_vertices)
    return fail(TC_ERR_INVALID_ARG, "tc_count_batch: a graph has %lld vertices, max_graph_vertices says %d",
                (long long)most, b->max_graph_vertices);
  int32_t* flags = static_cast<int32_t*>(ws);
  int32_t h = 0;
  TC_TRY(fill_i32(flags, 0, 1, s));
  offsets_kernel<<<grid_for(total_n + 1, kThreads, 16384), kThreads, 0, s>>>(b->row_offsets, total_n, nnz, flags);
  TC_HIP(hipGetLastError());
  TC_HIP(hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (h) return fail(TC_ERR_BAD_OFFSETS, "tc_count_batch: row_offsets must rise from 0 to total_nnz");
  if (nnz > 0) {
    batch_entries_kernel<<<static_cast<unsigned>(num_cus() * 8), kThreads, 0, s>>>(b->vbase, G, b->row_offsets,
                                                                                  b->cols, total_n, flags);
    TC_HIP(hipGetLastError());
    TC_HIP(hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h & 2) return fail(TC_ERR_OUT_OF_RANGE, "tc_count_batch: a column is not a local id of its graph");
    if (h & 4) return fail(TC_ERR_SELF_LOOP, "tc_count_batch: a row contains its own vertex");
    if (h & 8) return fail(TC_ERR_DUPLICATE, "tc_count_batch: a row repeats a column id");
    if (h & 16) return fail(TC_ERR_NOT_SORTED, "tc_count_batch: a row is not ascending");
    if (h & 32) return fail(TC_ERR_NOT_SYMMETRIC, "tc_count_batch: an entry (u, v) has no reverse entry (v, u)");
  }
  return TC_OK;
}

}  // namespace tc
