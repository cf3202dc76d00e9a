// support.hip -- triangles per edge (the support of k-truss decompositions)
// from a list of triangles: each triangle {a, b, c} adds one to both CSR
// entries of each of its edges (a, b), (a, c), (b, c).  The entries are found
// by binary search in the sorted rows; the additions are 32-bit atomics on
// distinct, mostly uncontended addresses.
#include "tc_internal.h"

namespace tc {

namespace {

// Position of v in the sorted row of u, or -1.
__device__ __forceinline__ int64_t find_pos(const int64_t* off, const int32_t* cols, int32_t u, int32_t v) {
  int64_t lo = off[u], hi = off[u + 1];
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (cols[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < end && cols[lo] == v) ? lo : -1;
}

__device__ __forceinline__ void bump(int32_t* sup, const int64_t* off, const int32_t* cols, int32_t a, int32_t b) {
  const int64_t p = find_pos(off, cols, a, b), q = find_pos(off, cols, b, a);
  if (p >= 0) atomicAdd(&sup[p], 1);
  if (q >= 0) atomicAdd(&sup[q], 1);
}

__global__ void support_kernel(const int64_t* off, const int32_t* cols, int64_t n, const int32_t* tri, int64_t ntri,
                               int32_t* sup) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntri; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
    // ids outside [0, n) would index rows that do not exist: such a triple is skipped
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) continue;
    bump(sup, off, cols, a, b);
    bump(sup, off, cols, a, c);
    bump(sup, off, cols, b, c);
  }
}

}  // namespace

int support_run(const tc_csr* g, const int32_t* tri, int64_t ntri, int32_t* support, hipStream_t s) {
  TC_TRY(fill_i32(support, 0, g->nnz, s));
  if (ntri <= 0 || g->n == 0) return TC_OK;
  support_kernel<<<grid_for(ntri, 256, 65536), 256, 0, s>>>(g->row_offsets, g->cols, g->n, tri, ntri, support);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
