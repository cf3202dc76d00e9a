// noalloc.hip -- tc_count_batch_noalloc: tc_count_batch for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).  The call's scratch (claim
// counter, parity bits, work-piece slots) lives in a file-scope device
// array instead of a caller workspace; the kernels are tc_count_batch's.
//
// The array's name is a host-side stand-in in host code: its device
// address is taken once per device with hipGetSymbolAddress (that device
// current) and only that address is handed to kernels.  Every call on one
// device uses the same array, so calls that overlap on a device race; the
// kernels clear what must start at zero on every call.
#include <mutex>

#include "tc_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// The device address of this device's copy of `scratch`.
int scratch_address(void** out) {
  int dev = -1;
  TC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return tc::fail(TC_ERR_HIP, "tc_count_batch_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch[dev] = p;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch[dev])
    return tc::fail(TC_ERR_HIP, "tc_count_batch_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch[dev];
  return TC_OK;
}

}  // namespace

extern "C" {

size_t tc_noalloc_scratch_bytes(void) { return kScratchBytes; }

int tc_count_batch_noalloc(const tc_batch* b, const tc_tuning* tuning, uint32_t flags, int64_t* triangles,
                           int64_t* h_count, int32_t* levels, tc_stream_t stream) {
  if (!b || !triangles) return tc::fail(TC_ERR_INVALID_ARG, "tc_count_batch_noalloc: NULL argument");
  if (b->num_graphs < 0 || b->total_vertices < 0 || b->total_nnz < 0)
    return tc::fail(TC_ERR_INVALID_ARG, "tc_count_batch_noalloc: negative size");
  if (b->max_graph_vertices > TC_BATCH_MAX_N)
    return tc::fail(TC_ERR_TOO_LARGE, "tc_count_batch_noalloc: a graph has more than %d vertices", TC_BATCH_MAX_N);
  if (b->num_graphs > 0 && (!b->vbase || !b->row_offsets || (b->total_nnz > 0 && !b->cols)))
    return tc::fail(TC_ERR_INVALID_ARG, "tc_count_batch_noalloc: NULL batch array");
  if (flags & TC_VALIDATE)
    return tc::fail(TC_ERR_INVALID_ARG,
                    "tc_count_batch_noalloc: TC_VALIDATE is not supported (check the batch with tc_count_batch)");
  const size_t need = tc::batch_ws_bytes(b->total_vertices, b->total_nnz, b->num_graphs);
  if (need > kScratchBytes)
    return tc::fail(TC_ERR_TOO_LARGE,
                    "tc_count_batch_noalloc: the batch needs %zu bytes of scratch, the static array holds %zu",
                    need, kScratchBytes);
  void* ptr = nullptr;
  TC_TRY(scratch_address(&ptr));
  return tc::batch_run(b, tuning, 0, triangles, h_count, levels, ptr, kScratchBytes,
                       static_cast<hipStream_t>(stream));
}

}  // extern "C"
