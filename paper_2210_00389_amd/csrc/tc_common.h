// tc_common.h -- internal helpers shared by the libtc HIP sources (device
// primitives for 64-lane wavefronts, workspace carving, error plumbing).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;

// ------------------------------------------------------------ errors
// Records the text of a failure for tc_last_error (thread-local) and returns
// the status.
int fail(int status, const char* fmt, ...);

#define TC_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::tc::fail(TC_ERR_HIP, "%s failed: %s (%s:%d)", #call,          \
                        hipGetErrorString(e_), __FILE__, __LINE__);          \
  } while (0)

#define TC_TRY(expr)            \
  do {                          \
    int s_ = (expr);            \
    if (s_ != TC_OK) return s_; \
  } while (0)

// ----------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures (used by tc_workspace_bytes), so sizing and carving share code.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
  size_t used() const { return off; }
};

// --------------------------------------------------------- profiling
// Stage markers: when profiling is on, record an event pair per stage on the
// stream of the call (see tc_profile_read).
void prof_begin_call(hipStream_t s);
void prof_stage(const char* name);  // closes the previous stage, opens this one
void prof_end_call();

// Grid size for a grid-stride kernel over `work` items with `per_block`
// items per block, capped to keep launches reasonable.
inline unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

int num_cus();

// Auxiliary streams (default priority) for fork/join concurrency inside one
// call, created once per host thread and device.
constexpr int kForkWays = 3;
struct Fork {
  hipStream_t aux[kForkWays];
  hipEvent_t fork;
  hipEvent_t join[kForkWays];
};
// Returns nullptr (and records the error) if streams/events cannot be made.
Fork* fork_for_device();
int fork_begin(Fork* f, hipStream_t s);  // aux streams wait for s
int fork_end(Fork* f, hipStream_t s);    // s waits for the aux streams

// ------------------------------------------------------ device helpers
__device__ __forceinline__ int lane() { return static_cast<int>(__lane_id()); }
__device__ __forceinline__ uint64_t lanemask_lt() { return __lanemask_lt(); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Inclusive prefix sum across the 64 lanes.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = __shfl_up(v, o, kWave);
    if (lane() >= o) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; `sh` must hold
// blockDim.x / 64 + 1 elements of T.  Returns the exclusive prefix and writes
// the block total to *total.  Contains __syncthreads.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T* total) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  T inc = wave_incl_scan(v);
  if (lane() == kWave - 1) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < nw; ++i) {
      T t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[nw] = run;
  }
  __syncthreads();
  T res = inc - v + sh[w];
  *total = sh[nw];
  __syncthreads();
  return res;
}

// Block-wide sum (result valid in every thread).  `sh` holds nw + 1 elements.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  v = wave_sum(v);
  if (lane() == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < nw; ++i) run += sh[i];
    sh[nw] = run;
  }
  __syncthreads();
  T r = sh[nw];
  __syncthreads();
  return r;
}

// First index i in [lo, hi) with a[i] > key (a ascending); hi if none.
template <class T, class K>
__device__ __forceinline__ int64_t upper_bound_dev(const T* a, int64_t lo, int64_t hi, K key) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First index i in [lo, hi) with a[i] >= key.
template <class T, class K>
__device__ __forceinline__ int64_t lower_bound_dev(const T* a, int64_t lo, int64_t hi, K key) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <class T>
__device__ __forceinline__ T load_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------ device scan
// Exclusive scan of `count` values (int32 or int64) into out[0..count]
// (out[count] = total).  `total_dev` (nullable) also receives the total.
// Temporary space comes from the carver.
template <class T>
int scan_exclusive(const T* in, int64_t* out, int64_t count, Carver& ws, hipStream_t s);
// Two counts at once, packed in one int64 (count < 2^32): the low half scans
// (in[i] == a), the high half (in[i] == b).
int scan_exclusive_pair(const int32_t* in, int32_t a, int32_t b, int64_t* out, int64_t count, Carver& ws,
                        hipStream_t s);
// The same over in[i * stride].
int scan_exclusive_strided(const int32_t* in, int64_t stride, int64_t* out, int64_t count, Carver& ws,
                           hipStream_t s);
size_t scan_ws_bytes(int64_t count);

// Fill helpers (kernels, never hipMemset, so the call sequence stays
// capturable without memset nodes).
int fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
int fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s);

}  // namespace tc
