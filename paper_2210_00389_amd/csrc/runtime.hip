// runtime.hip -- error text, profiling events, device scan and fill kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <string>
#include <vector>

#include "tc_common.h"

namespace tc {

// ------------------------------------------------------------- errors
static thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------- profiling
static std::atomic<int> g_prof_on{0};

struct ProfCall {
  hipStream_t stream = nullptr;
  std::vector<std::string> names;
  std::vector<hipEvent_t> pool;  // reused across calls
  int used = 0;                  // marks[i] = pool[i] opens stage i, pool[i+1] closes it
  bool open = false;
};
static thread_local ProfCall g_prof;

static hipEvent_t prof_next_event() {
  if (g_prof.used == static_cast<int>(g_prof.pool.size())) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
  }
  return g_prof.pool[g_prof.used++];
}

void prof_begin_call(hipStream_t s) {
  if (!g_prof_on.load()) return;
  g_prof.used = 0;
  g_prof.names.clear();
  g_prof.open = false;
  g_prof.stream = s;
}

void prof_stage(const char* name) {
  if (!g_prof_on.load()) return;
  if (g_prof.names.size() >= TC_PROFILE_MAX_STAGES) return;
  hipEvent_t e = prof_next_event();
  if (!e) return;
  (void)hipEventRecord(e, g_prof.stream);
  g_prof.names.push_back(name);
  g_prof.open = true;
}

void prof_end_call() {
  if (!g_prof_on.load() || !g_prof.open) return;
  hipEvent_t e = prof_next_event();
  if (!e) return;
  (void)hipEventRecord(e, g_prof.stream);
  g_prof.open = false;
}

int prof_read(tc_profile* out) {
  memset(out, 0, sizeof *out);
  if (g_prof.used < 2 || g_prof.open) return TC_OK;
  TC_HIP(hipEventSynchronize(g_prof.pool[g_prof.used - 1]));
  int ns = g_prof.used - 1;
  if (ns > TC_PROFILE_MAX_STAGES) ns = TC_PROFILE_MAX_STAGES;
  out->num_stages = ns;
  for (int i = 0; i < ns; ++i) {
    strncpy(out->names[i], g_prof.names[i].c_str(), sizeof out->names[i] - 1);
    float ms = 0.f;
    TC_HIP(hipEventElapsedTime(&ms, g_prof.pool[i], g_prof.pool[i + 1]));
    out->ms[i] = ms;
  }
  return TC_OK;
}

void prof_enable(int on) { g_prof_on.store(on ? 1 : 0); }

int num_cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cached = v;
    else
      cached = 256;
  }
  return cached;
}

// --------------------------------------------------------------- fork
static thread_local Fork g_forks[16];
static thread_local bool g_fork_ok[16];

Fork* fork_for_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) {
    fail(TC_ERR_HIP, "fork_for_device: no current device");
    return nullptr;
  }
  Fork& f = g_forks[dev];
  if (!g_fork_ok[dev]) {
    for (int i = 0; i < kForkWays; ++i) {
      if (hipStreamCreateWithFlags(&f.aux[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming) != hipSuccess) {
        fail(TC_ERR_HIP, "fork_for_device: cannot create auxiliary streams");
        return nullptr;
      }
    }
    if (hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) != hipSuccess) {
      fail(TC_ERR_HIP, "fork_for_device: cannot create events");
      return nullptr;
    }
    g_fork_ok[dev] = true;
  }
  return &f;
}

int fork_begin(Fork* f, hipStream_t s) {
  TC_HIP(hipEventRecord(f->fork, s));
  for (int i = 0; i < kForkWays; ++i) TC_HIP(hipStreamWaitEvent(f->aux[i], f->fork, 0));
  return TC_OK;
}

int fork_end(Fork* f, hipStream_t s) {
  for (int i = 0; i < kForkWays; ++i) {
    TC_HIP(hipEventRecord(f->join[i], f->aux[i]));
    TC_HIP(hipStreamWaitEvent(s, f->join[i], 0));
  }
  return TC_OK;
}

// --------------------------------------------------------------- fill
template <class T>
__global__ void fill_kernel(T* p, T v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return TC_OK;
  fill_kernel<int32_t><<<grid_for(count, 256 * 8, 65536), 256, 0, s>>>(p, v, count);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return TC_OK;
  fill_kernel<int64_t><<<grid_for(count, 256 * 8, 65536), 256, 0, s>>>(p, v, count);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

// --------------------------------------------------------------- scan
// Reduce-then-scan over tiles of kScanTile values (256 threads x 8 items,
// each thread owning 8 consecutive values).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

template <class T>
struct LoadAll {
  const T* p;
  __device__ __forceinline__ int64_t operator()(int64_t i) const { return static_cast<int64_t>(p[i]); }
};

struct LoadPair {
  const int32_t* p;
  int32_t a, b;
  __device__ __forceinline__ int64_t operator()(int64_t i) const {
    const int32_t v = p[i];
    return v == a ? 1 : (v == b ? (int64_t(1) << 32) : 0);
  }
};

struct LoadStrided {
  const int32_t* p;
  int64_t stride;
  __device__ __forceinline__ int64_t operator()(int64_t i) const { return static_cast<int64_t>(p[i * stride]); }
};

template <class F>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(F in, int64_t count, int64_t* partial) {
  __shared__ int64_t sh[kScanThreads / kWave + 1];
  const int64_t base = blockIdx.x * kScanTile + threadIdx.x * (int64_t)kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < count) s += in(base + i);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Scans each tile; adds the scanned tile offset (nullable -> 0); writes
// out[count] = total when this tile holds the last element.
template <class F>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(F in, int64_t count, const int64_t* tile_off,
                                                                   int64_t* out) {
  __shared__ int64_t sh[kScanThreads / kWave + 1];
  const int64_t base = blockIdx.x * kScanTile + threadIdx.x * (int64_t)kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < count) ? in(base + i) : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t run = block_excl_scan(s, sh, &tot);
  if (tile_off) run += tile_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) out[base + i] = run;
    run += v[i];
  }
  if (base < count && base + kScanItems >= count) out[count] = run;
}

size_t scan_ws_bytes(int64_t count) {
  size_t b = 0;
  while (count > kScanTile) {
    int64_t tiles = (count + kScanTile - 1) / kScanTile;
    b += 2 * (((tiles + 1) * sizeof(int64_t) + 255) & ~size_t(255));
    count = tiles;
  }
  return b + 256;
}

template <class F>
static int scan_impl(F in, int64_t* out, int64_t count, Carver& ws, hipStream_t s) {
  if (count <= 0) return fill_i64(out, 0, 1, s);
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    scan_apply_kernel<F><<<1, kScanThreads, 0, s>>>(in, count, nullptr, out);
    TC_HIP(hipGetLastError());
    return TC_OK;
  }
  int64_t* partial = ws.take<int64_t>(tiles + 1);
  scan_reduce_kernel<F><<<(unsigned)tiles, kScanThreads, 0, s>>>(in, count, partial);
  TC_HIP(hipGetLastError());
  // the tile sums are scanned into a fresh buffer (recursively)
  int64_t* partial_scan = ws.take<int64_t>(tiles + 1);
  TC_TRY(scan_impl(LoadAll<int64_t>{partial}, partial_scan, tiles, ws, s));
  scan_apply_kernel<F><<<(unsigned)tiles, kScanThreads, 0, s>>>(in, count, partial_scan, out);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

template <class T>
int scan_exclusive(const T* in, int64_t* out, int64_t count, Carver& ws, hipStream_t s) {
  return scan_impl(LoadAll<T>{in}, out, count, ws, s);
}

int scan_exclusive_pair(const int32_t* in, int32_t a, int32_t b, int64_t* out, int64_t count, Carver& ws,
                        hipStream_t s) {
  if (count >= (int64_t(1) << 32)) return TC_ERR_INVALID_ARG;
  return scan_impl(LoadPair{in, a, b}, out, count, ws, s);
}

int scan_exclusive_strided(const int32_t* in, int64_t stride, int64_t* out, int64_t count, Carver& ws,
                           hipStream_t s) {
  return scan_impl(LoadStrided{in, stride}, out, count, ws, s);
}

template int scan_exclusive<int32_t>(const int32_t*, int64_t*, int64_t, Carver&, hipStream_t);
template int scan_exclusive<int64_t>(const int64_t*, int64_t*, int64_t, Carver&, hipStream_t);

}  // namespace tc
