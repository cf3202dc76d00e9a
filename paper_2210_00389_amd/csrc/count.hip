// count.hip -- the intersection stage of Alg. 1 and of the comparator.
//
// The count of Alg. 1 is a sum over (cover edge (u,v), apex w) pairs.  With
// the level-class layout (split.hip) a common neighbour w of a cover edge
// (u, v), u < v, on level l is in exactly one class:
//   up    w on level l-1:  w in Up(u)   ∩ Up(v)     (always counted)
//   same  w on level l:    w in Hfwd(u) ∩ Hfwd(v)   (counted: w > v; Hfwd(v)
//                          holds exactly the same-level neighbours above v)
//   down  w on level l+1:  w in Down(u) ∩ Down(v)   (always counted)
// The down class is summed from the apex side: for every edge x -> w with
// w in Down(x), count the t in Up(w) with t > x and t in Hfwd(x); each
// (u, v, w) with u < v is met once, at x = u, t = v.  This is the same set of
// (edge, apex) pairs, enumerated the way the paper's distributed variant
// enumerates apexes per owner; it streams the short up-lists of the apexes
// instead of the long down-lists of the hub pairs.
//
// Every intersection is a "task": stream one sorted list S, test each element
// for membership in a probe list P of an anchor vertex.  Ownership rules pick
// the cheaper side per task:
//   up     anchor = u if |Up(v)| <= |Up(u)| else v; stream Up(other)
//   same   a = |Hfwd(u) ∩ (v,inf)|, b = |Hfwd(v)|; if b < a anchor u streams
//          Hfwd(v), else anchor v streams Hfwd(u) ∩ (v,inf)
//   down   anchor x streams Up(w) ∩ (x,inf)
// Anchors whose probe set Up(x) ∪ Hfwd(x) is short ("light") have their
// tasks merged right away by the thread that discovers them.  Heavy anchors
// get work items: a block builds an LDS hash of the anchor's probe set once
// per item and streams all of the item's lists through it, flattened across
// the block (a block-wide prefix over list lengths; every lane takes one
// element), so loads are coalesced and lanes stay busy whatever the list
// lengths.  Per-lane counts are reduced wave -> block -> one 64-bit atomic.
//
// The comparator (plain direction-oriented edge iterator) runs through the
// same kernels with up = 0, Hfwd = forward list N+(x), no down class.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kHeavyThreads = 256;
constexpr int kTabMax = 8192;  // LDS hash slots (32 KB)

enum Acc { kAccT = 0, kAccElems = 1, kAccLight = 2, kAccItems = 3, kAccDesc = 4, kAccItemCtr = 5,
           kAccItemNext = 6 };

__device__ __forceinline__ void add_pv(int64_t* pv, int32_t a, int32_t b, int32_t c) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[a]), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[b]), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[c]), 1ull);
}

// |{t in S : t > lo} ∩ P| by a two-pointer merge (both ascending).
template <bool kPV>
__device__ __forceinline__ int64_t merge_count(const int32_t* S, int ns, const int32_t* P, int np,
                                               int32_t lo, int64_t* pv, int32_t f1, int32_t f2) {
  int i = 0, j = 0;
  int64_t c = 0;
  while (i < ns && j < np) {
    int32_t s = S[i], p = P[j];
    if (s <= lo) { ++i; continue; }
    if (s < p) ++i;
    else if (s > p) ++j;
    else {
      ++c;
      if (kPV) add_pv(pv, f1, f2, s);
      ++i;
      ++j;
    }
  }
  return c;
}

__device__ __forceinline__ bool is_light(const VMeta& m, int light_max) {
  return (m.up + (m.sfe - m.hfb)) <= light_max;
}

__device__ __forceinline__ void block_acc(unsigned long long* acc, int slot, int64_t v, int64_t* sh) {
  int64_t s = block_sum(v, sh);
  if (threadIdx.x == 0 && s) atomicAdd(&acc[slot], static_cast<unsigned long long>(s));
}

// ------------------------------------------------------------ planning
// One thread per cover edge e = (u, v), v the i-th entry of Hfwd(u).
// kFill = false: light tasks are merged and counted, heavy "same" tasks whose
// anchor is v are counted per anchor.  kFill = true: those tasks are written.
template <bool kCover, bool kPV, bool kFill>
__global__ __launch_bounds__(kThreads) void plan_kernel(
    const int64_t* off, const int32_t* lc, const VMeta* meta, int64_t n, const int64_t* h_off,
    const int32_t* h_u, const int32_t* h_v, int light_max, int32_t* ecnt, const int64_t* task_off,
    int32_t* ecur, int64_t* task_begin, int32_t* task_len, int32_t* task_owner,
    unsigned long long* acc, int64_t* pv) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  const int64_t H = h_off[n];
  int64_t cnt = 0, light = 0, elems = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < H; e += stride) {
    const int32_t u = h_u[e], v = h_v[e];
    const VMeta mu = meta[u], mv = meta[v];
    const int64_t bu = off[u], bv = off[v];
    const int i = static_cast<int>(e - h_off[u]);
    if (kCover && !kFill) {
      const bool anchor_u = mv.up <= mu.up;
      const VMeta& ma = anchor_u ? mu : mv;
      const VMeta& mo = anchor_u ? mv : mu;
      if (mo.up > 0 && is_light(ma, light_max)) {
        const int64_t ba = anchor_u ? bu : bv, bo = anchor_u ? bv : bu;
        cnt += merge_count<kPV>(lc + bo, mo.up, lc + ba, ma.up, -1, pv, u, v);
        ++light;
        elems += mo.up;
      }
    }
    const int a = (mu.sfe - mu.hfb) - i - 1;
    const int b = mv.sfe - mv.hfb;
    if (a > 0 && b > 0) {
      const int32_t* Su = lc + bu + mu.hfb + i + 1;  // Hfwd(u) above v
      const int32_t* Sv = lc + bv + mv.hfb;          // Hfwd(v)
      if (b < a) {  // anchor u
        if (!kFill && is_light(mu, light_max)) {
          cnt += merge_count<kPV>(Sv, b, Su, a, -1, pv, u, v);
          ++light;
          elems += b;
        }
      } else {  // anchor v
        if (is_light(mv, light_max)) {
          if (!kFill) {
            cnt += merge_count<kPV>(Su, a, Sv, b, -1, pv, u, v);
            ++light;
            elems += a;
          }
        } else if (!kFill) {
          atomicAdd(&ecnt[v], 1);
        } else {
          const int64_t pos = task_off[v] + atomicAdd(&ecur[v], 1);
          task_begin[pos] = bu + mu.hfb + i + 1;
          task_len[pos] = a;
          task_owner[pos] = u;
        }
      }
    }
  }
  if (!kFill) {
    block_acc(acc, kAccT, cnt, sh);
    block_acc(acc, kAccLight, light, sh);
    block_acc(acc, kAccElems, elems, sh);
  }
}

// Down class for light anchors: x -> w with w in Down(x); t in Up(w), t > x,
// t in Hfwd(x).  Short down-lists by one thread, long ones by one wave.
template <bool kPV>
__global__ __launch_bounds__(kThreads) void light_down_kernel(const int64_t* off, const int32_t* lc,
                                                              const VMeta* meta, int64_t n, int light_max,
                                                              unsigned long long* acc, int64_t* pv) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t cnt = 0, elems = 0, light = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  constexpr int kShortDown = 16;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += stride) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb, nd = m.deg - m.sfe;
    if (hf == 0 || nd == 0 || nd > kShortDown || !is_light(m, light_max)) continue;
    const int64_t bx = off[x];
    for (int k = 0; k < nd; ++k) {
      const int32_t w = lc[bx + m.sfe + k];
      const int upw = meta[w].up;
      cnt += merge_count<kPV>(lc + off[w], upw, lc + bx + m.hfb, hf, static_cast<int32_t>(x), pv,
                              static_cast<int32_t>(x), w);
      elems += upw;
      ++light;
    }
  }
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = stride / kWave;
  for (int64_t x = wid; x < n; x += nw) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb, nd = m.deg - m.sfe;
    if (hf == 0 || nd <= kShortDown || !is_light(m, light_max)) continue;
    const int64_t bx = off[x];
    for (int k = lane(); k < nd; k += kWave) {
      const int32_t w = lc[bx + m.sfe + k];
      const int upw = meta[w].up;
      cnt += merge_count<kPV>(lc + off[w], upw, lc + bx + m.hfb, hf, static_cast<int32_t>(x), pv,
                              static_cast<int32_t>(x), w);
      elems += upw;
      ++light;
    }
  }
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccElems, elems, sh);
  block_acc(acc, kAccLight, light, sh);
}

// ---------------------------------------------------------- heavy items
struct Desc {
  int nB, nC, nD, nE;
  __device__ __forceinline__ int total() const { return nB + nC + nD + nE; }
};

__device__ __forceinline__ Desc desc_of(const VMeta& m, bool cover, int nE) {
  Desc d;
  const int hf = m.sfe - m.hfb;
  d.nB = (cover && hf > 0) ? m.deg - m.sfe : 0;
  d.nC = hf;
  d.nD = (cover && m.up > 0) ? m.hfb - m.up : 0;
  d.nE = nE;
  return d;
}

__global__ void items_kernel(const VMeta* meta, int64_t n, const int64_t* task_off, bool cover,
                             int light_max, int chunk, int2* items, unsigned long long* acc) {
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = x0 + threadIdx.x;
    int k = 0;
    if (x < n) {
      const VMeta m = meta[x];
      if (!is_light(m, light_max)) {
        const Desc d = desc_of(m, cover, static_cast<int>(task_off[x + 1] - task_off[x]));
        k = (d.total() + chunk - 1) / chunk;
      }
    }
    const int incl = wave_incl_scan(k);
    const int tot = __shfl(incl, kWave - 1, kWave);
    unsigned long long base = 0;
    if (lane() == kWave - 1 && tot) base = atomicAdd(&acc[kAccItemCtr], static_cast<unsigned long long>(tot));
    base = __shfl(base, kWave - 1, kWave);
    for (int j = 0; j < k; ++j) items[base + incl - k + j] = make_int2(static_cast<int>(x), j);
  }
}

__device__ __forceinline__ uint32_t hslot(int32_t key, int shift) {
  return (static_cast<uint32_t>(key) * 0x9E3779B1u) >> shift;
}

// Membership of t in a sorted global list [p, p + len).
__device__ __forceinline__ bool gsearch(const int32_t* p, int len, int32_t t) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int32_t v = p[mid];
    if (v < t) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && p[lo] == t;
}

template <bool kCover, bool kPV>
__global__ __launch_bounds__(kHeavyThreads) void heavy_kernel(
    const int64_t* off, const int32_t* lc, const VMeta* meta, const int2* items, const int64_t* task_off,
    const int64_t* task_begin, const int32_t* task_len, const int32_t* task_owner, int chunk,
    unsigned long long* acc, int64_t* pv) {
  __shared__ int32_t tab[kTabMax];
  __shared__ int64_t s_pre[kHeavyThreads + 1];
  __shared__ int64_t s_beg1[kHeavyThreads];
  __shared__ int64_t s_beg2[kHeavyThreads];
  __shared__ int32_t s_len1[kHeavyThreads];
  __shared__ int32_t s_flt[kHeavyThreads];
  __shared__ int32_t s_oth[kHeavyThreads];
  __shared__ uint8_t s_kind[kHeavyThreads];
  __shared__ int64_t sh[kHeavyThreads / kWave + 1];
  __shared__ int s_item;

  const int64_t num_items = static_cast<int64_t>(acc[kAccItemCtr]);
  const int tid = threadIdx.x;
  int64_t cnt = 0, elems = 0, descs = 0;
  int32_t cur_x = -1;
  for (;;) {
    if (tid == 0) s_item = static_cast<int>(atomicAdd(&acc[kAccItemNext], 1ull));
    __syncthreads();
    const int64_t it = s_item;
    __syncthreads();
    if (it >= num_items) break;
    const int2 item = items[it];
    const int32_t x = item.x;
    const VMeta mx = meta[x];
    const int64_t bx = off[x];
    const int hf = mx.sfe - mx.hfb;
    const int P = mx.up + hf;
    const int64_t toff = task_off[x];
    const Desc D = desc_of(mx, kCover, static_cast<int>(task_off[x + 1] - toff));
    const int d0 = item.y * chunk;
    const int d1 = min(D.total(), d0 + chunk);
    const bool use_tab = P <= kTabMax / 2;
    int cap = 64, lg = 6;
    while (cap < 2 * P) { cap <<= 1; ++lg; }
    const int shift = 32 - lg;
    if (use_tab && x != cur_x) {
      for (int i = tid; i < cap; i += kHeavyThreads) tab[i] = -1;
      __syncthreads();
      for (int i = tid; i < P; i += kHeavyThreads) {
        const int32_t key = i < mx.up ? lc[bx + i] : lc[bx + mx.hfb + (i - mx.up)];
        uint32_t h = hslot(key, shift);
        while (atomicCAS(&tab[h], -1, key) != -1) h = (h + 1) & (cap - 1);
      }
      __syncthreads();
      cur_x = x;
    } else if (!use_tab) {
      cur_x = -1;
    }
    descs += d1 - d0;
    for (int db = d0; db < d1; db += kHeavyThreads) {
      const int d = db + tid;
      int len1 = 0, len2 = 0, flt = -1, oth = x;
      int64_t beg1 = 0, beg2 = 0;
      uint8_t kind = 0;  // bit0: stream 1 probes Up(x); bit1: stream 2 probes Up(x)
      if (d < d1) {
        if (d < D.nB) {  // down class: Up(w) above x
          const int32_t w = lc[bx + mx.sfe + d];
          len1 = meta[w].up;
          beg1 = off[w];
          flt = x;
          oth = w;
        } else if (d < D.nB + D.nC) {  // forward cover edges (x, v)
          const int i = d - D.nB;
          const int32_t v = lc[bx + mx.hfb + i];
          const VMeta mv = meta[v];
          const int64_t bv = off[v];
          oth = v;
          if (kCover && mv.up > 0 && mv.up <= mx.up) {
            len1 = mv.up;
            beg1 = bv;
            kind |= 1;
          }
          const int a = hf - i - 1, b = mv.sfe - mv.hfb;
          if (a > 0 && b > 0 && b < a) {
            len2 = b;
            beg2 = bv + mv.hfb;
          }
        } else if (d < D.nB + D.nC + D.nD) {  // backward cover edges (u, x), up class
          const int j = d - D.nB - D.nC;
          const int32_t u = lc[bx + mx.up + j];
          const VMeta mu = meta[u];
          oth = u;
          if (mu.up > 0 && mu.up < mx.up) {
            len1 = mu.up;
            beg1 = off[u];
            kind |= 1;
          }
        } else {  // emitted same-class tasks: Hfwd(u) above x
          const int64_t q = toff + (d - D.nB - D.nC - D.nD);
          len1 = task_len[q];
          beg1 = task_begin[q];
          oth = task_owner[q];
        }
      }
      int64_t tot;
      const int64_t ex = block_excl_scan(static_cast<int64_t>(len1 + len2), sh, &tot);
      s_pre[tid] = ex;
      s_beg1[tid] = beg1;
      s_beg2[tid] = beg2;
      s_len1[tid] = len1;
      s_flt[tid] = flt;
      s_oth[tid] = oth;
      s_kind[tid] = kind;
      if (tid == 0) s_pre[kHeavyThreads] = tot;
      __syncthreads();
      elems += (tid == 0) ? tot : 0;
      for (int64_t e = tid; e < tot; e += kHeavyThreads) {
        // owner thread j: s_pre[j] <= e < s_pre[j + 1]
        int lo = 0, hi = kHeavyThreads;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] <= e) lo = mid;
          else hi = mid;
        }
        const int j = lo;
        const int64_t r = e - s_pre[j];
        const int l1 = s_len1[j];
        int64_t addr;
        int32_t fl;
        bool up_probe;
        if (r < l1) {
          addr = s_beg1[j] + r;
          fl = s_flt[j];
          up_probe = s_kind[j] & 1;
        } else {
          addr = s_beg2[j] + (r - l1);
          fl = -1;
          up_probe = (s_kind[j] >> 1) & 1;
        }
        const int32_t t = lc[addr];
        if (t > fl) {
          bool hit;
          if (use_tab) {
            uint32_t h = hslot(t, shift);
            int32_t k;
            while ((k = tab[h]) != t && k != -1) h = (h + 1) & (cap - 1);
            hit = k == t;
          } else {
            hit = up_probe ? gsearch(lc + bx, mx.up, t) : gsearch(lc + bx + mx.hfb, hf, t);
          }
          if (hit) {
            ++cnt;
            if (kPV) add_pv(pv, x, s_oth[j], t);
          }
        }
      }
      __syncthreads();
    }
  }
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccElems, elems, sh);
  block_acc(acc, kAccDesc, descs, sh);
}

__global__ void finish_kernel(const unsigned long long* acc, const int64_t* h_off, int64_t n,
                              int64_t* triangles, int64_t* h_count, int64_t* stats) {
  *triangles = static_cast<int64_t>(acc[kAccT]);
  if (h_count) *h_count = h_off[n];
  stats[2] = h_off[n];
  stats[4] = static_cast<int64_t>(acc[kAccElems]);
  stats[5] = static_cast<int64_t>(acc[kAccLight]);
  stats[6] = static_cast<int64_t>(acc[kAccItemCtr]);
  stats[7] = static_cast<int64_t>(acc[kAccDesc]);
}

__global__ void forward_meta_kernel(const int64_t* off, const int32_t* cols, int64_t n, VMeta* meta) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = off[x], e = off[x + 1];
    const int64_t fb = upper_bound_dev(cols, b, e, static_cast<int32_t>(x));
    const int32_t deg = static_cast<int32_t>(e - b);
    meta[x] = VMeta{0, static_cast<int32_t>(fb - b), deg, deg};
  }
}

template <bool kCover, bool kPV>
int launch_all(const CountArgs& a, CountWs& w, hipStream_t s) {
  const tc_csr* g = a.g;
  const int64_t n = g->n;
  const unsigned gedge = static_cast<unsigned>(num_cus() * 16);
  plan_kernel<kCover, kPV, false><<<gedge, kThreads, 0, s>>>(
      g->row_offsets, a.cols, a.meta, n, w.h_off, w.h_u, w.h_v, a.light_max, w.ecnt, w.task_off,
      w.ecur, w.task_begin, w.task_len, w.task_owner, w.acc, a.per_vertex_out);
  TC_HIP(hipGetLastError());
  prof_stage("light_down");
  if (kCover) {
    light_down_kernel<kPV><<<gedge, kThreads, 0, s>>>(g->row_offsets, a.cols, a.meta, n, a.light_max, w.acc,
                                                      a.per_vertex_out);
    TC_HIP(hipGetLastError());
  }
  prof_stage("plan_tasks");
  Carver sc(w.scratch);
  TC_TRY(scan_exclusive<int32_t>(w.ecnt, w.task_off, n, sc, s));
  plan_kernel<kCover, kPV, true><<<gedge, kThreads, 0, s>>>(
      g->row_offsets, a.cols, a.meta, n, w.h_off, w.h_u, w.h_v, a.light_max, w.ecnt, w.task_off,
      w.ecur, w.task_begin, w.task_len, w.task_owner, w.acc, a.per_vertex_out);
  items_kernel<<<grid_for(n, kThreads, 16384), kThreads, 0, s>>>(a.meta, n, w.task_off, kCover, a.light_max,
                                                                 a.heavy_chunk, w.items, w.acc);
  TC_HIP(hipGetLastError());
  prof_stage("heavy");
  heavy_kernel<kCover, kPV><<<static_cast<unsigned>(num_cus() * 8), kHeavyThreads, 0, s>>>(
      g->row_offsets, a.cols, a.meta, w.items, w.task_off, w.task_begin, w.task_len, w.task_owner,
      a.heavy_chunk, w.acc, a.per_vertex_out);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace

CountWs count_reserve(Carver& c, int64_t n, int64_t nnz) {
  CountWs w;
  // |H| <= nnz/2 for a symmetric graph; nnz bounds it for any input
  const int64_t hmax = nnz + 1;
  w.h_off = c.take<int64_t>(n + 2);
  w.h_u = c.take<int32_t>(hmax);
  w.h_v = c.take<int32_t>(hmax);
  w.ecnt = c.take<int32_t>(n + 1);
  w.ecur = c.take<int32_t>(n + 1);
  w.task_off = c.take<int64_t>(n + 2);
  w.task_begin = c.take<int64_t>(hmax);
  w.task_len = c.take<int32_t>(hmax);
  w.task_owner = c.take<int32_t>(hmax);
  w.items = c.take<int2>(n + nnz + 2);
  w.acc = c.take<unsigned long long>(16);
  w.stats = c.take<int64_t>(16);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1) + (n + 1) * sizeof(int32_t) + 256);
  return w;
}

int forward_meta_run(const tc_csr* g, VMeta* meta, hipStream_t s) {
  if (g->n == 0) return TC_OK;
  forward_meta_kernel<<<grid_for(g->n, kThreads, 16384), kThreads, 0, s>>>(g->row_offsets, g->cols, g->n,
                                                                          meta);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int count_run(const CountArgs& a, CountWs& w, int64_t* triangles, int64_t* h_count, hipStream_t s) {
  const tc_csr* g = a.g;
  const int64_t n = g->n;
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.acc), 0, 16, s));
  TC_TRY(fill_i64(w.stats, 0, 16, s));
  if (n == 0) {
    TC_TRY(fill_i64(triangles, 0, 1, s));
    if (h_count) TC_TRY(fill_i64(h_count, 0, 1, s));
    return TC_OK;
  }
  TC_TRY(fill_i32(w.ecnt, 0, n, s));
  TC_TRY(fill_i32(w.ecur, 0, n, s));
  prof_stage("hlist");
  TC_TRY(hlist_run(g, a.meta, a.cols, w.h_off, w.h_u, w.h_v, g->nnz + 1, nullptr, w.scratch, s));
  prof_stage("plan_light");
  if (a.cover) {
    if (a.per_vertex) TC_TRY((launch_all<true, true>(a, w, s)));
    else TC_TRY((launch_all<true, false>(a, w, s)));
  } else {
    if (a.per_vertex) TC_TRY((launch_all<false, true>(a, w, s)));
    else TC_TRY((launch_all<false, false>(a, w, s)));
  }
  finish_kernel<<<1, 1, 0, s>>>(w.acc, w.h_off, n, triangles, h_count, w.stats);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
