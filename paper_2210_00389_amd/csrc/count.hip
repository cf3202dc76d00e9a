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
// (edge, apex) pairs, enumerated per apex the way the paper's distributed
// variant enumerates the apexes a processor owns; it streams the short
// up-lists of the apexes instead of the long down-lists of hub pairs.
//
// Every intersection is a "task": stream one sorted list S, test each element
// for membership in a probe list P of an anchor vertex.  Ownership rules pick
// the cheaper side per task:
//   up     anchor = u if |Up(v)| <= |Up(u)| else v; stream Up(other)
//   same   a = |Hfwd(u) ∩ (v,inf)|, b = |Hfwd(v)|; if b < a anchor u streams
//          Hfwd(v), else anchor v streams Hfwd(u) ∩ (v,inf)
//   down   anchor x streams Up(w) ∩ (x,inf)
// Light anchors (short probe set, few down-neighbours) have their tasks
// merged by the thread that discovers them.  Heavy anchors become work items
// of at most D descriptors, binned by probe-set size: a block builds an LDS
// hash of the anchor's probe set Up(x) ∪ Hfwd(x) (2 KB .. 128 KB of the
// 160 KB LDS), resolves all descriptors of the item with independent loads,
// then every lane takes K consecutive elements of the flattened streams (one
// LDS search, K independent global loads in flight, K probes).  Probe sets
// beyond the largest table are searched in their sorted rows instead.
// Per-lane counts are reduced wave -> block -> one 64-bit atomic.
//
// The comparator (plain direction-oriented edge iterator) runs through the
// same kernels with up = 0, Hfwd = forward list N+(x), no down class.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kDnLight = 16;  // light anchors have at most this many down-neighbours
constexpr int kK = 8;         // elements per lane per round
constexpr int kBins = 4;

// Bins of heavy anchors by the LDS table they need: 2 KB, 16 KB, 128 KB, or
// none (bin 3: search the sorted rows).  The probe set P(x) = Up(x) ∪ Hfwd(x)
// lies in the id window [min P, max P] of R ids; it is held as a bitmap of R
// bits when that is at most about four words per member (so setting it up
// costs O(|P|)), else as a hash table of 2|P| (rounded up) slots.
constexpr int kBinWords0 = 512, kBinWords1 = 4096, kBinWords2 = 32768;

__host__ __device__ constexpr int bin_words(int b) {
  return b == 0 ? kBinWords0 : (b == 1 ? kBinWords1 : (b == 2 ? kBinWords2 : 0));
}

__device__ __forceinline__ bool bitmap_fits(int64_t R, int P, int words) {
  const int64_t need = (R + 31) >> 5;
  return need <= words && need <= 4 * static_cast<int64_t>(P) + 64;
}

__device__ __forceinline__ bool hash_fits(int P, int words) { return 2 * P <= words; }

enum Acc {
  kAccT = 0, kAccElems = 1, kAccLight = 2, kAccBuild = 3, kAccDesc = 4, kAccItems = 5,
  kAccHeavyElems = 6, kAccBinCount = 8, kAccBinOff = 13, kAccBinCur = 18, kAccBinNext = 23
};
constexpr int kAccSlots = 28;

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

// Membership of t in a sorted list [p, p + len) in global memory.
__device__ __forceinline__ bool gsearch(const int32_t* p, int len, int32_t t) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (p[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && p[lo] == t;
}

__device__ __forceinline__ int probe_size(const VMeta& m) { return m.up + (m.sfe - m.hfb); }

// Heavy anchors get work items; every task of a light anchor is merged by
// the planning kernels.  Must be the same predicate everywhere.
__device__ __forceinline__ bool is_heavy(const VMeta& m, bool cover, int light_max) {
  if (probe_size(m) > light_max) return true;
  return cover && (m.sfe - m.hfb) > 0 && (m.deg - m.sfe) > kDnLight;
}

__device__ __forceinline__ void block_acc(unsigned long long* acc, int slot, int64_t v, int64_t* sh) {
  int64_t s = block_sum(v, sh);
  if (threadIdx.x == 0 && s) atomicAdd(&acc[slot], static_cast<unsigned long long>(s));
}

// ------------------------------------------------------------ planning
// One thread per cover edge e = (u, v), v the i-th entry of Hfwd(u).
// kFill = false: light tasks are merged and counted; heavy "same" tasks whose
// anchor is v are counted per anchor.  kFill = true: those tasks are written.
template <bool kCover, bool kPV, bool kFill>
__global__ __launch_bounds__(kThreads) void plan_kernel(
    const int32_t* lc, const VMeta* meta, int64_t n, const int64_t* h_off, const int32_t* h_u,
    const int32_t* h_v, int light_max, int32_t* ecnt, const int64_t* task_off, int32_t* ecur,
    int64_t* task_begin, int32_t* task_len, int32_t* task_owner, unsigned long long* acc, int64_t* pv) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  const int64_t H = h_off[n];
  int64_t cnt = 0, light = 0, elems = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < H; e += stride) {
    const int32_t u = h_u[e], v = h_v[e];
    const VMeta mu = meta[u], mv = meta[v];
    const int i = static_cast<int>(e - h_off[u]);
    if (kCover && !kFill) {
      const bool anchor_u = mv.up <= mu.up;
      const VMeta& ma = anchor_u ? mu : mv;
      const VMeta& mo = anchor_u ? mv : mu;
      if (mo.up > 0 && !is_heavy(ma, kCover, light_max)) {
        cnt += merge_count<kPV>(lc + mo.begin, mo.up, lc + ma.begin, ma.up, -1, pv, u, v);
        ++light;
        elems += mo.up;
      }
    }
    const int a = (mu.sfe - mu.hfb) - i - 1;
    const int b = mv.sfe - mv.hfb;
    if (a > 0 && b > 0) {
      const int32_t* Su = lc + mu.begin + mu.hfb + i + 1;  // Hfwd(u) above v
      const int32_t* Sv = lc + mv.begin + mv.hfb;          // Hfwd(v)
      if (b < a) {  // anchor u
        if (!kFill && !is_heavy(mu, kCover, light_max)) {
          cnt += merge_count<kPV>(Sv, b, Su, a, -1, pv, u, v);
          ++light;
          elems += b;
        }
      } else {  // anchor v
        if (!is_heavy(mv, kCover, light_max)) {
          if (!kFill) {
            cnt += merge_count<kPV>(Su, a, Sv, b, -1, pv, u, v);
            ++light;
            elems += a;
          }
        } else if (!kFill) {
          atomicAdd(&ecnt[v], 1);
        } else {
          const int64_t pos = task_off[v] + atomicAdd(&ecur[v], 1);
          task_begin[pos] = mu.begin + mu.hfb + i + 1;
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

// Down class of light anchors (at most kDnLight down-neighbours): one
// thread per pair (x, k-th down-neighbour w) counts |Up(w) ∩ Hfwd(x)| (every
// element of Hfwd(x) lies above x, so no filter is needed), by a merge, or
// by searching the short list in the long one when Up(w) is long.
template <bool kPV>
__global__ __launch_bounds__(kThreads) void light_down_kernel(const int32_t* lc, const VMeta* meta, int64_t n,
                                                              int light_max, unsigned long long* acc,
                                                              int64_t* pv) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t cnt = 0, elems = 0, light = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t total = n * kDnLight;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t x = idx / kDnLight;
    const int k = static_cast<int>(idx % kDnLight);
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb, nd = m.deg - m.sfe;
    if (hf == 0 || k >= nd || is_heavy(m, true, light_max)) continue;
    const int32_t w = lc[m.begin + m.sfe + k];
    const VMeta mw = meta[w];
    const int32_t* S = lc + mw.begin;
    const int32_t* P = lc + m.begin + m.hfb;
    if (mw.up > 4 * hf) {
      for (int i = 0; i < hf; ++i) {
        const int32_t t = P[i];
        if (gsearch(S, mw.up, t)) {
          ++cnt;
          if (kPV) add_pv(pv, static_cast<int32_t>(x), w, t);
        }
      }
      elems += hf;
    } else {
      cnt += merge_count<kPV>(S, mw.up, P, hf, -1, pv, static_cast<int32_t>(x), w);
      elems += mw.up;
    }
    ++light;
  }
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccElems, elems, sh);
  block_acc(acc, kAccLight, light, sh);
}

// ---------------------------------------------------------- heavy items
// Descriptor index space of an anchor: [down | fwd-up | fwd-same | bwd-up | tasks].
struct Desc {
  int nB, nCu, nCs, nD, nE;
  __device__ __forceinline__ int total() const { return nB + nCu + nCs + nD + nE; }
};

__device__ __forceinline__ Desc desc_of(const VMeta& m, bool cover, int nE) {
  Desc d;
  const int hf = m.sfe - m.hfb;
  d.nB = (cover && hf > 0) ? m.deg - m.sfe : 0;
  d.nCu = (cover && m.up > 0) ? hf : 0;
  d.nCs = hf;
  d.nD = (cover && m.up > 0) ? m.hfb - m.up : 0;
  d.nE = nE;
  return d;
}

// Id window [lo, lo + R) of the probe set (R = 0 when it is empty).
__device__ __forceinline__ void probe_window(const int32_t* lc, const VMeta& m, int32_t& lo, int64_t& R) {
  const int hf = m.sfe - m.hfb;
  int32_t mn = 0x7FFFFFFF, mx = -1;
  if (m.up > 0) {
    mn = lc[m.begin];
    mx = lc[m.begin + m.up - 1];
  }
  if (hf > 0) {
    mn = min(mn, lc[m.begin + m.hfb]);
    mx = max(mx, lc[m.begin + m.sfe - 1]);
  }
  lo = mn;
  R = mx >= mn ? static_cast<int64_t>(mx) - mn + 1 : 0;
}

__device__ __forceinline__ int bin_of(int64_t R, int P) {
  for (int b = 0; b < 3; ++b)
    if (bitmap_fits(R, P, bin_words(b)) || hash_fits(P, bin_words(b))) return b;
  return 3;
}

__host__ __device__ constexpr int bin_chunk(int b) { return b == 0 ? 256 : 1024; }

// kFill = false: count items per bin.  kFill = true: write them.
template <bool kFill>
__global__ __launch_bounds__(kThreads) void items_kernel(const int32_t* lc, const VMeta* meta, int64_t n,
                                                         const int64_t* task_off,
                                                         bool cover, int light_max, int2* items,
                                                         unsigned long long* acc) {
  __shared__ int s_cnt[kBins];
  __shared__ unsigned long long s_base[kBins];
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < kBins) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t x = x0 + threadIdx.x;
    int k = 0, b = 0, mine = 0;
    if (x < n) {
      const VMeta m = meta[x];
      if (is_heavy(m, cover, light_max)) {
        const Desc d = desc_of(m, cover, static_cast<int>(task_off[x + 1] - task_off[x]));
        int32_t lo;
        int64_t R;
        probe_window(lc, m, lo, R);
        b = bin_of(R, probe_size(m));
        const int ch = bin_chunk(b);
        k = (d.total() + ch - 1) / ch;
        if (k) mine = atomicAdd(&s_cnt[b], k);
      }
    }
    __syncthreads();
    if (threadIdx.x < kBins && s_cnt[threadIdx.x]) {
      const unsigned long long c = static_cast<unsigned long long>(s_cnt[threadIdx.x]);
      if (!kFill) atomicAdd(&acc[kAccBinCount + threadIdx.x], c);
      else s_base[threadIdx.x] = acc[kAccBinOff + threadIdx.x] + atomicAdd(&acc[kAccBinCur + threadIdx.x], c);
    }
    __syncthreads();
    if (kFill && k) {
      const unsigned long long base = s_base[b] + mine;
      for (int j = 0; j < k; ++j) items[base + j] = make_int2(static_cast<int>(x), j);
    }
    __syncthreads();
  }
}

__global__ void bin_offsets_kernel(unsigned long long* acc) {
  unsigned long long run = 0;
  for (int b = 0; b < kBins; ++b) {
    acc[kAccBinOff + b] = run;
    run += acc[kAccBinCount + b];
  }
  acc[kAccItems] = run;
}

__device__ __forceinline__ uint32_t hslot(int32_t key, int shift) {
  return (static_cast<uint32_t>(key) * 0x9E3779B1u) >> shift;
}


enum ProbeMode { kBitmap = 0, kHash = 1, kSearch = 2 };

// Membership of t in the anchor's probe set: LDS bitmap over the id window
// [lo, lo + R), LDS hash table, or binary search in the sorted Up / Hfwd
// segments of the anchor's row.
template <int MODE>
__device__ __forceinline__ bool probe(const uint32_t* tab, int cap, int shift, int32_t lo, uint32_t R,
                                      const int32_t* lc, const VMeta& mx, bool up_side, int32_t t) {
  if (MODE == kBitmap) {
    const uint32_t d = static_cast<uint32_t>(t - lo);
    const bool in = d < R;
    const uint32_t word = tab[in ? (d >> 5) : 0];
    return in && ((word >> (d & 31)) & 1u);
  } else if (MODE == kHash) {
    uint32_t h = hslot(t, shift);
    int32_t k;
    while ((k = static_cast<int32_t>(tab[h])) != t && k != -1) h = (h + 1) & (cap - 1);
    return k == t;
  }
  return up_side ? gsearch(lc + mx.begin, mx.up, t) : gsearch(lc + mx.begin + mx.hfb, mx.sfe - mx.hfb, t);
}

// `mode` is the same for the whole block (one item at a time).
__device__ __forceinline__ bool probe_any(int mode, const uint32_t* tab, int cap, int shift, int32_t lo, uint32_t R,
                                          const int32_t* lc, const VMeta& mx, bool up_side, int32_t t) {
  if (mode == kBitmap) return probe<kBitmap>(tab, cap, shift, lo, R, lc, mx, up_side, t);
  if (mode == kHash) return probe<kHash>(tab, cap, shift, lo, R, lc, mx, up_side, t);
  return probe<kSearch>(tab, cap, shift, lo, R, lc, mx, up_side, t);
}

// One block per work item (anchor x, descriptor chunk).  WORDS is the LDS
// table size in 32-bit words (0: search the sorted rows); each item picks a
// bitmap or a hash table (see bitmap_fits); D = descriptors per item.  Short streams (<= kShortStream elements) are handled by the lane
// that resolved them, with all loads issued before the probes; longer
// streams are flattened across the block, K consecutive elements per lane.
constexpr int kShortStream = 16;

template <int WORDS, int THREADS, int D, bool kCover, bool kPV>
__global__ __launch_bounds__(THREADS) void heavy_kernel(const int32_t* lc, const VMeta* meta, int bin,
                                                        const int2* items, const int64_t* task_off,
                                                        const int64_t* task_begin, const int32_t* task_len,
                                                        const int32_t* task_owner, unsigned long long* acc,
                                                        int64_t* pv) {
  constexpr int R = D / THREADS;  // descriptors resolved per thread
  static_assert(R * THREADS == D, "D must be a multiple of THREADS");
  __shared__ uint32_t tab[WORDS > 0 ? WORDS : 1];
  __shared__ int64_t s_beg[D];
  __shared__ int64_t s_pre[D + 1];
  __shared__ int32_t s_flt[D];
  __shared__ int32_t s_oth[kPV ? D : 1];
  __shared__ uint8_t s_up[WORDS == 0 ? D : 1];
  __shared__ int64_t sh[THREADS / kWave + 1];
  __shared__ int32_t shi[THREADS / kWave + 1];
  __shared__ unsigned long long s_item;

  const unsigned long long first = acc[kAccBinOff + bin];
  const unsigned long long count = acc[kAccBinCount + bin];
  const int tid = threadIdx.x;
  int64_t cnt = 0, elems = 0, descs = 0, builds = 0;
  int32_t cur_x = -1;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(&acc[kAccBinNext + bin], 1ull);
    __syncthreads();
    const unsigned long long it = s_item;
    __syncthreads();
    if (it >= count) break;
    const int2 item = items[first + it];
    const int32_t x = item.x;
    const VMeta mx = meta[x];
    const int hf = mx.sfe - mx.hfb;
    const int P = mx.up + hf;
    const int64_t toff = task_off[x];
    const Desc Dx = desc_of(mx, kCover, static_cast<int>(task_off[x + 1] - toff));
    const int d0 = item.y * D;
    const int nd = min(Dx.total() - d0, D);
    int cap = 64, shift = 26;
    int32_t wlo = 0;
    uint32_t wR = 0;
    int mode = kSearch;
    if (WORDS > 0) {
      int64_t R64;
      probe_window(lc, mx, wlo, R64);
      wR = static_cast<uint32_t>(R64);
      mode = bitmap_fits(R64, P, WORDS) ? kBitmap : kHash;
      if (x != cur_x) {
        if (mode == kBitmap) {
          const int words = static_cast<int>((R64 + 31) >> 5);
          for (int i = tid; i < words; i += THREADS) tab[i] = 0u;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const int32_t key = i < mx.up ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            const uint32_t d = static_cast<uint32_t>(key - wlo);
            atomicOr(&tab[d >> 5], 1u << (d & 31));
          }
        } else {
          while (cap < 2 * P) {
            cap <<= 1;
            --shift;
          }
          for (int i = tid; i < cap; i += THREADS) tab[i] = 0xFFFFFFFFu;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const int32_t key = i < mx.up ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            uint32_t h = hslot(key, shift);
            while (atomicCAS(&tab[h], 0xFFFFFFFFu, static_cast<uint32_t>(key)) != 0xFFFFFFFFu)
              h = (h + 1) & (cap - 1);
          }
        }
        __syncthreads();
        cur_x = x;
        builds += tid == 0 ? P : 0;
      } else if (mode == kHash) {
        while (cap < 2 * P) {
          cap <<= 1;
          --shift;
        }
      }
    }
    // ---- resolve this item's descriptors (R per thread, independent loads)
    int64_t lbeg[R];
    int32_t llen[R], lflt[R], loth[R];
    bool lup[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int dl = tid * R + r;
      lbeg[r] = 0;
      llen[r] = 0;
      lflt[r] = -1;
      loth[r] = x;
      lup[r] = false;
      if (dl < nd) {
        int k = d0 + dl;
        if (k < Dx.nB) {  // down class: Up(w) above x
          const int32_t w = lc[mx.begin + mx.sfe + k];
          const VMeta mw = meta[w];
          lbeg[r] = mw.begin;
          llen[r] = mw.up;
          lflt[r] = x;
          loth[r] = w;
        } else if ((k -= Dx.nB) < Dx.nCu) {  // forward cover edge, up class
          const int32_t v = lc[mx.begin + mx.hfb + k];
          const VMeta mv = meta[v];
          loth[r] = v;
          if (mv.up > 0 && mv.up <= mx.up) {
            lbeg[r] = mv.begin;
            llen[r] = mv.up;
            lup[r] = true;
          }
        } else if ((k -= Dx.nCu) < Dx.nCs) {  // forward cover edge, same class
          const int32_t v = lc[mx.begin + mx.hfb + k];
          const VMeta mv = meta[v];
          loth[r] = v;
          const int a = hf - k - 1, b = mv.sfe - mv.hfb;
          if (a > 0 && b > 0 && b < a) {
            lbeg[r] = mv.begin + mv.hfb;
            llen[r] = b;
          }
        } else if ((k -= Dx.nCs) < Dx.nD) {  // backward cover edge, up class
          const int32_t u = lc[mx.begin + mx.up + k];
          const VMeta mu = meta[u];
          loth[r] = u;
          if (mu.up > 0 && mu.up < mx.up) {
            lbeg[r] = mu.begin;
            llen[r] = mu.up;
            lup[r] = true;
          }
        } else {  // emitted same-class task: Hfwd(u) above x
          const int64_t q = toff + (k - Dx.nD);
          lbeg[r] = task_begin[q];
          llen[r] = task_len[q];
          loth[r] = task_owner[q];
        }
      }
    }
    // ---- short streams: by the resolving lane, all loads before the probes
    int64_t longsum = 0;
    int nlong = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int len = llen[r];
      if (len > kShortStream) {
        longsum += len;
        ++nlong;
        continue;
      }
      if (len == 0) continue;
      int32_t val[kShortStream];
#pragma unroll
      for (int q = 0; q < kShortStream; ++q) val[q] = q < len ? lc[lbeg[r] + q] : -1;
#pragma unroll
      for (int q = 0; q < kShortStream; ++q) {
        const int32_t t = val[q];
        if (q < len && t > lflt[r] && probe_any(mode, tab, cap, shift, wlo, wR, lc, mx, lup[r], t)) {
          ++cnt;
          if (kPV) add_pv(pv, x, loth[r], t);
        }
      }
      elems += len;
    }
    // ---- long streams: compact them, then flatten across the block
    int32_t ltot;
    const int32_t lfirst = block_excl_scan(nlong, shi, &ltot);
    int64_t tot;
    int64_t run = block_excl_scan(longsum, sh, &tot);
    {
      int slot = lfirst;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (llen[r] <= kShortStream) continue;
        s_pre[slot] = run;
        s_beg[slot] = lbeg[r];
        s_flt[slot] = lflt[r];
        if (kPV) s_oth[slot] = loth[r];
        if (WORDS == 0) s_up[slot] = lup[r];
        run += llen[r];
        ++slot;
      }
    }
    if (tid == 0) s_pre[ltot] = tot;
    __syncthreads();
    if (tid == 0) {
      elems += tot;
      descs += nd;
    }
    for (int64_t base = 0; base < tot; base += (int64_t)THREADS * kK) {
      const int64_t e0 = base + (int64_t)tid * kK;
      if (e0 < tot) {
        int lo = 0, hi = ltot;  // largest j with s_pre[j] <= e0
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] <= e0) lo = mid;
          else hi = mid;
        }
        int j = lo;
        int64_t cb = s_beg[j], cp = s_pre[j], ce = s_pre[j + 1];
        int32_t cf = s_flt[j];
        int64_t addr[kK];
        int32_t flt[kK];
        int jj[kK];
#pragma unroll
        for (int q = 0; q < kK; ++q) {
          const int64_t e = e0 + q;
          if (e < tot) {
            while (e >= ce) {
              ++j;
              cb = s_beg[j];
              cp = ce;
              ce = s_pre[j + 1];
              cf = s_flt[j];
            }
            addr[q] = cb + (e - cp);
            flt[q] = cf;
          } else {
            addr[q] = -1;
            flt[q] = 0x7FFFFFFF;
          }
          jj[q] = j;
        }
        int32_t val[kK];
#pragma unroll
        for (int q = 0; q < kK; ++q) val[q] = addr[q] >= 0 ? lc[addr[q]] : -1;
#pragma unroll
        for (int q = 0; q < kK; ++q) {
          const int32_t t = val[q];
          if (t > flt[q] && probe_any(mode, tab, cap, shift, wlo, wR, lc, mx, WORDS == 0 && s_up[jj[q]], t)) {
            ++cnt;
            if (kPV) add_pv(pv, x, s_oth[jj[q]], t);
          }
        }
      }
    }
    __syncthreads();
  }
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccHeavyElems, elems, sh);
  block_acc(acc, kAccDesc, descs, sh);
  block_acc(acc, kAccBuild, builds, sh);
}

__global__ void finish_kernel(const unsigned long long* acc, const int64_t* h_off, int64_t n,
                              int64_t* triangles, int64_t* h_count, int64_t* stats) {
  *triangles = static_cast<int64_t>(acc[kAccT]);
  if (h_count) *h_count = h_off[n];
  stats[2] = h_off[n];
  stats[4] = static_cast<int64_t>(acc[kAccElems] + acc[kAccHeavyElems]);
  stats[5] = static_cast<int64_t>(acc[kAccLight]);
  stats[6] = static_cast<int64_t>(acc[kAccItems]);
  stats[7] = static_cast<int64_t>(acc[kAccDesc]);
  stats[8] = static_cast<int64_t>(acc[kAccHeavyElems]);
  stats[9] = static_cast<int64_t>(acc[kAccBuild]);
  stats[10] = static_cast<int64_t>(acc[kAccElems]);
}

__global__ void forward_meta_kernel(const int64_t* off, const int32_t* cols, int64_t n, VMeta* meta) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = off[x], e = off[x + 1];
    const int64_t fb = upper_bound_dev(cols, b, e, static_cast<int32_t>(x));
    const int32_t deg = static_cast<int32_t>(e - b);
    meta[x] = VMeta{b, 0, static_cast<int32_t>(fb - b), deg, deg, {0, 0}};
  }
}

template <int WORDS, int THREADS, int D, bool kCover, bool kPV>
int launch_heavy(const CountArgs& a, CountWs& w, int bin, int blocks_per_cu, hipStream_t s) {
  heavy_kernel<WORDS, THREADS, D, kCover, kPV>
      <<<static_cast<unsigned>(num_cus() * blocks_per_cu), THREADS, 0, s>>>(
          a.cols, a.meta, bin, w.items, w.task_off, w.task_begin, w.task_len, w.task_owner, w.acc,
          a.per_vertex_out);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

template <bool kCover, bool kPV>
int launch_all(const CountArgs& a, CountWs& w, hipStream_t s) {
  const tc_csr* g = a.g;
  const int64_t n = g->n;
  const unsigned gedge = static_cast<unsigned>(num_cus() * 16);
  plan_kernel<kCover, kPV, false><<<gedge, kThreads, 0, s>>>(
      a.cols, a.meta, n, w.h_off, w.h_u, w.h_v, a.light_max, w.ecnt, w.task_off, w.ecur, w.task_begin,
      w.task_len, w.task_owner, w.acc, a.per_vertex_out);
  TC_HIP(hipGetLastError());
  prof_stage("light_down");
  if (kCover) {
    light_down_kernel<kPV><<<grid_for(n * kDnLight, kThreads, 32768), kThreads, 0, s>>>(
        a.cols, a.meta, n, a.light_max, w.acc, a.per_vertex_out);
    TC_HIP(hipGetLastError());
  }
  prof_stage("plan_tasks");
  Carver sc(w.scratch);
  TC_TRY(scan_exclusive<int32_t>(w.ecnt, w.task_off, n, sc, s));
  plan_kernel<kCover, kPV, true><<<gedge, kThreads, 0, s>>>(
      a.cols, a.meta, n, w.h_off, w.h_u, w.h_v, a.light_max, w.ecnt, w.task_off, w.ecur, w.task_begin,
      w.task_len, w.task_owner, w.acc, a.per_vertex_out);
  const unsigned gv = grid_for(n, kThreads, 16384);
  items_kernel<false><<<gv, kThreads, 0, s>>>(a.cols, a.meta, n, w.task_off, kCover, a.light_max, w.items, w.acc);
  bin_offsets_kernel<<<1, 1, 0, s>>>(w.acc);
  items_kernel<true><<<gv, kThreads, 0, s>>>(a.cols, a.meta, n, w.task_off, kCover, a.light_max, w.items, w.acc);
  TC_HIP(hipGetLastError());
  prof_stage("heavy");
  // the four bins are independent: run them side by side
  Fork* f = fork_for_device();
  if (!f) return TC_ERR_HIP;
  TC_TRY(fork_begin(f, s));
  TC_TRY((launch_heavy<kBinWords2, 1024, 1024, kCover, kPV>(a, w, 2, 1, s)));
  TC_TRY((launch_heavy<kBinWords1, 512, 1024, kCover, kPV>(a, w, 1, 3, f->aux[0])));
  TC_TRY((launch_heavy<kBinWords0, 256, 256, kCover, kPV>(a, w, 0, 8, f->aux[1])));
  TC_TRY((launch_heavy<0, 512, 1024, kCover, kPV>(a, w, 3, 4, f->aux[2])));
  TC_TRY(fork_end(f, s));
  prof_stage("finish");
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
  // items: one per heavy anchor plus one per started chunk of >= 256
  // descriptors; descriptors per anchor <= 2 deg + emitted tasks
  w.items = c.take<int2>(n + (3 * nnz) / 256 + 8);
  w.acc = c.take<unsigned long long>(kAccSlots);
  w.stats = c.take<int64_t>(16);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1) + (n + 1) * sizeof(int32_t) + 256);
  return w;
}

int forward_meta_run(const tc_csr* g, VMeta* meta, hipStream_t s) {
  if (g->n == 0) return TC_OK;
  forward_meta_kernel<<<grid_for(g->n, kThreads, 16384), kThreads, 0, s>>>(g->row_offsets, g->cols, g->n, meta);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int count_run(const CountArgs& a, CountWs& w, int64_t* triangles, int64_t* h_count, hipStream_t s) {
  const tc_csr* g = a.g;
  const int64_t n = g->n;
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.acc), 0, kAccSlots, s));
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
