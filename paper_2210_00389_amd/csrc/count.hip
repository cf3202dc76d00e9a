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
// merged by the thread that discovers them.  For heavy anchors every task
// descriptor is resolved into a stream record (begin, length, flags) by a
// separate pass; the records of an anchor are cut into work items of about
// kElemChunk elements, binned by the on-chip table the anchor's probe set
// Up(x) ∪ Hfwd(x) needs (2 KB .. 128 KB of the 160 KB LDS; bitmap over the
// id window or hash table).  A block builds the table once per anchor and
// streams the item's records in chunks of 8 elements of one stream per lane;
// probe sets beyond the largest table are searched in their sorted rows.
// Per-lane counts are reduced wave -> block -> one 64-bit atomic.
//
// The comparator (plain direction-oriented edge iterator) runs through the
// same kernels with up = 0, Hfwd = forward list N+(x), no down class.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kDnLight = 16;  // light anchors have at most this many down-neighbours
constexpr int kBins = 4;

// Bins of heavy anchors by the LDS table they need: 2 KB, 32 KB, 128 KB, or
// none (bin 3: search the sorted rows).  The probe set P(x) = Up(x) ∪ Hfwd(x)
// lies in the id window [min P, max P] of R ids.  It is held as a bitmap of
// R + 1 bits (bit R stays clear and absorbs every id outside the window)
// when clearing that bitmap costs little next to the anchor's work (at most
// four words per member, or per four streamed elements), else as a hash
// table filling the bin's whole table (at most half full).
constexpr int kBinWords0 = 512, kBinWords1 = 8192, kBinWords2 = 32768;

__host__ __device__ constexpr int bin_words(int b) {
  return b == 0 ? kBinWords0 : (b == 1 ? kBinWords1 : (b == 2 ? kBinWords2 : 0));
}

__device__ __forceinline__ int64_t bitmap_words(int64_t R) { return (R + 32) >> 5; }

// Bin of an anchor with window R, probe-set size P and E streamed elements;
// *bitmap tells the table kind.
__device__ __forceinline__ int choose_bin(int64_t R, int P, int64_t E, bool* bitmap) {
  const int64_t need = bitmap_words(R);
  if (need <= 4 * static_cast<int64_t>(P) + 64 || 4 * need <= E) {
    for (int b = 0; b < 3; ++b)
      if (need <= bin_words(b)) {
        *bitmap = true;
        return b;
      }
  }
  *bitmap = false;
  for (int b = 0; b < 3; ++b)
    if (2 * static_cast<int64_t>(P) <= bin_words(b)) return b;
  return 3;
}

enum Acc {
  kAccT = 0, kAccElems = 1, kAccLight = 2, kAccBuild = 3, kAccDesc = 4, kAccItems = 5,
  kAccHeavyElems = 6, kAccChunks = 7, kAccBinCount = 8, kAccBinOff = 13, kAccBinCur = 18, kAccBinNext = 23,
  kAccBinElems = 28
};
constexpr int kAccSlots = 33;
constexpr int kResolveChunk = 1024;   // descriptors per resolution chunk
constexpr int64_t kElemChunk = 65536;  // elements per work item (target)
// stream record flags (in the length word)
constexpr int32_t kFlagUp = 1 << 29;     // probe the anchor's Up list (row search)
// work item flag (in the stream-count word): the anchor's table is a bitmap
constexpr int32_t kItemBitmap = 1 << 30;
constexpr int64_t kItemMaxStreams = 1 << 29;
constexpr int32_t kLenMask = kFlagUp - 1;

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


// Descriptor counts of heavy anchors and their resolution chunks.
// kFill = false: ndesc per vertex and the chunk count; kFill = true: chunks.
template <bool kFill>
__global__ __launch_bounds__(kThreads) void desc_plan_kernel(const VMeta* meta, int64_t n, const int64_t* task_off,
                                                             bool cover, int light_max, int32_t* ndesc,
                                                             int2* rchunks, int64_t rcap, unsigned long long* acc) {
  __shared__ int s_cnt;
  __shared__ unsigned long long s_base;
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t x = x0 + threadIdx.x;
    int k = 0, mine = 0, total = 0;
    if (x < n) {
      const VMeta m = meta[x];
      if (is_heavy(m, cover, light_max))
        total = desc_of(m, cover, static_cast<int>(task_off[x + 1] - task_off[x])).total();
      k = (total + kResolveChunk - 1) / kResolveChunk;
      if (!kFill) ndesc[x] = total;
      if (k) mine = atomicAdd(&s_cnt, k);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) {
      if (!kFill) atomicAdd(&acc[kAccChunks], static_cast<unsigned long long>(s_cnt));
      else s_base = atomicAdd(&acc[kAccDesc], static_cast<unsigned long long>(s_cnt));
    }
    __syncthreads();
    if (kFill)
      for (int j = 0; j < k; ++j)
        if (static_cast<int64_t>(s_base + mine + j) < rcap) rchunks[s_base + mine + j] = make_int2(static_cast<int>(x), j);
    __syncthreads();
  }
}

// Resolves every descriptor of every heavy anchor into a stream record:
// begin, length | flags, owner of the streamed list.  One block per chunk of
// kResolveChunk descriptors; no LDS, so many blocks hide the two dependent
// loads (descriptor id, vertex record) per descriptor.
template <bool kCover>
__global__ __launch_bounds__(kThreads) void resolve_kernel(
    const int32_t* lc, const VMeta* meta, const int64_t* task_off, const int64_t* task_begin,
    const int32_t* task_len, const int32_t* task_owner, const int2* rchunks, int64_t rcap,
    const unsigned long long* acc, const int64_t* so, int64_t scap, int64_t* sbeg, int32_t* slen, int32_t* soth) {
  const int64_t nchunks = min(static_cast<int64_t>(acc[kAccChunks]), rcap);
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int2 ch = rchunks[c];
    const int32_t x = ch.x;
    const VMeta mx = meta[x];
    const int hf = mx.sfe - mx.hfb;
    const int64_t toff = task_off[x];
    const Desc Dx = desc_of(mx, kCover, static_cast<int>(task_off[x + 1] - toff));
    const int d_end = min(Dx.total(), (ch.y + 1) * kResolveChunk);
    const int64_t base = so[x];
    for (int d = ch.y * kResolveChunk + threadIdx.x; d < d_end; d += blockDim.x) {
      int64_t beg = 0;
      int32_t len = 0, oth = x;
      int k = d;
      if (k < Dx.nB) {  // down class: Up(w); its members in P(x) are in Hfwd(x), so above x
        const int32_t w = lc[mx.begin + mx.sfe + k];
        const VMeta mw = meta[w];
        beg = mw.begin;
        len = mw.up;
        oth = w;
      } else if ((k -= Dx.nB) < Dx.nCu) {  // forward cover edge, up class
        const int32_t v = lc[mx.begin + mx.hfb + k];
        const VMeta mv = meta[v];
        oth = v;
        if (mv.up > 0 && mv.up <= mx.up) {
          beg = mv.begin;
          len = mv.up | kFlagUp;
        }
      } else if ((k -= Dx.nCu) < Dx.nCs) {  // forward cover edge, same class
        const int32_t v = lc[mx.begin + mx.hfb + k];
        const VMeta mv = meta[v];
        oth = v;
        const int a = hf - k - 1, b = mv.sfe - mv.hfb;
        if (a > 0 && b > 0 && b < a) {
          beg = mv.begin + mv.hfb;
          len = b;
        }
      } else if ((k -= Dx.nCs) < Dx.nD) {  // backward cover edge, up class
        const int32_t u = lc[mx.begin + mx.up + k];
        const VMeta mu = meta[u];
        oth = u;
        if (mu.up > 0 && mu.up < mx.up) {
          beg = mu.begin;
          len = mu.up | kFlagUp;
        }
      } else {  // emitted same-class task: Hfwd(u) above x
        const int64_t q = toff + (k - Dx.nD);
        beg = task_begin[q];
        len = task_len[q];
        oth = task_owner[q];
      }
      const int64_t pos = base + d;
      if (pos < scap) {
        sbeg[pos] = beg;
        slen[pos] = len;
        soth[pos] = oth;
      }
    }
  }
}

// Work items: the streams of anchor x are split into at most
// ceil(E / kElemChunk) ranges of about equal element count E / nit (cut at
// stream starts).  kFill = false counts items per bin; kFill = true writes
// int4 {x, first stream (lo, hi), stream count | kItemBitmap}.
template <bool kFill>
__global__ __launch_bounds__(kThreads) void items_kernel(const int32_t* lc, const VMeta* meta, int64_t n,
                                                         const int32_t* ndesc, const int64_t* so, const int64_t* epre,
                                                         int64_t scap, int4* items, unsigned long long* acc) {
  __shared__ int s_cnt[kBins];
  __shared__ unsigned long long s_base[kBins];
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < kBins) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t x = x0 + threadIdx.x;
    int k = 0, b = 0, mine = 0;
    bool bm = false;
    int64_t s0 = 0, s1 = 0, e0 = 0, E = 0;
    if (x < n && ndesc[x] > 0) {
      s0 = min(so[x], scap);
      s1 = min(so[x + 1], scap);
      e0 = epre[s0];
      E = epre[s1] - e0;
      if (E > 0) {
        const VMeta m = meta[x];
        int32_t lo;
        int64_t R;
        probe_window(lc, m, lo, R);
        b = choose_bin(R, probe_size(m), E, &bm);
        int64_t want = (E + kElemChunk - 1) / kElemChunk;
        want = max(want, (s1 - s0 + kItemMaxStreams - 1) / kItemMaxStreams);
        k = static_cast<int>(min(want, s1 - s0));
        mine = atomicAdd(&s_cnt[b], k);
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
      int64_t prev = s0;
      for (int j = 0; j < k; ++j) {
        // first stream starting at or after e0 + (j+1) E / k
        const int64_t cut = e0 + (E * (j + 1)) / k;
        const int64_t nxt = j + 1 == k ? s1 : lower_bound_dev(epre, prev, s1, cut);
        items[base + j] = make_int4(static_cast<int>(x), static_cast<int>(prev & 0xFFFFFFFF),
                                    static_cast<int>(prev >> 32),
                                    static_cast<int>(nxt - prev) | (bm ? kItemBitmap : 0));
        prev = nxt;
      }
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

// Probe set P(x) = Up(x) ∪ Hfwd(x) of the block's current anchor.
struct ProbeSet {
  const uint32_t* tab;
  int32_t lo;      // bitmap: id of bit 0
  uint32_t R;      // bitmap: window length; bit R is kept clear
  int cap, shift;  // hash: slot count (power of two) and hslot shift
  const int32_t* up_row;
  const int32_t* hf_row;
  int up_len, hf_len;
};

// 1 if t is in the probe set, else 0.  t may be any value (the tail of a
// chunk past the stream end is probed and masked afterwards).
template <int MODE>
__device__ __forceinline__ uint32_t probe(const ProbeSet& ps, int32_t t, bool up_side) {
  if (MODE == kBitmap) {
    const uint32_t d = min(static_cast<uint32_t>(t) - static_cast<uint32_t>(ps.lo), ps.R);
    return (ps.tab[d >> 5] >> (d & 31)) & 1u;
  } else if (MODE == kHash) {
    uint32_t h = hslot(t, ps.shift);
    int32_t k;
    while ((k = static_cast<int32_t>(ps.tab[h])) != t && k != -1) h = (h + 1) & (ps.cap - 1);
    return k == t ? 1u : 0u;
  }
  return (up_side ? gsearch(ps.up_row, ps.up_len, t) : gsearch(ps.hf_row, ps.hf_len, t)) ? 1u : 0u;
}

// Streams are cut into chunks of kChunk consecutive elements that never
// cross a stream end; a lane takes one chunk at a time (kChunk independent
// loads in flight, one 64-bit address).  The column buffers carry kColPad
// readable entries past nnz, so the tail of a stream's last chunk is loaded
// unconditionally and masked.
constexpr int kChunk = 8;
constexpr int kWinIters = 8;  // chunk rounds of the block per window
static_assert(kChunk <= kColPad, "chunk tail must stay inside the padded columns");

template <int MODE, bool kPV>
__device__ __forceinline__ uint32_t chunk_hits(const int32_t* p, int len, const ProbeSet& ps, bool up_side,
                                               int32_t x, int32_t oth, int64_t* pv) {
  int32_t v[kChunk];
#pragma unroll
  for (int q = 0; q < kChunk; ++q) v[q] = p[q];
  const uint32_t lenmask = len >= kChunk ? ((1u << kChunk) - 1u) : ((1u << len) - 1u);
  uint32_t hits = 0;
  if (MODE == kHash) {
    // all first probes in flight together; collision chains (rare at load
    // factor <= 1/2) are walked afterwards, one slot per round for all
    uint32_t h[kChunk];
    uint32_t pend = 0;
#pragma unroll
    for (int q = 0; q < kChunk; ++q) h[q] = hslot(v[q], ps.shift);
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      const int32_t k = static_cast<int32_t>(ps.tab[h[q]]);
      hits |= static_cast<uint32_t>(k == v[q]) << q;
      pend |= static_cast<uint32_t>(k != v[q] && k != -1) << q;
    }
    pend &= lenmask;
    while (pend) {
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const uint32_t pb = (pend >> q) & 1u;
        h[q] = (h[q] + pb) & static_cast<uint32_t>(ps.cap - 1);
        const int32_t k = static_cast<int32_t>(ps.tab[h[q]]);
        hits |= (pb & static_cast<uint32_t>(k == v[q])) << q;
        pend &= ~(static_cast<uint32_t>(k == v[q] || k == -1) << q);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < kChunk; ++q) hits |= probe<MODE>(ps, v[q], up_side) << q;
  }
  hits &= lenmask;
  if (kPV && hits) {
#pragma unroll
    for (int q = 0; q < kChunk; ++q)
      if ((hits >> q) & 1u) add_pv(pv, x, oth, v[q]);
  }
  return static_cast<uint32_t>(__popc(hits));
}

// All chunks of one batch of streams.  The chunk space [0, C) is walked in
// windows of THREADS * kWinIters chunks; a window is split into tiles of 64
// chunks, one per wave and round, and for each tile the block first records
// the number of streams that start before it (s_tb) and a 64-bit mask of the
// streams that start inside it (s_M).  Lane i of a wave then finds the
// stream of its chunk as s_tb + popcount(mask bits <= i) - 1, with no search.
template <int MODE, int THREADS, bool kPV>
__device__ __forceinline__ uint32_t run_chunks(int C, int nslots, const int2* s_cl, const int64_t* s_beg,
                                               const int32_t* s_oth, const uint8_t* s_up, uint64_t* s_M,
                                               int32_t* s_tb, const int32_t* lc, const ProbeSet& ps, int32_t x,
                                               int64_t* pv) {
  constexpr int kWin = THREADS * kWinIters;
  constexpr int kTiles = kWin / kWave;
  static_assert(THREADS % kWave == 0, "block must be whole waves");
  const int tid = threadIdx.x;
  const uint32_t ln = static_cast<uint32_t>(lane());
  uint32_t cnt = 0;
  for (int w0 = 0; w0 < C; w0 += kWin) {
    for (int t = tid; t < kTiles; t += THREADS) {
      const int ct = w0 + t * kWave;
      if (ct < C) {
        int lo = 0, hi = nslots;  // first stream starting at or after ct
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_cl[mid].x < ct) lo = mid + 1;
          else hi = mid;
        }
        uint64_t M = 0;
        for (int j = lo; j < nslots; ++j) {
          const int f = s_cl[j].x;
          if (f >= ct + kWave) break;
          M |= 1ull << (f - ct);
        }
        s_tb[t] = lo;
        s_M[t] = M;
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int i = 0; i < kWinIters; ++i) {
      const int rel = i * THREADS + tid;
      const int c = w0 + rel;
      if (c < C) {
        const int t = rel >> 6;
        const uint64_t M = s_M[t];
        const int below = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
            static_cast<uint32_t>(M >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(M), 0u)));
        const int j = s_tb[t] + below + static_cast<int>((M >> ln) & 1ull) - 1;
        const int2 cl = s_cl[j];
        const int k = c - cl.x;
        const int32_t* p = lc + s_beg[j] + static_cast<int64_t>(k) * kChunk;
        cnt += chunk_hits<MODE, kPV>(p, cl.y - k * kChunk, ps, MODE == kSearch && s_up[j] != 0, x,
                                     kPV ? s_oth[j] : 0, pv);
      }
    }
    __syncthreads();
  }
  return cnt;
}

// One block per work item (anchor x, range of resolved streams).  WORDS is
// the LDS table size in 32-bit words (0: search the sorted rows); the item
// says whether the anchor's table is a bitmap or a hash table.  Stream records are
// loaded D at a time (R per thread), the non-empty ones are compacted into
// LDS with their first chunk, and run_chunks streams them.
template <int WORDS, int THREADS, int D, bool kPV>
__global__ __launch_bounds__(THREADS) void heavy_kernel(const int32_t* lc, const VMeta* meta, int bin,
                                                        const int4* items, const int64_t* sbeg,
                                                        const int32_t* slen, const int32_t* soth,
                                                        unsigned long long* acc, int64_t* pv) {
  constexpr int R = D / THREADS;  // records loaded per thread
  static_assert(R * THREADS == D, "D must be a multiple of THREADS");
  constexpr int kTiles = THREADS * kWinIters / kWave;
  __shared__ uint32_t tab[WORDS > 0 ? WORDS : 1];
  __shared__ int64_t s_beg[D];
  __shared__ int2 s_cl[D + 1];  // (first chunk, length) of each non-empty stream
  __shared__ int32_t s_oth[kPV ? D : 1];
  __shared__ uint8_t s_up[WORDS == 0 ? D : 1];
  __shared__ uint64_t s_M[kTiles];
  __shared__ int32_t s_tb[kTiles];
  __shared__ int64_t sh[THREADS / kWave + 1];
  __shared__ int32_t shi[THREADS / kWave + 1];
  __shared__ unsigned long long s_item;

  const unsigned long long first = acc[kAccBinOff + bin];
  const unsigned long long count = acc[kAccBinCount + bin];
  const int tid = threadIdx.x;
  int64_t cnt = 0, elems = 0, builds = 0;
  int32_t cur_x = -1;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(&acc[kAccBinNext + bin], 1ull);
    __syncthreads();
    const unsigned long long it = s_item;
    __syncthreads();
    if (it >= count) break;
    const int4 item = items[first + it];
    const int32_t x = item.x;
    const int64_t sa = static_cast<int64_t>(static_cast<uint32_t>(item.y)) | (static_cast<int64_t>(item.z) << 32);
    const int64_t sb = sa + (item.w & (kItemBitmap - 1));
    const VMeta mx = meta[x];
    const int P = mx.up + (mx.sfe - mx.hfb);
    ProbeSet ps;
    ps.tab = tab;
    ps.lo = 0;
    ps.R = 0;
    ps.cap = 64;
    ps.shift = 26;
    ps.up_row = lc + mx.begin;
    ps.up_len = mx.up;
    ps.hf_row = lc + mx.begin + mx.hfb;
    ps.hf_len = mx.sfe - mx.hfb;
    int mode = kSearch;
    if (WORDS > 0) {
      int64_t R64;
      probe_window(lc, mx, ps.lo, R64);
      ps.R = static_cast<uint32_t>(R64);
      mode = (item.w & kItemBitmap) ? kBitmap : kHash;
      ps.cap = WORDS;
      ps.shift = 32 - __builtin_ctz(WORDS);
      if (x != cur_x) {
        if (mode == kBitmap) {
          const int words = static_cast<int>(bitmap_words(R64));
          for (int i = tid; i < words; i += THREADS) tab[i] = 0u;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const int32_t key = i < mx.up ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            const uint32_t d = static_cast<uint32_t>(key - ps.lo);
            atomicOr(&tab[d >> 5], 1u << (d & 31));
          }
        } else {
          for (int i = tid; i < ps.cap; i += THREADS) tab[i] = 0xFFFFFFFFu;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const int32_t key = i < mx.up ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            uint32_t h = hslot(key, ps.shift);
            while (atomicCAS(&tab[h], 0xFFFFFFFFu, static_cast<uint32_t>(key)) != 0xFFFFFFFFu)
              h = (h + 1) & (ps.cap - 1);
          }
        }
        __syncthreads();
        cur_x = x;
        builds += tid == 0 ? P : 0;
      }
    }
    for (int64_t bs = sa; bs < sb; bs += D) {
      const int nd = static_cast<int>(min(static_cast<int64_t>(D), sb - bs));
      int64_t lbeg[R];
      int32_t llen[R], loth[R];
      bool lup[R];
      int nne = 0, nch = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int dl = tid * R + r;
        lbeg[r] = 0;
        llen[r] = 0;
        loth[r] = x;
        lup[r] = false;
        if (dl < nd) {
          const int64_t k = bs + dl;
          const int32_t lf = slen[k];
          lbeg[r] = sbeg[k];
          llen[r] = lf & kLenMask;
          lup[r] = (lf & kFlagUp) != 0;
          if (kPV) loth[r] = soth[k];
        }
        if (llen[r] > 0) {
          ++nne;
          nch += (llen[r] + kChunk - 1) / kChunk;
          elems += llen[r];
        }
      }
      int32_t nslots, C;
      int slot = block_excl_scan(nne, shi, &nslots);
      int cb = block_excl_scan(nch, shi, &C);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (llen[r] <= 0) continue;
        s_cl[slot] = make_int2(cb, llen[r]);
        s_beg[slot] = lbeg[r];
        if (kPV) s_oth[slot] = loth[r];
        if (WORDS == 0) s_up[slot] = lup[r] ? 1 : 0;
        cb += (llen[r] + kChunk - 1) / kChunk;
        ++slot;
      }
      if (tid == 0) s_cl[nslots] = make_int2(C, 0);
      __syncthreads();
      if (WORDS == 0) {
        cnt += run_chunks<kSearch, THREADS, kPV>(C, nslots, s_cl, s_beg, s_oth, s_up, s_M, s_tb, lc, ps, x, pv);
      } else if (mode == kBitmap) {
        cnt += run_chunks<kBitmap, THREADS, kPV>(C, nslots, s_cl, s_beg, s_oth, s_up, s_M, s_tb, lc, ps, x, pv);
      } else {
        cnt += run_chunks<kHash, THREADS, kPV>(C, nslots, s_cl, s_beg, s_oth, s_up, s_M, s_tb, lc, ps, x, pv);
      }
    }
  }
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccHeavyElems, elems, sh);
  block_acc(acc, kAccBinElems + bin, elems, sh);
  block_acc(acc, kAccBuild, builds, sh);
}

__global__ void finish_kernel(const unsigned long long* acc, const int64_t* h_off, int64_t n, const int64_t* so,
                              int64_t* triangles, int64_t* h_count, int64_t* stats) {
  *triangles = static_cast<int64_t>(acc[kAccT]);
  if (h_count) *h_count = h_off[n];
  stats[2] = h_off[n];
  stats[4] = static_cast<int64_t>(acc[kAccElems] + acc[kAccHeavyElems]);
  stats[5] = static_cast<int64_t>(acc[kAccLight]);
  stats[6] = static_cast<int64_t>(acc[kAccItems]);
  stats[7] = so[n];
  stats[8] = static_cast<int64_t>(acc[kAccHeavyElems]);
  stats[9] = static_cast<int64_t>(acc[kAccBuild]);
  stats[10] = static_cast<int64_t>(acc[kAccElems]);
  for (int b = 0; b < kBins; ++b) {
    stats[11 + b] = static_cast<int64_t>(acc[kAccBinElems + b]);
    stats[11 + kBins + b] = static_cast<int64_t>(acc[kAccBinCount + b]);
  }
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

template <int WORDS, int THREADS, int D, bool kPV>
int launch_heavy(const CountArgs& a, CountWs& w, int bin, int blocks_per_cu, hipStream_t s) {
  heavy_kernel<WORDS, THREADS, D, kPV><<<static_cast<unsigned>(num_cus() * blocks_per_cu), THREADS, 0, s>>>(
      a.cols, a.meta, bin, w.items, w.sbeg, w.slen, w.soth, w.acc, a.per_vertex_out);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

template <bool kCover, bool kPV>
int launch_all(const CountArgs& a, CountWs& w, hipStream_t s) {
  const tc_csr* g = a.g;
  const int64_t n = g->n;
  const unsigned gedge = static_cast<unsigned>(num_cus() * 16);
  const unsigned gv = grid_for(n, kThreads, 16384);
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
  prof_stage("resolve");
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.acc) + kAccChunks, 0, 1, s));
  desc_plan_kernel<false><<<gv, kThreads, 0, s>>>(a.meta, n, w.task_off, kCover, a.light_max, w.ndesc, w.rchunks,
                                                  w.rcap, w.acc);
  desc_plan_kernel<true><<<gv, kThreads, 0, s>>>(a.meta, n, w.task_off, kCover, a.light_max, w.ndesc, w.rchunks,
                                                 w.rcap, w.acc);
  {
    Carver sc2(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.ndesc, w.so, n, sc2, s));
  }
  resolve_kernel<kCover><<<static_cast<unsigned>(num_cus() * 16), kThreads, 0, s>>>(
      a.cols, a.meta, w.task_off, w.task_begin, w.task_len, w.task_owner, w.rchunks, w.rcap, w.acc, w.so, w.scap,
      w.sbeg, w.slen, w.soth);
  TC_HIP(hipGetLastError());
  // element prefix over the streams actually written
  int64_t nstreams = 0;
  TC_HIP(hipMemcpyAsync(&nstreams, w.so + n, sizeof nstreams, hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  // a symmetric simple graph has at most 2 nnz descriptors (deg + |Hfwd| +
  // emitted tasks per anchor); more means an unvalidated asymmetric input
  if (nstreams > w.scap)
    return fail(TC_ERR_NOT_SYMMETRIC, "tc_count: %lld intersection descriptors exceed the bound 2 nnz of a "
                "symmetric graph (validate the input with TC_VALIDATE)", (long long)nstreams);
  const int64_t sc_n = nstreams;
  {
    Carver sc3(w.scratch);
    TC_TRY(scan_exclusive_masked(w.slen, kLenMask, w.epre, sc_n, sc3, s));
  }
  items_kernel<false><<<gv, kThreads, 0, s>>>(a.cols, a.meta, n, w.ndesc, w.so, w.epre, sc_n, w.items, w.acc);
  bin_offsets_kernel<<<1, 1, 0, s>>>(w.acc);
  items_kernel<true><<<gv, kThreads, 0, s>>>(a.cols, a.meta, n, w.ndesc, w.so, w.epre, sc_n, w.items, w.acc);
  TC_HIP(hipGetLastError());
  prof_stage("heavy");
  // the bins are independent: run them side by side
  Fork* f = fork_for_device();
  if (!f) return TC_ERR_HIP;
  TC_TRY(fork_begin(f, s));
  TC_TRY((launch_heavy<kBinWords2, 1024, 1024, kPV>(a, w, 2, 1, s)));
  TC_TRY((launch_heavy<kBinWords1, 512, 1024, kPV>(a, w, 1, 3, f->aux[0])));
  TC_TRY((launch_heavy<kBinWords0, 64, 256, kPV>(a, w, 0, 24, f->aux[1])));
  TC_TRY((launch_heavy<0, 512, 1024, kPV>(a, w, 3, 4, f->aux[2])));
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
  w.ndesc = c.take<int32_t>(n + 1);
  w.so = c.take<int64_t>(n + 2);
  // descriptors of a simple graph: at most deg + |Hfwd| + emitted tasks per
  // anchor, i.e. <= 2 nnz in total; records beyond the capacity are dropped
  w.scap = 2 * nnz + 2;
  w.rcap = n + w.scap / kResolveChunk + 8;
  w.rchunks = c.take<int2>(w.rcap);
  w.sbeg = c.take<int64_t>(w.scap);
  w.slen = c.take<int32_t>(w.scap);
  w.soth = c.take<int32_t>(w.scap);
  w.epre = c.take<int64_t>(w.scap + 1);
  w.items = c.take<int4>(w.scap + 8);
  w.acc = c.take<unsigned long long>(kAccSlots);
  w.stats = c.take<int64_t>(24);
  w.scratch = c.take<char>(scan_ws_bytes(w.scap + 1) + (n + 1) * sizeof(int32_t) + 256);
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
  TC_TRY(fill_i64(w.stats, 0, 24, s));
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
  finish_kernel<<<1, 1, 0, s>>>(w.acc, w.h_off, n, w.so, triangles, h_count, w.stats);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
