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
// w in Down(x), count the t in Up(w) that lie in Hfwd(x); each (u, v, w)
// with u < v is met once, at x = u, t = v.  This is the same set of (edge,
// apex) pairs, enumerated per apex the way the paper's distributed variant
// enumerates the apexes a processor owns; it streams the short up-lists of
// the apexes instead of the long down-lists of hub pairs.
//
// Every intersection is a task: stream one sorted list S and test each
// element for membership in the probe set P(x) = Up(x) ∪ Hfwd(x) of an
// anchor x.  Ownership rules pick the cheaper side per task:
//   up     anchor = u if |Up(v)| <= |Up(u)| else v; stream Up(other)
//   same   a = |Hfwd(u) ∩ (v,inf)|, b = |Hfwd(v)|; if b < a anchor u streams
//          Hfwd(v), else anchor v streams Hfwd(u) ∩ (v,inf)
//   down   anchor x streams Up(w)
// A streamed list lies on one level, so the members of P(x) it can meet are
// in one segment: Up(x) for the up class, Hfwd(x) for the others.
//
// Every vertex x owns the descriptors [down | forward cover edges | backward
// cover edges]: deg(x) - sfe (when Hfwd(x) is not empty), |Hfwd(x)|, and
// its same-level neighbours below x.  One pass over all descriptors applies
// the ownership rules from x's side.  Light anchors (short probe set, few
// down-neighbours) merge their tasks at once.  Heavy anchors emit stream
// records, compacted per block, and the block cuts its records into work
// items of about kElemChunk elements of one anchor, tagged with the on-chip
// table the anchor needs (2 KB .. 128 KB of the 160 KB LDS: a bitmap over the
// probe set's id window, or a hash table) or row search beyond that.  The
// streaming kernel builds the table once per item and hands each lane chunks
// of 8 elements of one stream.  Per-lane counts are reduced wave -> block ->
// one 64-bit atomic; the count runs without a host synchronisation.
//
// The comparator (plain direction-oriented edge iterator) runs through the
// same kernels with up = 0, Hfwd = forward list N+(x), no down class.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kDnLight = 32;  // default: light anchors have at most this many down-neighbours
constexpr int kLightMax = 32; // and a probe set of at most this many ids (the register capacity
                              // of light_kernel, so the tuned bound never exceeds it)
constexpr int kBins = 4;

// Bins of heavy anchors by the LDS table they need: 2 KB, 32 KB, 128 KB, or
// none (bin 3: search the sorted rows).  The probe set P(x) lies in the id
// window [min P, max P] of R ids.  It is held as a bitmap of R + 1 bits (bit
// R stays clear and absorbs every id outside the window) when clearing that
// bitmap costs little next to the anchor's work (at most four words per
// member plus 64, or 16 words per descriptor), else as a hash table filling
// the bin's whole table (at most half full).
constexpr int kBinWords0 = 512, kBinWords1 = 8192, kBinWords2 = 32768;

__host__ __device__ constexpr int bin_words(int b) {
  return b == 0 ? kBinWords0 : (b == 1 ? kBinWords1 : (b == 2 ? kBinWords2 : 0));
}

__device__ __forceinline__ int64_t bitmap_words(int64_t R) { return (R + 32) >> 5; }

// Two-level table of a probe set too large for an LDS bitmap or hash table:
// in LDS one bit per block of 32 ids of the window (set when the block holds
// a member) and, per 32 such bits, the number of set bits before them; in
// global memory the 32-bit member word of every non-empty block, in block
// order.  Words of LDS it needs for a window of R ids:
__device__ __forceinline__ int64_t twolevel_words(int64_t R) { return 2 * (((R >> 5) + 32) >> 5); }

enum TableKind { kKindHash = 0, kKindBitmap = 1, kKindTwoLevel = 2 };

// Bin of an anchor whose bitmap (two parts) takes `need` words, with joint
// window R, probe-set size P, D descriptors and deg row entries; *kind
// tells the table kind.  A two-level table's block bits
// are also kept in global memory at the anchor's row positions (so an item
// copies them instead of inserting |P| ids), hence they must fit in deg
// words.
__device__ __forceinline__ int choose_bin(int64_t need, int64_t R, int P, int64_t D, int64_t deg, int* kind,
                                          const CountParams& prm) {
  // the smallest-table bin streams an item with one wave: only anchors with
  // few tasks go there
  const int b0 = (prm.bin0_max_desc >= 0 && D > prm.bin0_max_desc) ? 1 : 0;
  if (need <= prm.bm_member * static_cast<int64_t>(P) + 64 || need <= prm.bm_desc * D) {
    for (int b = b0; b < 3; ++b)
      if (need <= bin_words(b)) {
        *kind = kKindBitmap;
        return b;
      }
  }
  const int64_t tw = twolevel_words(R);
  const bool tl_fits = tw <= kBinWords2 && tw / 2 <= deg;
  *kind = kKindHash;
  for (int b = b0; b < 3; ++b)
    if (2 * static_cast<int64_t>(P) <= bin_words(b)) {
      // a sparse set of the largest hash bin: most probes miss, and a
      // two-level table rejects them with one LDS read
      if (b == 2 && tl_fits && prm.tl_sparsity > 0 && R >= static_cast<int64_t>(prm.tl_sparsity) * P)
        *kind = kKindTwoLevel;
      return b;
    }
  if (tl_fits) {
    *kind = kKindTwoLevel;
    return 2;
  }
  return 3;
}

enum Acc {
  kAccT = 0, kAccElems = 1, kAccBuild = 3, kAccRecs = 4, kAccItems = 5, kAccHeavyElems = 6,
  kAccH = 7, kAccBinCount = 8, kAccBinOff = 12, kAccBinCur = 16, kAccBinNext = 20, kAccBinElems = 24,
  kAccTwoLevelElems = 28
};
constexpr int kAccSlots = 29;
constexpr int kElemChunkLog = 19;  // default: 2^19 elements per work item (target)
// stream record flag (in the length word): probe the anchor's Up list
constexpr int32_t kFlagUp = 1 << 29;
constexpr int32_t kLenMask = kFlagUp - 1;
// stream slot in LDS (s_cl.y): length | kClUp when the stream probes Up(x)
constexpr int32_t kClUp = 1 << 30;
// work item word: stream count | bin << 28 | kItemBitmap | kItemTwoLevel
constexpr int32_t kItemCountMask = (1 << 28) - 1;
constexpr int32_t kItemBitmap = 1 << 30;
constexpr int32_t kItemTwoLevel = static_cast<int32_t>(0x80000000u);
// per-vertex plan byte: kViHeavy | two-level << 3 | bitmap << 2 | bin
constexpr uint8_t kViHeavy = 0x80;
constexpr uint8_t kViTwoLevel = 0x08;
constexpr uint8_t kViBitmap = 0x04;

__device__ __forceinline__ void add_pv(int64_t* pv, int32_t a, int32_t b, int32_t c) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[a]), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[b]), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long*>(&pv[c]), 1ull);
}

// What the counting kernels do with each triangle they find:
//   kOutNone  count only;
//   kOutPV    also add one to each of its three vertices (per-vertex counts);
//   kOutRec   also record every work unit's count (ucnt: heavy items by their
//             index in the item array, then light tasks by their index);
//   kOutEmit  write it at its work unit's offset (uoff) as three caller ids,
//             ascending (the second pass of triangle finding).
enum OutKind { kOutNone = 0, kOutPV = 1, kOutRec = 2, kOutEmit = 3 };

struct Out {
  int64_t* pv;
  int32_t* ucnt;
  const int64_t* uoff;
  int32_t* tri;          // [3 * cap]
  int64_t cap;
  const int32_t* order;  // layout id -> caller id (null: the same)
};

__host__ __device__ constexpr bool needs_oth(int k) { return k == kOutPV || k == kOutEmit; }

// a and b are caller ids already (mapped once per task or stream), c is a
// layout id.
__device__ __forceinline__ void write_tri(const Out& o, int64_t at, int32_t a, int32_t b, int32_t c) {
  if (at >= o.cap) return;
  if (o.order) c = o.order[c];
  int32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
  o.tri[3 * at] = a;
  o.tri[3 * at + 1] = b;
  o.tri[3 * at + 2] = c;
}

__device__ __forceinline__ int32_t caller_id(const Out& o, int32_t v) { return o.order ? o.order[v] : v; }

// One triangle {x, oth, w} found by a thread that writes sequentially (for
// kOutEmit x and oth are caller ids, w a layout id).
template <int kOut>
__device__ __forceinline__ void on_hit(const Out& o, int32_t x, int32_t oth, int32_t w, int64_t& at) {
  if (kOut == kOutPV) add_pv(o.pv, x, oth, w);
  else if (kOut == kOutEmit) write_tri(o, at++, x, oth, w);
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
__device__ __forceinline__ bool is_heavy(const VMeta& m, bool cover, const CountParams& prm) {
  if (probe_size(m) > prm.light_max) return true;
  return cover && (m.sfe - m.hfb) > 0 && (m.deg - m.sfe) > prm.dn_light;
}

__device__ __forceinline__ void block_acc(unsigned long long* acc, int slot, int64_t v, int64_t* sh) {
  int64_t s = block_sum(v, sh);
  if (threadIdx.x == 0 && s) atomicAdd(&acc[slot], static_cast<unsigned long long>(s));
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

// A bitmap table is two bitmaps, one over the id window of Up(x) and one
// over that of Hfwd(x), each with its always-clear bit R (a part with no
// member is one word): a streamed list meets only one of the two segments
// (it lies on one level), and each part's window is usually far narrower
// than the window of both, which spans the gap between the two levels.
struct SplitWindow {
  int32_t lo_up, lo_hf;
  int64_t R_up, R_hf;
};

__device__ __forceinline__ SplitWindow split_window(const int32_t* lc, const VMeta& m) {
  SplitWindow w{0, 0, 0, 0};
  const int hf = m.sfe - m.hfb;
  if (m.up > 0) {
    w.lo_up = lc[m.begin];
    w.R_up = static_cast<int64_t>(lc[m.begin + m.up - 1]) - w.lo_up + 1;
  }
  if (hf > 0) {
    w.lo_hf = lc[m.begin + m.hfb];
    w.R_hf = static_cast<int64_t>(lc[m.begin + m.sfe - 1]) - w.lo_hf + 1;
  }
  return w;
}

// Words of the two bitmaps.
__device__ __forceinline__ int64_t split_words(const SplitWindow& w) {
  return bitmap_words(w.R_up) + bitmap_words(w.R_hf);
}

// The window of the whole probe set (for two-level tables), from its parts.
__device__ __forceinline__ void joint_window(const SplitWindow& w, int32_t& lo, int64_t& R) {
  int64_t mn = 0x7FFFFFFFFFFFFFFFll, mx = -1;
  if (w.R_up > 0) {
    mn = w.lo_up;
    mx = w.lo_up + w.R_up - 1;
  }
  if (w.R_hf > 0) {
    mn = min(mn, static_cast<int64_t>(w.lo_hf));
    mx = max(mx, w.lo_hf + w.R_hf - 1);
  }
  lo = mx >= 0 ? static_cast<int32_t>(mn) : 0x7FFFFFFF;
  R = mx >= 0 ? mx - mn + 1 : 0;
}


// The fields of a vertex record that the resolution reads of a neighbour
// (begin, up, hfb, sfe) in one 16-byte word, so that the random read of a
// neighbour's record is one request instead of two:
//   x = begin bits 0..31, y = begin bits 32..39 | up << 8, z = hfb, w = sfe.
// A record whose begin needs more than 40 bits or whose up is 2^24 - 1 or
// more gets y = kPmFull: the reader then takes the full record.
constexpr uint32_t kPmFull = 0xFFFFFFFFu;

__device__ __forceinline__ uint4 pack_record(const VMeta& m) {
  const uint64_t b = static_cast<uint64_t>(m.begin);
  if ((b >> 40) != 0 || m.up >= 0xFFFFFF) return make_uint4(0u, kPmFull, 0u, 0u);
  return make_uint4(static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32) | (static_cast<uint32_t>(m.up) << 8),
                    static_cast<uint32_t>(m.hfb), static_cast<uint32_t>(m.sfe));
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // loaded whole, in one instruction

// Record of vertex v for the resolution from its packed word q = pm[v]
// (deg is not filled in).
__device__ __forceinline__ VMeta unpack_record(u32x4 q, const VMeta* meta, int32_t v) {
  VMeta m;
  m.begin = static_cast<int64_t>(q.x | (static_cast<uint64_t>(q.y & 0xFFu) << 32));
  m.up = static_cast<int32_t>(q.y >> 8);
  m.hfb = static_cast<int32_t>(q.z);
  m.sfe = static_cast<int32_t>(q.w);
  m.deg = 0;
  if (q.y == kPmFull) m = meta[v];
  return m;
}

// ------------------------------------------------------------ planning
// One thread per vertex: descriptor count, |Hfwd| (for |H|), and for heavy
// anchors the table bin.
template <bool kCover>
__global__ __launch_bounds__(kThreads) void plan_kernel(const int32_t* lc, const VMeta* meta, int64_t n,
                                                        int32_t* ndesc, uint8_t* vinfo, uint4* pm,
                                                        unsigned long long* acc, CountParams prm) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  int64_t h = 0;
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = x0 + threadIdx.x;
    if (x >= n) continue;
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb;
    const int nB = (kCover && hf > 0) ? m.deg - m.sfe : 0;
    const int nU = (kCover && prm.up_anchor_min >= 0 && m.up > prm.up_anchor_min) ? m.up : 0;
    const int D = nB + hf + (m.hfb - m.up) + nU;
    h += hf;
    uint8_t vi = 0;
    if (D > 0 && is_heavy(m, kCover, prm)) {
      const SplitWindow sw = split_window(lc, m);
      int32_t lo;
      int64_t R;
      joint_window(sw, lo, R);
      int kind = kKindHash;
      const int b = choose_bin(split_words(sw), R, probe_size(m), D, m.deg, &kind, prm);
      vi = static_cast<uint8_t>(kViHeavy | (kind == kKindBitmap ? kViBitmap : 0) |
                                (kind == kKindTwoLevel ? kViTwoLevel : 0) | b);
    }
    ndesc[x] = D;
    vinfo[x] = vi;
    pm[x] = pack_record(m);
  }
  block_acc(acc, kAccH, h, sh);
}

// ------------------------------------------------------------ resolution
// One thread per descriptor, chunks of kResChunk descriptors per block.  A
// descriptor yields at most two tasks with its vertex x as anchor (slot 0:
// up or down class, slot 1: same class).  Tasks of heavy anchors become
// stream records (from the front of the record arrays), tasks of light
// anchors go to the light list (from the back), merged by light_kernel.
constexpr int kResThreads = 256;
constexpr int kResPer = 2;  // descriptors per thread, resolved in lockstep
constexpr int kSampStride = 32;  // one column sample per 128-byte line
constexpr int kResChunk = kResThreads * kResPer;
constexpr int kResRecs = 2 * kResChunk;
constexpr int kResSpan = 2 * kResChunk;  // vertex offsets staged in LDS

struct Task {
  int64_t beg;  // stream begin in the columns
  int32_t len;  // stream length (0: no task) | kFlagUp
  int32_t oth;  // vertex whose list is streamed
};

enum DescKind { kDown = 0, kFwd = 1, kBwd = 2, kNone = 3, kUpD = 4 };

// Tasks of kResPer descriptors (vertex x[j], index k[j] in its descriptor
// space) with x[j] as the anchor of every returned task.  The steps run in
// lockstep over the descriptors so that their dependent loads (neighbour
// id, its record, the search of x in Hfwd(u)) are in flight together.
// A vertex's descriptors are [down | fwd | bwd | upd]: one per vertex of
// Down(x) (when Hfwd(x) is not empty), of Hfwd(x), of the same-level
// neighbours below x, and (cover count, |Up(x)| > upa) of Up(x).
template <bool kCover>
__device__ __forceinline__ void describe_all(const int32_t* lc, const int32_t* samp, const VMeta* meta,
                                             const uint4* pm, const int32_t* x, const VMeta* mx, const int* kin,
                                             int upa, Task* ta, Task* tb) {
  int kind[kResPer], k[kResPer];
  int32_t nb[kResPer];
  int64_t pos[kResPer];
  // positions first, without branches, so that the column loads of all
  // descriptors are in flight together (an idle slot reads column 0)
#pragma unroll
  for (int j = 0; j < kResPer; ++j) {
    ta[j] = Task{0, 0, 0};
    tb[j] = Task{0, 0, 0};
    const int hf = mx[j].sfe - mx[j].hfb;
    const int nB = (kCover && hf > 0) ? mx[j].deg - mx[j].sfe : 0;
    const int nS = mx[j].hfb - mx[j].up;
    const int kk = kin[j];
    const bool dn = kk < nB, fw = !dn && kk - nB < hf;
    const bool bw = !dn && !fw && (!kCover || kk - nB - hf < nS);
    kind[j] = kk < 0 ? kNone : (dn ? kDown : (fw ? kFwd : (bw ? kBwd : kUpD)));
    k[j] = dn ? kk : (fw ? kk - nB : (bw ? kk - nB - hf : kk - nB - hf - nS));
    const int32_t seg = dn ? mx[j].sfe : (fw ? mx[j].hfb : (bw ? mx[j].up : 0));
    pos[j] = kk < 0 ? 0 : mx[j].begin + seg + k[j];
  }
#pragma unroll
  for (int j = 0; j < kResPer; ++j) nb[j] = lc[pos[j]];
  // the neighbours' packed records, all loads issued before any is used
  u32x4 q[kResPer];
#pragma unroll
  for (int j = 0; j < kResPer; ++j) q[j] = *reinterpret_cast<const u32x4*>(pm + (kind[j] != kNone ? nb[j] : 0));
  VMeta mo[kResPer];
#pragma unroll
  for (int j = 0; j < kResPer; ++j)
    if (kind[j] != kNone) mo[j] = unpack_record(q[j], meta, nb[j]);
  // Backward same class, cover edge (u, x) with u < x: the rule compares
  // a = |Hfwd(u) ∩ (x, inf)| with b = |Hfwd(x)|.  The entry b + 1 places
  // before the end of Hfwd(u) decides it with one load: above x, a > b and
  // the forward descriptor of u takes the pair; equal to x, a = b; below,
  // x lies among the last b entries, and only they are searched for it.
  int64_t lo[kResPer], hi[kResPer], pp[kResPer];
  bool srch[kResPer], prb[kResPer];
#pragma unroll
  for (int j = 0; j < kResPer; ++j) {
    srch[j] = prb[j] = false;
    lo[j] = hi[j] = pp[j] = 0;
    const int b = mx[j].sfe - mx[j].hfb, lu = mo[j].sfe - mo[j].hfb;
    if (kind[j] == kBwd && b > 0 && lu > 0) {
      srch[j] = true;
      lo[j] = mo[j].begin + mo[j].hfb;
      hi[j] = mo[j].begin + mo[j].sfe;
      prb[j] = b + 1 < lu;
      pp[j] = prb[j] ? hi[j] - b - 1 : 0;
    }
  }
  {
    int32_t pv[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) pv[j] = lc[pp[j]];  // an idle slot reads column 0
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      if (!prb[j]) continue;
      if (pv[j] > x[j]) srch[j] = false;
      else if (pv[j] == x[j]) lo[j] = hi[j] = pp[j];
      else lo[j] = pp[j] + 1;
    }
  }
  // First over the column samples (every kSampStride-th column, a compact
  // array): the first sampled block start >= x narrows the range to one
  // block, so the search touches about two cache lines instead of one per
  // halving of a long list.
  {
    int64_t blo[kResPer], bhi[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      blo[j] = (lo[j] + kSampStride - 1) / kSampStride;  // samples inside [lo, hi)
      bhi[j] = srch[j] ? (hi[j] - 1) / kSampStride + 1 : blo[j];
      if (bhi[j] < blo[j]) bhi[j] = blo[j];
    }
    const int64_t b0[kResPer] = {blo[0], blo[1]};
    static_assert(kResPer == 2, "the sample search is written for two descriptors");
    for (;;) {  // first sample index in [blo, bhi) whose value is >= x
      bool any = false;
      int32_t v[kResPer];
      int64_t mid[kResPer];
#pragma unroll
      for (int j = 0; j < kResPer; ++j) {
        mid[j] = blo[j] + ((bhi[j] - blo[j]) >> 1);
        v[j] = blo[j] < bhi[j] ? samp[mid[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < kResPer; ++j) {
        if (!(blo[j] < bhi[j])) continue;
        if (v[j] < x[j]) blo[j] = mid[j] + 1;
        else bhi[j] = mid[j];
        any |= blo[j] < bhi[j];
      }
      if (!any) break;
    }
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      if (!srch[j]) continue;
      // samples b0 .. blo-1 are < x, so entries up to (blo-1) * stride are < x;
      // the sample at blo (if inside the range) is >= x
      if (blo[j] > b0[j]) lo[j] = (blo[j] - 1) * kSampStride + 1;
      const int64_t cap = blo[j] * kSampStride;
      if (cap < hi[j]) hi[j] = cap;
    }
  }
  for (;;) {
    bool any = false;
    int32_t v[kResPer];
    int64_t mid[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      mid[j] = lo[j] + ((hi[j] - lo[j]) >> 1);
      v[j] = (srch[j] && lo[j] < hi[j]) ? lc[mid[j]] : 0;
    }
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      if (!(srch[j] && lo[j] < hi[j])) continue;
      if (v[j] < x[j]) lo[j] = mid[j] + 1;
      else hi[j] = mid[j];
      any |= lo[j] < hi[j];
    }
    if (!any) break;
  }
#pragma unroll
  for (int j = 0; j < kResPer; ++j) {
    const VMeta& m = mx[j];
    const VMeta& o = mo[j];
    const int hf = m.sfe - m.hfb;
    if (kind[j] == kDown) {  // stream Up(w), unless w anchors the pair (see kUpD)
      if (o.up > 0 && !(upa >= 0 && o.up > upa && o.up > hf)) ta[j] = Task{o.begin, o.up, nb[j]};
    } else if (kind[j] == kUpD) {
      // u = nb in Up(x), x one level below u: when Up(x) (longer than upa)
      // is also longer than Hfwd(u), x anchors the down-class pair (u, x)
      // and streams Hfwd(u) against the Up part of its table; every cover
      // edge (u, v) with v in Up(x) closes a triangle
      const int hu = o.sfe - o.hfb;
      if (kCover && hu > 0 && m.up > hu) ta[j] = Task{o.begin + o.hfb, hu | kFlagUp, nb[j]};
    } else if (kind[j] == kFwd) {  // forward cover edge (x, v)
      if (kCover && o.up > 0 && o.up <= m.up) ta[j] = Task{o.begin, o.up | kFlagUp, nb[j]};
      const int a = hf - k[j] - 1, b = o.sfe - o.hfb;
      if (a > 0 && b > 0 && b < a) tb[j] = Task{o.begin + o.hfb, b, nb[j]};
    } else if (kind[j] == kBwd) {  // backward cover edge (u, x), u < x
      if (kCover && o.up > 0 && o.up < m.up) ta[j] = Task{o.begin, o.up | kFlagUp, nb[j]};
      if (srch[j]) {
        const int a = static_cast<int>(o.begin + o.sfe - lo[j]) - 1;  // lo = position of x
        if (a > 0 && hf >= a) tb[j] = Task{lo[j] + 1, a, nb[j]};
      }
    }
  }
}

// The tables of the two-level anchors (plan byte kViTwoLevel), at anchor x's
// row positions [begin, begin + deg):
//   words[begin + r]        the bits of its probe-set members in the r-th
//                           non-empty block of 32 ids of its window (the
//                           blocks number at most |P| <= deg(x));
//   l1[begin + i], i < nw   block bits (bit j of word i: block 32 i + j holds
//                           a member), copied into LDS by every item of x
//                           (nw <= deg(x) by the bin rule).
// One wave per anchor; the anchors are found 64 vertices at a time.
__global__ void twolevel_words_kernel(const int32_t* lc, const VMeta* meta, const uint8_t* vinfo, int64_t n,
                                      uint32_t* words, uint32_t* l1) {
  const int64_t wid = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwv = (static_cast<int64_t>(gridDim.x) * blockDim.x) / kWave;
  const int ln = lane();
  for (int64_t x0 = wid * kWave; x0 < n; x0 += nwv * kWave) {
    const int64_t xl = x0 + ln;
    uint64_t mask = __ballot(xl < n && (vinfo[xl] & kViTwoLevel));
    while (mask) {
      const int j = __ffsll(static_cast<unsigned long long>(mask)) - 1;
      mask &= mask - 1;
      const VMeta m = meta[x0 + j];
      int32_t lo;
      int64_t R;
      probe_window(lc, m, lo, R);
      const int P = probe_size(m);
      const int nw = static_cast<int>(twolevel_words(R) >> 1);
      uint32_t* wx = words + m.begin;
      uint32_t* lx = l1 + m.begin;
      for (int i = ln; i < P; i += kWave) wx[i] = 0u;
      for (int i = ln; i < nw; i += kWave) lx[i] = 0u;
      __threadfence();
      int carry = 0;       // non-empty blocks before this round
      int32_t prevb = -1;  // block of the last member of the previous round
      for (int base = 0; base < P; base += kWave) {
        const int i = base + ln;
        int32_t b = -1;
        uint32_t d = 0;
        if (i < P) {
          const int32_t key = i < m.up ? lc[m.begin + i] : lc[m.begin + m.hfb + (i - m.up)];
          d = static_cast<uint32_t>(key - lo);
          b = static_cast<int32_t>(d >> 5);
        }
        int32_t pb = __shfl_up(b, 1, kWave);
        if (ln == 0) pb = prevb;
        const int start = (i < P && b != pb) ? 1 : 0;
        const int incl = wave_incl_scan(start);
        if (i < P) {
          atomicOr(&wx[carry + incl - 1], 1u << (d & 31));
          if (start) atomicOr(&lx[b >> 5], 1u << (b & 31));
        }
        carry += __shfl(incl, kWave - 1, kWave);
        prevb = __shfl(b, kWave - 1, kWave);  // a later round exists only if all 64 lanes were members
      }
    }
  }
}

// Column samples for the searches of the resolution: samp[b] = lc[b * kSampStride].
__global__ void sample_kernel(const int32_t* lc, int64_t nnz, int32_t* samp) {
  const int64_t nb = (nnz + kSampStride - 1) / kSampStride;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x)
    samp[b] = lc[b * kSampStride];
}

// First vertex of every chunk of kResChunk descriptors: chunk c starts at
// descriptor c * kResChunk, owned by the vertex x with so[x] <= it < so[x+1].
// cx0[nchunks] = n - 1 closes the last chunk.
__global__ void chunk_start_kernel(const int64_t* so, int64_t n, int32_t* cx0) {
  const int64_t total = so[n];
  const int64_t nch = (total + kResChunk - 1) / kResChunk;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c0 = (so[x] + kResChunk - 1) / kResChunk, c1 = (so[x + 1] + kResChunk - 1) / kResChunk;
    for (int64_t c = c0; c < c1; ++c) cx0[c] = static_cast<int32_t>(x);
    if (x == n - 1) cx0[nch] = static_cast<int32_t>(n - 1);
  }
}

// Chunk c owns the record region [2 d0, 2 d1) of its descriptors [d0, d1):
// records of heavy anchors from the front, tasks of light anchors from the
// back, its work items at the same offsets of items_raw; ccnt[c] = (heavy
// records, light tasks, items).  No counter is shared between blocks.
// Thread t takes descriptors d0 + t + j * kResThreads; records are placed in
// descriptor order (j-major).
template <bool kCover>
__global__ __launch_bounds__(kResThreads) void resolve_kernel(
    const int32_t* lc, const int32_t* samp, const VMeta* meta, const uint4* pm, const uint8_t* vinfo,
    const int64_t* so, const int32_t* cx0, int64_t n, int64_t* sbeg, int32_t* slen, int32_t* soth, int32_t* sx,
    int4* items_raw, int4* ccnt, int item_log2, int upa) {
  __shared__ int64_t sh[kResThreads / kWave + 1];
  __shared__ int64_t s_so[kResSpan];
  __shared__ int32_t s_x[kResRecs];
  __shared__ int64_t s_pre[kResRecs];
  __shared__ int32_t s_first[kResRecs + 1];
  const int tid = threadIdx.x;
  const int64_t total = so[n];
  const int64_t nch = (total + kResChunk - 1) / kResChunk;
  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const int64_t d0 = c * kResChunk;
    const int64_t d1 = min(d0 + kResChunk, total);
    const int64_t xa = cx0[c], xz = cx0[c + 1];  // the vertex of d1 - 1 is in [xa, xz]
    const int64_t span = xz - xa + 2;            // so[xa .. xz + 1]
    const bool staged = span <= kResSpan;
    if (staged)
      for (int i = tid; i < span; i += kResThreads) s_so[i] = so[xa + i];
    __syncthreads();
    int32_t xi[kResPer];
    int kk[kResPer];
    bool heavy[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      const int64_t d = d0 + tid + j * kResThreads;
      xi[j] = 0;
      kk[j] = -1;
      heavy[j] = false;
      if (d >= d1) continue;
      int64_t x, xb;
      if (staged) {
        int lo = 0, hi = static_cast<int>(span);  // first index with s_so > d
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_so[mid] <= d) lo = mid + 1;
          else hi = mid;
        }
        x = xa + lo - 1;
        xb = s_so[lo - 1];
      } else {
        x = upper_bound_dev(so, xa, xz + 2, d) - 1;
        xb = so[x];
      }
      xi[j] = static_cast<int32_t>(x);
      kk[j] = static_cast<int>(d - xb);
    }
    VMeta mx[kResPer];
    uint8_t vi[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {  // loads of all slots together (an idle slot reads vertex 0's)
      mx[j] = meta[xi[j]];
      vi[j] = vinfo[xi[j]];
    }
#pragma unroll
    for (int j = 0; j < kResPer; ++j) heavy[j] = kk[j] >= 0 && (vi[j] & kViHeavy) != 0;
    Task ta[kResPer], tb[kResPer];
    describe_all<kCover>(lc, samp, meta, pm, xi, mx, kk, upa, ta, tb);
    // ---- counts: light tasks, heavy records, heavy elements (per j, j-major)
    int64_t nl = 0, nh = 0;
    int64_t he[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      const int64_t cnt = (ta[j].len != 0) + (tb[j].len != 0);
      he[j] = heavy[j] ? static_cast<int64_t>(ta[j].len & kLenMask) + (tb[j].len & kLenMask) : 0;
      nl |= (heavy[j] ? 0 : cnt) << (16 * j);  // kResPer * 16 bits: counts <= 2 per descriptor
      nh |= (heavy[j] ? cnt : 0) << (16 * j);
    }
    int64_t ltot_p, htot_p;
    const int64_t lpre_p = block_excl_scan(nl, sh, &ltot_p);
    const int64_t hpre_p = block_excl_scan(nh, sh, &htot_p);
    int32_t lslot[kResPer], hslot[kResPer];
    int32_t ltot = 0, htot = 0;
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      // slots of descriptor group j start after all groups before it
      lslot[j] = ltot + static_cast<int32_t>((lpre_p >> (16 * j)) & 0xFFFF);
      hslot[j] = htot + static_cast<int32_t>((hpre_p >> (16 * j)) & 0xFFFF);
      ltot += static_cast<int32_t>((ltot_p >> (16 * j)) & 0xFFFF);
      htot += static_cast<int32_t>((htot_p >> (16 * j)) & 0xFFFF);
    }
    int64_t ebase = 0;
    int64_t epre[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      int64_t et;
      epre[j] = ebase + block_excl_scan(he[j], sh, &et);
      ebase += et;
    }
    const int64_t rbase = 2 * d0, rend = 2 * d1;
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      const Task* tt[2] = {&ta[j], &tb[j]};
      if (!heavy[j]) {  // light tasks to the back of the region
        int64_t pos = rend - 1 - lslot[j];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (!tt[q]->len) continue;
          sbeg[pos] = tt[q]->beg;
          slen[pos] = tt[q]->len;
          soth[pos] = tt[q]->oth;
          sx[pos] = xi[j];
          --pos;
        }
      } else {  // heavy records to the front
        int sl = hslot[j];
        int64_t e = epre[j];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (!tt[q]->len) continue;
          sbeg[rbase + sl] = tt[q]->beg;
          slen[rbase + sl] = tt[q]->len;
          soth[rbase + sl] = tt[q]->oth;
          s_x[sl] = xi[j];
          s_pre[sl] = e;
          e += tt[q]->len & kLenMask;
          ++sl;
        }
      }
    }
    if (htot == 0) {  // block-uniform
      if (tid == 0) ccnt[c] = make_int4(0, ltot, 0, 0);
      continue;
    }
    __syncthreads();
    // ---- cut into work items: a new item starts where the anchor changes
    // or the record's element offset enters the next 2^item_log2
    // item starts are numbered in slot order: per descriptor group j (the
    // slots of group j follow all of group j - 1), like the records
    int64_t ns = 0;
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      const int cnt = heavy[j] ? (ta[j].len != 0) + (tb[j].len != 0) : 0;
      int64_t nsj = 0;
      for (int q = hslot[j]; q < hslot[j] + cnt; ++q)
        nsj += (q == 0 || s_x[q] != s_x[q - 1] || (s_pre[q] >> item_log2) != (s_pre[q - 1] >> item_log2));
      ns |= nsj << (16 * j);  // at most 2 per thread, at most kResRecs per group
    }
    int64_t ns_tot;
    const int64_t ns_pre = block_excl_scan(ns, sh, &ns_tot);
    int nitems = 0;
    int itj[kResPer];
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      itj[j] = nitems + static_cast<int>((ns_pre >> (16 * j)) & 0xFFFF);
      nitems += static_cast<int>((ns_tot >> (16 * j)) & 0xFFFF);
    }
#pragma unroll
    for (int j = 0; j < kResPer; ++j) {
      const int cnt = heavy[j] ? (ta[j].len != 0) + (tb[j].len != 0) : 0;
      int it = itj[j];
      for (int q = hslot[j]; q < hslot[j] + cnt; ++q)
        if (q == 0 || s_x[q] != s_x[q - 1] || (s_pre[q] >> item_log2) != (s_pre[q - 1] >> item_log2))
          s_first[it++] = q;
    }
    if (tid == 0) {
      s_first[nitems] = htot;
      ccnt[c] = make_int4(htot, ltot, nitems, 0);
    }
    __syncthreads();
    for (int i = tid; i < nitems; i += kResThreads) {
      const int32_t x = s_x[s_first[i]];
      const uint8_t vi = vinfo[x];
      const int64_t r0 = rbase + s_first[i];
      const int cntr = s_first[i + 1] - s_first[i];
      const int32_t w = cntr | ((vi & 3) << 28) | ((vi & kViBitmap) ? kItemBitmap : 0) |
                        ((vi & kViTwoLevel) ? kItemTwoLevel : 0);
      items_raw[rbase + i] = make_int4(x, static_cast<int>(r0 & 0xFFFFFFFF), static_cast<int>(r0 >> 32), w);
    }
    __syncthreads();
  }
}

// Tasks of light anchors, read from the back of every chunk's region; one
// thread per task, found from the scan lpre of the per-chunk task counts.
// The probe segment (at most kLightMax ids) and a stream of at most
// kLightMax ids are loaded into registers with independent loads and
// compared pairwise; a longer stream (down class) is searched for every
// probe id, all searches advancing together.

template <int kOut>
__global__ __launch_bounds__(kThreads) void light_kernel(const int32_t* lc, const VMeta* meta, const int64_t* so,
                                                         int64_t n, const int64_t* lpre, int64_t nchunk_cap,
                                                         const int64_t* sbeg, const int32_t* slen,
                                                         const int32_t* soth, const int32_t* sx,
                                                         unsigned long long* acc, Out o) {
  __shared__ int64_t sh[kThreads / kWave + 1];
  const int64_t total = so[n];
  const int64_t nl = lpre[nchunk_cap];
  // light tasks follow the heavy items in the unit numbering
  const int64_t ubase = (kOut == kOutRec || kOut == kOutEmit) ? static_cast<int64_t>(acc[kAccItems]) : 0;
  int64_t cnt = 0, elems = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nl; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = upper_bound_dev(lpre, 0, nchunk_cap + 1, i) - 1;
    const int64_t pos = 2 * min((c + 1) * kResChunk, total) - 1 - (i - lpre[c]);
    const int32_t x = sx[pos];
    const int32_t lf = slen[pos];
    const int32_t oth = needs_oth(kOut) ? soth[pos] : 0;
    int64_t at = kOut == kOutEmit ? o.uoff[ubase + i] : 0;
    // the ids a hit reports: caller ids when writing triangles
    const int32_t hx = kOut == kOutEmit ? caller_id(o, x) : x;
    const int32_t ho = kOut == kOutEmit ? caller_id(o, oth) : oth;
    int64_t tc = 0;
    const VMeta mx = meta[x];
    const int len = lf & kLenMask;
    const bool up = (lf & kFlagUp) != 0;
    const int32_t* P = lc + mx.begin + (up ? 0 : mx.hfb);
    const int np = up ? mx.up : mx.sfe - mx.hfb;
    const int32_t* S = lc + sbeg[pos];
    int32_t pr[kLightMax];
#pragma unroll
    for (int q = 0; q < kLightMax; ++q) pr[q] = q < np ? P[q] : -1;
    if (len <= kLightMax) {
      int32_t sv[kLightMax];
#pragma unroll
      for (int q = 0; q < kLightMax; ++q) sv[q] = q < len ? S[q] : -2;
#pragma unroll
      for (int q = 0; q < kLightMax; ++q) {
        int m = 0;
#pragma unroll
        for (int j = 0; j < kLightMax; ++j) m |= sv[q] == pr[j];
        tc += m;
        if (m) on_hit<kOut>(o, hx, ho, sv[q], at);
      }
      elems += len;
    } else {
      // probes in groups of 8: lower bound of each in S by binary lifting
      for (int q0 = 0; q0 < np; q0 += 8) {
        int32_t pv[8];
        int lo[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          pv[j] = q0 + j < np ? P[q0 + j] : 0x7FFFFFFF;
          lo[j] = 0;
        }
        for (int step = 1 << (31 - __clz(len)); step > 0; step >>= 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int probe_at = lo[j] + step - 1;
            const int32_t v = (q0 + j < np && probe_at < len) ? S[probe_at] : 0x7FFFFFFF;
            if (v < pv[j]) lo[j] += step;
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool m = q0 + j < np && lo[j] < len && S[lo[j]] == pv[j];
          tc += m;
          if (m) on_hit<kOut>(o, hx, ho, pv[j], at);
        }
      }
      elems += np;
    }
    cnt += tc;
    if (kOut == kOutRec) o.ucnt[ubase + i] = static_cast<int32_t>(tc);
  }
  if (kOut != kOutEmit) {
    block_acc(acc, kAccT, cnt, sh);
    block_acc(acc, kAccElems, elems, sh);
  }
}

// Items grouped by bin, in chunk order within each block of chunks (so the
// consecutive items of one anchor stay adjacent).  One thread per chunk;
// kFill = false counts per bin, kFill = true scatters.
template <bool kFill>
__global__ __launch_bounds__(kThreads) void bin_split_kernel(const int64_t* so, int64_t n, const int4* ccnt,
                                                             const int4* items_raw, int4* items,
                                                             unsigned long long* acc) {
  __shared__ unsigned long long s_base[kBins];
  __shared__ int64_t sh[kThreads / kWave + 1];
  const int64_t total = so[n];
  const int64_t nch = (total + kResChunk - 1) / kResChunk;
  int64_t recs = 0;
  for (int64_t c0 = blockIdx.x * (int64_t)blockDim.x; c0 < nch; c0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + threadIdx.x;
    int ni = 0;
    int k[kBins] = {0, 0, 0, 0};
    if (c < nch) {
      ni = ccnt[c].z;
      if (!kFill) recs += ccnt[c].x;
      for (int i = 0; i < ni; ++i) k[(items_raw[2 * c * kResChunk + i].w >> 28) & 3] += 1;
    }
    // per-bin exclusive offsets within the block, two bins per 64-bit word
    // (at most 2^17 items per bin and block)
    int64_t t01, t23;
    const int64_t p01 = block_excl_scan(static_cast<int64_t>(k[0]) | (static_cast<int64_t>(k[1]) << 32), sh, &t01);
    const int64_t p23 = block_excl_scan(static_cast<int64_t>(k[2]) | (static_cast<int64_t>(k[3]) << 32), sh, &t23);
    if (threadIdx.x < kBins) {
      const int64_t t = threadIdx.x < 2 ? t01 : t23;
      const unsigned long long kb = static_cast<unsigned long long>((t >> (32 * (threadIdx.x & 1))) & 0xFFFFFFFF);
      if (kb) {
        if (!kFill) atomicAdd(&acc[kAccBinCount + threadIdx.x], kb);
        else s_base[threadIdx.x] = acc[kAccBinOff + threadIdx.x] + atomicAdd(&acc[kAccBinCur + threadIdx.x], kb);
      }
    }
    __syncthreads();
    if (kFill && ni) {
      int64_t pos[kBins] = {static_cast<int64_t>(s_base[0]) + (p01 & 0xFFFFFFFF), static_cast<int64_t>(s_base[1]) + (p01 >> 32),
                            static_cast<int64_t>(s_base[2]) + (p23 & 0xFFFFFFFF), static_cast<int64_t>(s_base[3]) + (p23 >> 32)};
      for (int i = 0; i < ni; ++i) {
        const int4 item = items_raw[2 * c * kResChunk + i];
        const int b = (item.w >> 28) & 3;
        int64_t q;
        if (b == 0) q = pos[0]++;
        else if (b == 1) q = pos[1]++;
        else if (b == 2) q = pos[2]++;
        else q = pos[3]++;
        items[q] = item;
      }
    }
    __syncthreads();
  }
  if (!kFill) block_acc(acc, kAccRecs, recs, sh);
}

__global__ void bin_offsets_kernel(unsigned long long* acc) {
  unsigned long long run = 0;
  for (int b = 0; b < kBins; ++b) {
    acc[kAccBinOff + b] = run;
    run += acc[kAccBinCount + b];
  }
  acc[kAccItems] = run;
}

// ------------------------------------------------------------ streaming
// Multiplicative hash on the top bits of a 32-bit product; the id's bits
// above 24 are folded in first so that the multiply is the full-rate 24-bit
// one (a 32-bit integer multiply issues at a quarter of the rate).  HIP's
// __umul24 returns int: the product is taken as unsigned before the shift,
// so that the slot stays below 2^(32 - shift).
__device__ __forceinline__ uint32_t hslot(int32_t key, int shift) {
  const uint32_t k = static_cast<uint32_t>(key);
  return static_cast<uint32_t>(__umul24(k ^ (k >> 24), 0x9E3779u)) >> shift;
}

// Hash tables (linear probing, at most half full) hold the ids in the low
// 31 bits of a slot; kHashEmpty is no vertex id (ids are below 2^31 - 1).
// Bit 31 of a slot says that a key whose home is this slot was placed
// further on: a probe that finds another key in its home slot with that
// bit clear is a miss at once, and only a flagged home is walked until the
// key or an empty slot.  (Keys are never removed, so a key lies before the
// first empty slot after its home.)
constexpr uint32_t kHashEmpty = 0x7FFFFFFFu;
constexpr uint32_t kHashMoved = 0x80000000u;

enum ProbeMode { kBitmap = 0, kHash = 1, kSearch = 2, kTwoLevel = 3 };

// Probe set P(x) = Up(x) ∪ Hfwd(x) of the block's current anchor.
struct ProbeSet {
  const uint32_t* tab;
  int32_t lo;      // two-level: id of bit 0 of the joint window
  uint32_t R;      // two-level: window length (ids >= R miss)
  int32_t lo_up, lo_hf;  // bitmap: id of bit 0 of the Up and the Hfwd part
  uint32_t R_up, R_hf;   // bitmap: window lengths; bit R of each part is kept clear
  uint32_t off_hf;       // bitmap: first word of the Hfwd part
  int nw;          // two-level: LDS words of block bits (their prefix counts follow)
  const uint32_t* words;  // two-level: the member words of the non-empty blocks
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
    // the part of the stream's segment (uniform over a chunk)
    const uint32_t lo = static_cast<uint32_t>(up_side ? ps.lo_up : ps.lo_hf);
    const uint32_t R = up_side ? ps.R_up : ps.R_hf;
    const uint32_t* tb = up_side ? ps.tab : ps.tab + ps.off_hf;
    const uint32_t d = min(static_cast<uint32_t>(t) - lo, R);
    return (tb[d >> 5] >> (d & 31)) & 1u;
  } else if (MODE == kTwoLevel) {
    const uint32_t d = static_cast<uint32_t>(t) - static_cast<uint32_t>(ps.lo);
    if (d >= ps.R) return 0u;
    const uint32_t b = d >> 5;
    const uint32_t w1 = ps.tab[b >> 5];
    if (!((w1 >> (b & 31)) & 1u)) return 0u;  // an empty block: no member
    const uint32_t r = ps.tab[ps.nw + (b >> 5)] + __popc(w1 & ((1u << (b & 31)) - 1u));
    return (ps.words[r] >> (d & 31)) & 1u;
  } else if (MODE == kHash) {
    uint32_t h = hslot(t, ps.shift);
    const uint32_t w = ps.tab[h];
    if ((w & kHashEmpty) == static_cast<uint32_t>(t)) return 1u;
    if (!(w & kHashMoved)) return 0u;
    for (;;) {
      h = (h + 1) & (ps.cap - 1);
      const uint32_t k = ps.tab[h] & kHashEmpty;
      if (k == static_cast<uint32_t>(t)) return 1u;
      if (k == kHashEmpty) return 0u;
    }
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
constexpr int kClaim = 4;     // work items a block claims at once
// Chunk slots per lane whose loads are in flight together: two where the
// registers allow (the 128 KB bin and row search, whose blocks are limited
// by LDS or run four waves per SIMD), one in the small-table bins compiled
// for six waves per SIMD (a second slot spills there).
template <int WORDS>
constexpr int ahead_of() { return (WORDS == kBinWords2 || WORDS == 0) ? 2 : 1; }
static_assert(kChunk <= kColPad, "chunk tail must stay inside the padded columns");

// Hits of one chunk whose entries v (len of them valid) are loaded.
template <int MODE, int kOut>
// Called by every lane of the wave (a lane with no chunk passes len = 0);
// wq: the wave's queue of kWave ids in LDS (hash tables, counting only).
__device__ __forceinline__ uint32_t chunk_probe(const int32_t (&v)[kChunk], int len, const ProbeSet& ps, bool up_side,
                                                int32_t x, int32_t oth, const Out& o, int64_t ebase, int* s_pos,
                                                int32_t* wq) {
  const uint32_t lenmask = len >= kChunk ? ((1u << kChunk) - 1u) : ((1u << len) - 1u);
  uint32_t hits = 0;
  if (MODE == kHash) {
    // all first probes in flight together; the chains of flagged homes are
    // walked afterwards, one slot per round for all
    uint32_t h[kChunk], w[kChunk];
    uint32_t pend = 0;
#pragma unroll
    for (int q = 0; q < kChunk; ++q) h[q] = hslot(v[q], ps.shift);
    // every home slot's read is issued before any is compared
#pragma unroll
    for (int q = 0; q < kChunk; ++q) w[q] = ps.tab[h[q]];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      const bool eq = (w[q] & kHashEmpty) == static_cast<uint32_t>(v[q]);
      hits |= static_cast<uint32_t>(eq) << q;
      pend |= static_cast<uint32_t>(!eq && (w[q] & kHashMoved) != 0) << q;
    }
    pend &= lenmask;
    if (kOut == kOutNone || kOut == kOutRec) {
      // Counting only: the ids still pending in the whole wave (about 1% of
      // them) go to the wave's queue, kWave at a time, and each lane walks
      // at most one chain from the home slot on, instead of every lane
      // stepping all 8 of its slots until the wave's longest walk ends.
      const int np = __popc(pend);
      const int incl = wave_incl_scan(np);
      const int total = __shfl(incl, kWave - 1, kWave);
      uint32_t walked = 0;
      for (int base = 0; base < total; base += kWave) {  // uniform across the wave
        int pos = incl - np - base;
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          if ((pend >> q) & 1u) {
            if (pos >= 0 && pos < kWave) wq[pos] = v[q];
            ++pos;
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (base + lane() < total) {
          const int32_t t = wq[lane()];
          uint32_t hq = hslot(t, ps.shift);
          for (;;) {
            hq = (hq + 1) & static_cast<uint32_t>(ps.cap - 1);
            const uint32_t k = ps.tab[hq] & kHashEmpty;
            if (k == static_cast<uint32_t>(t)) {
              ++walked;
              break;
            }
            if (k == kHashEmpty) break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the next batch overwrites the queue
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      return static_cast<uint32_t>(__popc(hits & lenmask)) + walked;
    }
    while (pend) {
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const uint32_t pb = (pend >> q) & 1u;
        h[q] = (h[q] + pb) & static_cast<uint32_t>(ps.cap - 1);
        const uint32_t k = ps.tab[h[q]] & kHashEmpty;
        const bool eq = k == static_cast<uint32_t>(v[q]);
        hits |= (pb & static_cast<uint32_t>(eq)) << q;
        pend &= ~(static_cast<uint32_t>(eq || k == kHashEmpty) << q);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < kChunk; ++q) hits |= probe<MODE>(ps, v[q], up_side) << q;
  }
  hits &= lenmask;
  if (kOut == kOutPV && hits) {
#pragma unroll
    for (int q = 0; q < kChunk; ++q)
      if ((hits >> q) & 1u) add_pv(o.pv, x, oth, v[q]);
  }
  if (kOut == kOutEmit) {
    // The item's triangles fill [ebase, ebase + its count) in any order; a
    // wave takes one range per round and its lanes write consecutive parts
    // of it (called by every lane of the wave).
    const int nh = __popc(hits);
    int incl = nh;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int t = __shfl_up(incl, d, kWave);
      if (lane() >= d) incl += t;
    }
    int wbase = 0;
    if (lane() == kWave - 1 && incl > 0) wbase = atomicAdd(s_pos, incl);
    wbase = __shfl(wbase, kWave - 1, kWave);
    int64_t at = ebase + wbase + (incl - nh);
#pragma unroll
    for (int q = 0; q < kChunk; ++q)
      if ((hits >> q) & 1u) write_tri(o, at++, x, oth, v[q]);
  }
  return static_cast<uint32_t>(__popc(hits));
}

template <int MODE, int kOut>
__device__ __forceinline__ uint32_t chunk_hits(const int32_t* p, int len, const ProbeSet& ps, bool up_side,
                                               int32_t x, int32_t oth, const Out& o, int64_t ebase, int* s_pos,
                                               int32_t* wq) {
  int32_t v[kChunk];
#pragma unroll
  for (int q = 0; q < kChunk; ++q) v[q] = p[q];
  return chunk_probe<MODE, kOut>(v, len, ps, up_side, x, oth, o, ebase, s_pos, wq);
}

// All chunks of one batch of streams.  The chunk space [0, C) is walked in
// windows of THREADS * kWinIters chunks; a window is split into tiles of 64
// chunks, one per wave and round, and for each tile the block first records
// the number of streams that start before it (s_tb) and a 64-bit mask of the
// streams that start inside it (s_M).  Lane i of a wave then finds the
// stream of its chunk as s_tb + popcount(mask bits <= i) - 1, with no search.
template <int MODE, int THREADS, int kOut, int kAhead>
__device__ __forceinline__ uint32_t run_chunks(int C, int nslots, const int2* s_cl, const int64_t* s_beg,
                                               const int32_t* s_oth, uint64_t* s_M,
                                               int32_t* s_tb, const int32_t* lc, const ProbeSet& ps, int32_t x,
                                               const Out& o, int64_t ebase, int* s_pos, int32_t* s_q) {
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
    int32_t* wq = s_q + (tid & ~(kWave - 1));  // this wave's queue
    if (kOut != kOutEmit && kAhead == 1) {
      // every lane of a wave with work takes part (a lane past the end
      // probes nothing); a wave with none skips the round
#pragma unroll 2
      for (int i = 0; i < kWinIters; ++i) {
        if (w0 + i * THREADS >= C) break;  // the block's remaining slots are all past the end
        const int rel = i * THREADS + tid;
        const int c = w0 + rel;
        if (__ballot(c < C) == 0) continue;
        const int32_t* p = lc;
        int len = 0;
        int32_t ot = 0;
        bool upside = false;
        if (c < C) {
          const int t = rel >> 6;
          const uint64_t M = s_M[t];
          const int below = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
              static_cast<uint32_t>(M >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(M), 0u)));
          const int j = s_tb[t] + below + static_cast<int>((M >> ln) & 1ull) - 1;
          const int2 cl = s_cl[j];
          const int k = c - cl.x;
          p = lc + s_beg[j] + static_cast<int64_t>(k) * kChunk;
          len = (cl.y & kLenMask) - k * kChunk;
          if (needs_oth(kOut)) ot = s_oth[j];
          upside = (cl.y & kClUp) != 0;
        }
        cnt += chunk_hits<MODE, kOut>(p, len, ps, upside, x, ot, o, ebase, s_pos, wq);
      }
    } else if (kOut != kOutEmit) {
      // kAhead chunk slots per lane at a time: every slot's loads are issued
      // before any is probed (a slot past the end reads entry 0 and probes
      // nothing), so a wave keeps kAhead chunks of memory reads in flight
      for (int i = 0; i < kWinIters; i += kAhead) {
        if (w0 + i * THREADS >= C) break;  // the block's remaining slots are all past the end
        int len[kAhead];
        int64_t e[kAhead];
        int32_t oth[kAhead];
        bool up[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
          const int rel = (i + u) * THREADS + tid;
          const int c = w0 + rel;
          len[u] = 0;
          e[u] = 0;
          oth[u] = 0;
          up[u] = false;
          if (c < C) {
            const int t = rel >> 6;
            const uint64_t M = s_M[t];
            const int below = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                static_cast<uint32_t>(M >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(M), 0u)));
            const int j = s_tb[t] + below + static_cast<int>((M >> ln) & 1ull) - 1;
            const int2 cl = s_cl[j];
            const int k = c - cl.x;
            e[u] = s_beg[j] + static_cast<int64_t>(k) * kChunk;
            len[u] = (cl.y & kLenMask) - k * kChunk;
            if (needs_oth(kOut)) oth[u] = s_oth[j];
            up[u] = (cl.y & kClUp) != 0;
          }
        }
        int32_t v[kAhead][kChunk];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
#pragma unroll
          for (int q = 0; q < kChunk; ++q) v[u][q] = lc[e[u] + q];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
          cnt += chunk_probe<MODE, kOut>(v[u], len[u], ps, up[u], x, oth[u], o, ebase, s_pos, wq);
      }
    } else {
      // writing triangles: the whole wave takes part in every round (the
      // writes are placed by a wave scan); lanes past the end probe nothing
#pragma unroll 2
      for (int i = 0; i < kWinIters; ++i) {
        const int rel = i * THREADS + tid;
        const int c = w0 + rel;
        const int32_t* p = lc;
        int len = 0;
        int32_t ot = 0;
        bool upside = false;
        if (c < C) {
          const int t = rel >> 6;
          const uint64_t M = s_M[t];
          const int below = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
              static_cast<uint32_t>(M >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(M), 0u)));
          const int j = s_tb[t] + below + static_cast<int>((M >> ln) & 1ull) - 1;
          const int2 cl = s_cl[j];
          const int k = c - cl.x;
          p = lc + s_beg[j] + static_cast<int64_t>(k) * kChunk;
          len = (cl.y & kLenMask) - k * kChunk;
          ot = s_oth[j];
          upside = (cl.y & kClUp) != 0;
        }
        cnt += chunk_hits<MODE, kOut>(p, len, ps, upside, x, ot, o, ebase, s_pos, wq);
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
template <int WORDS, int THREADS, int D, int WPE, int kOut, bool kRoundRobin>
__global__ __launch_bounds__(THREADS, WPE) void heavy_kernel(const int32_t* lc, const VMeta* meta, int bin,
                                                        const int4* items, const int64_t* sbeg,
                                                        const int32_t* slen, const int32_t* soth,
                                                        const uint32_t* tl_words, const uint32_t* tl_l1,
                                                        unsigned long long* acc, Out o) {
  constexpr int R = D / THREADS;  // records loaded per thread
  static_assert(R * THREADS == D, "D must be a multiple of THREADS");
  constexpr int kTiles = THREADS * kWinIters / kWave;
  __shared__ uint32_t tab[WORDS > 0 ? WORDS : 1];
  __shared__ int64_t s_beg[D];
  __shared__ int2 s_cl[D + 1];  // (first chunk, length) of each non-empty stream
  __shared__ int32_t s_oth[needs_oth(kOut) ? D : 1];
  __shared__ int s_pos;  // triangles of the current item written so far (kOutEmit)
  __shared__ uint64_t s_M[kTiles];
  __shared__ int32_t s_tb[kTiles];
  __shared__ int32_t s_q[WORDS > 0 ? THREADS : 1];  // per wave: its queue of pending hash probes
  __shared__ int64_t sh[THREADS / kWave + 1];
  __shared__ int32_t shi[THREADS / kWave + 1];
  __shared__ unsigned long long s_item;

  const unsigned long long first = acc[kAccBinOff + bin];
  const unsigned long long count = acc[kAccBinCount + bin];
  const int tid = threadIdx.x;
  int64_t cnt = 0, elems = 0, builds = 0, tl_elems = 0;
  int32_t cur_x = -1;
  // blocks claim kClaim consecutive items at a time (consecutive items of
  // one anchor share the table); the next claim is fetched while the
  // current one is processed.  kRoundRobin: block b takes items b, b + G,
  // b + 2G, ... (G blocks) one at a time, with no counter.
  constexpr unsigned long long kC = kRoundRobin ? 1 : kClaim;
  if (tid == 0)
    s_item = kRoundRobin ? static_cast<unsigned long long>(blockIdx.x)
                         : atomicAdd(&acc[kAccBinNext + bin], static_cast<unsigned long long>(kClaim));
  __syncthreads();
  unsigned long long claim = s_item;
  while (claim < count) {
    unsigned long long next = 0;
    if (tid == 0)
      next = kRoundRobin ? claim + gridDim.x
                         : atomicAdd(&acc[kAccBinNext + bin], static_cast<unsigned long long>(kClaim));
    const unsigned long long claim_end = min(claim + kC, count);
    for (unsigned long long it = claim; it < claim_end; ++it) {
    const int64_t gi = static_cast<int64_t>(first + it);  // unit index of this item
    const int4 item = items[gi];
    const int32_t x = item.x;
    const int64_t sa = static_cast<int64_t>(static_cast<uint32_t>(item.y)) | (static_cast<int64_t>(item.z) << 32);
    const int64_t sb = sa + (item.w & kItemCountMask);
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
    ps.nw = 0;
    ps.words = tl_words + mx.begin;
    int mode = kSearch;
    if (WORDS > 0) {
      const SplitWindow sw = split_window(lc, mx);
      int64_t R64;
      joint_window(sw, ps.lo, R64);
      ps.R = static_cast<uint32_t>(R64);
      ps.lo_up = sw.lo_up;
      ps.lo_hf = sw.lo_hf;
      ps.R_up = static_cast<uint32_t>(sw.R_up);
      ps.R_hf = static_cast<uint32_t>(sw.R_hf);
      ps.off_hf = static_cast<uint32_t>(bitmap_words(sw.R_up));
      mode = (item.w & kItemBitmap) ? kBitmap : ((item.w & kItemTwoLevel) ? kTwoLevel : kHash);
      ps.cap = WORDS;
      ps.shift = 32 - __builtin_ctz(WORDS);
      ps.nw = static_cast<int>(twolevel_words(R64) >> 1);
      if (x != cur_x) {
        if (WORDS == kBinWords2 && mode == kTwoLevel) {
          // the block bits as the planning pass wrote them at the anchor's
          // row positions, then per word the number of set bits before it
          const uint32_t* lx = tl_l1 + mx.begin;
          const int nw = ps.nw;
          constexpr int kPer = WORDS > 0 ? (WORDS / 2 + THREADS - 1) / THREADS : 1;  // words per thread
          uint32_t wv[kPer];
          int mine = 0;
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int i = tid * kPer + j;
            wv[j] = i < nw ? lx[i] : 0u;
            mine += __popc(wv[j]);
          }
          int32_t tot;
          int run = block_excl_scan(mine, shi, &tot);
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int i = tid * kPer + j;
            if (i < nw) {
              tab[i] = wv[j];
              tab[nw + i] = static_cast<uint32_t>(run);
            }
            run += __popc(wv[j]);
          }
        } else if (mode == kBitmap) {
          const int words = static_cast<int>(ps.off_hf + bitmap_words(sw.R_hf));
          for (int i = tid; i < words; i += THREADS) tab[i] = 0u;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const bool upm = i < mx.up;
            const int32_t key = upm ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            const uint32_t d = static_cast<uint32_t>(key - (upm ? ps.lo_up : ps.lo_hf));
            atomicOr(&tab[(upm ? 0u : ps.off_hf) + (d >> 5)], 1u << (d & 31));
          }
        } else {
          for (int i = tid; i < ps.cap; i += THREADS) tab[i] = kHashEmpty;
          __syncthreads();
          for (int i = tid; i < P; i += THREADS) {
            const int32_t key = i < mx.up ? lc[mx.begin + i] : lc[mx.begin + mx.hfb + (i - mx.up)];
            const uint32_t h0 = hslot(key, ps.shift);
            uint32_t h = h0;
            while (atomicCAS(&tab[h], kHashEmpty, static_cast<uint32_t>(key)) != kHashEmpty)
              h = (h + 1) & (ps.cap - 1);
            if (h != h0) atomicOr(&tab[h0], kHashMoved);  // the home is occupied, so it stays a key
          }
        }
        __syncthreads();
        cur_x = x;
        // ids inserted (bitmap, hash) or words copied (two-level)
        builds += tid == 0 ? (mode == kTwoLevel ? ps.nw : P) : 0;
      }
    }
    int64_t ebase = 0;
    int32_t hx = x;  // the anchor as hits report it (a caller id when writing triangles)
    if (kOut == kOutEmit) {
      hx = caller_id(o, x);
      ebase = o.uoff[gi];
      if (tid == 0) s_pos = 0;
      __syncthreads();
    }
    int64_t icnt = 0;
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
          if (needs_oth(kOut)) loth[r] = kOut == kOutEmit ? caller_id(o, soth[k]) : soth[k];
        }
        if (llen[r] > 0) {
          ++nne;
          nch += (llen[r] + kChunk - 1) / kChunk;
          elems += llen[r];
          if (mode == kTwoLevel) tl_elems += llen[r];
        }
      }
      int32_t nslots, C;
      int slot = block_excl_scan(nne, shi, &nslots);
      int cb = block_excl_scan(nch, shi, &C);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (llen[r] <= 0) continue;
        s_cl[slot] = make_int2(cb, llen[r] | (lup[r] ? kClUp : 0));
        s_beg[slot] = lbeg[r];
        if (needs_oth(kOut)) s_oth[slot] = loth[r];
        cb += (llen[r] + kChunk - 1) / kChunk;
        ++slot;
      }
      if (tid == 0) s_cl[nslots] = make_int2(C, 0);
      __syncthreads();
      uint32_t got;
      if (WORDS == 0) {
        got = run_chunks<kSearch, THREADS, kOut, ahead_of<WORDS>()>(C, nslots, s_cl, s_beg, s_oth, s_M, s_tb, lc, ps, hx, o,
                                                 ebase, &s_pos, s_q);
      } else if (mode == kBitmap) {
        got = run_chunks<kBitmap, THREADS, kOut, ahead_of<WORDS>()>(C, nslots, s_cl, s_beg, s_oth, s_M, s_tb, lc, ps, hx, o,
                                                 ebase, &s_pos, s_q);
      } else if (WORDS == kBinWords2 && mode == kTwoLevel) {
        got = run_chunks<kTwoLevel, THREADS, kOut, ahead_of<WORDS>()>(C, nslots, s_cl, s_beg, s_oth, s_M, s_tb, lc, ps, hx, o,
                                                   ebase, &s_pos, s_q);
      } else {
        got = run_chunks<kHash, THREADS, kOut, ahead_of<WORDS>()>(C, nslots, s_cl, s_beg, s_oth, s_M, s_tb, lc, ps, hx, o,
                                               ebase, &s_pos, s_q);
      }
      // the per-item count is kept only where it is recorded
      if (kOut == kOutRec) icnt += got;
      else cnt += got;
    }
    if (kOut == kOutRec) {
      cnt += icnt;
      const int64_t t = block_sum(icnt, sh);
      if (tid == 0) o.ucnt[gi] = static_cast<int32_t>(t);
    }
    }
    __syncthreads();
    if (tid == 0) s_item = next;
    __syncthreads();
    claim = s_item;
  }
  if (kOut == kOutEmit) return;
  block_acc(acc, kAccT, cnt, sh);
  block_acc(acc, kAccHeavyElems, elems, sh);
  block_acc(acc, kAccBinElems + bin, elems, sh);
  block_acc(acc, kAccBuild, builds, sh);
  block_acc(acc, kAccTwoLevelElems, tl_elems, sh);
}


__global__ void finish_kernel(const unsigned long long* acc, const int64_t* so, int64_t n, const int64_t* lpre,
                              int64_t nchunk_cap, int64_t* triangles, int64_t* h_count, int64_t* stats) {
  *triangles = static_cast<int64_t>(acc[kAccT]);
  if (h_count) *h_count = static_cast<int64_t>(acc[kAccH]);
  stats[2] = static_cast<int64_t>(acc[kAccH]);
  stats[4] = static_cast<int64_t>(acc[kAccElems] + acc[kAccHeavyElems]);
  stats[5] = n > 0 ? lpre[nchunk_cap] : 0;
  stats[6] = static_cast<int64_t>(acc[kAccItems]);
  stats[7] = static_cast<int64_t>(acc[kAccRecs]);
  stats[8] = static_cast<int64_t>(acc[kAccHeavyElems]);
  stats[9] = static_cast<int64_t>(acc[kAccBuild]);
  stats[10] = static_cast<int64_t>(acc[kAccElems]);
  for (int b = 0; b < kBins; ++b) {
    stats[11 + b] = static_cast<int64_t>(acc[kAccBinElems + b]);
    stats[11 + kBins + b] = static_cast<int64_t>(acc[kAccBinCount + b]);
  }
  stats[19] = n > 0 ? so[n] : 0;
  stats[20] = static_cast<int64_t>(acc[kAccTwoLevelElems]);
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


// WPE: waves per SIMD the kernel is compiled for (HIP's second launch
// bound), matched to the blocks per CU that the bin's LDS allows.
template <int WORDS, int THREADS, int D, int WPE, int kOut, bool kRoundRobin = false>
int launch_heavy(const CountArgs& a, CountWs& w, const Out& o, int bin, int blocks_per_cu, hipStream_t s) {
  heavy_kernel<WORDS, THREADS, D, WPE, kOut, kRoundRobin><<<static_cast<unsigned>(num_cus() * blocks_per_cu), THREADS, 0, s>>>(
      a.cols, a.meta, bin, w.items, w.sbeg, w.slen, w.soth, w.tl_words, w.tl_l1, w.acc, o);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

// The four bins of heavy items, one after another on the call's stream
// (bins_mode 1) or side by side on forked streams (2).
template <int kOut>
int launch_bins(const CountArgs& a, CountWs& w, const Out& o, hipStream_t s) {
  if (a.prm.bins_mode == 1) {
    TC_TRY((launch_heavy<kBinWords2, 1024, 1024, 4, kOut>(a, w, o, 2, 1, s)));
    TC_TRY((launch_heavy<kBinWords1, 512, 1024, 6, kOut>(a, w, o, 1, 3, s)));
    // bin 0: two-wave blocks taking items round robin, or one-wave blocks
    // claiming them (count_params picks by graph size)
    if (a.prm.bin0_mode == 2) TC_TRY((launch_heavy<kBinWords0, 128, 256, 6, kOut, true>(a, w, o, 0, 12, s)));
    else TC_TRY((launch_heavy<kBinWords0, 64, 256, 6, kOut>(a, w, o, 0, 24, s)));
    return launch_heavy<0, 512, 1024, 4, kOut>(a, w, o, 3, 4, s);
  }
  Fork* f = fork_for_device();
  if (!f) return TC_ERR_HIP;
  TC_TRY(fork_begin(f, s));
  TC_TRY((launch_heavy<kBinWords2, 1024, 1024, 4, kOut>(a, w, o, 2, 1, s)));
  TC_TRY((launch_heavy<kBinWords1, 512, 1024, 6, kOut>(a, w, o, 1, 3, f->aux[0])));
  if (a.prm.bin0_mode == 2) TC_TRY((launch_heavy<kBinWords0, 128, 256, 6, kOut, true>(a, w, o, 0, 12, f->aux[1])));
  else TC_TRY((launch_heavy<kBinWords0, 64, 256, 6, kOut>(a, w, o, 0, 24, f->aux[1])));
  TC_TRY((launch_heavy<0, 512, 1024, 4, kOut>(a, w, o, 3, 4, f->aux[2])));
  return fork_end(f, s);
}

template <int kOut>
int launch_light(const CountArgs& a, CountWs& w, const Out& o, hipStream_t s) {
  // one thread per task; there are at most two tasks per CSR entry
  const int64_t need = (2 * (a.g->nnz + 1) + kThreads - 1) / kThreads;
  const int64_t cap = static_cast<int64_t>(num_cus()) * 16;
  light_kernel<kOut><<<static_cast<unsigned>(need < cap ? need : cap), kThreads, 0, s>>>(
      a.cols, a.meta, w.so, a.g->n, w.lpre, w.nchunk_cap, w.sbeg, w.slen, w.soth, w.sx, w.acc, o);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

template <bool kCover, int kOut>
int launch_all(const CountArgs& a, CountWs& w, const Out& o, hipStream_t s) {
  const int64_t n = a.g->n;
  const unsigned gv = grid_for(n, kThreads, 16384);
  // kernels over the resolve chunks need at most one block (resolve) or one
  // thread (bin split) per chunk; nchunk_cap bounds the chunk count
  const int64_t gmax = static_cast<int64_t>(num_cus()) * 16;
  const unsigned gr = static_cast<unsigned>(w.nchunk_cap < gmax ? w.nchunk_cap : gmax);
  const int64_t gct = (w.nchunk_cap + kThreads - 1) / kThreads;
  const unsigned gc = static_cast<unsigned>(gct < gmax ? gct : gmax);
  plan_kernel<kCover><<<gv, kThreads, 0, s>>>(a.cols, a.meta, n, w.ndesc, w.vinfo, w.pm, w.acc, a.prm);
  TC_HIP(hipGetLastError());
  // a wave scans 64 vertices per round: about two rounds per wave (one
  // block of a graph of 16 K vertices scanned them in 19 us)
  twolevel_words_kernel<<<grid_for(n, kThreads * 2, 4096), kThreads, 0, s>>>(a.cols, a.meta, w.vinfo, n,
                                                                           w.tl_words, w.tl_l1);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.ndesc, w.so, n, sc, s));
  }
  TC_TRY(fill_i32(reinterpret_cast<int32_t*>(w.ccnt), 0, 4 * w.nchunk_cap, s));
  chunk_start_kernel<<<gv, kThreads, 0, s>>>(w.so, n, w.cx0);
  TC_HIP(hipGetLastError());
  prof_stage("resolve");
  sample_kernel<<<grid_for(a.g->nnz / kSampStride + 1, kThreads, 16384), kThreads, 0, s>>>(a.cols, a.g->nnz,
                                                                                           w.samp);
  resolve_kernel<kCover><<<gr, kResThreads, 0, s>>>(a.cols, w.samp, a.meta, w.pm, w.vinfo, w.so, w.cx0, n, w.sbeg,
                                                    w.slen, w.soth, w.sx, w.items_raw, w.ccnt, a.prm.item_log2,
                                                    a.prm.up_anchor_min);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive_strided(reinterpret_cast<const int32_t*>(w.ccnt) + 1, 4, w.lpre, w.nchunk_cap, sc, s));
  }
  bin_split_kernel<false><<<gc, kThreads, 0, s>>>(w.so, n, w.ccnt, w.items_raw, w.items, w.acc);
  bin_offsets_kernel<<<1, 1, 0, s>>>(w.acc);
  bin_split_kernel<true><<<gc, kThreads, 0, s>>>(w.so, n, w.ccnt, w.items_raw, w.items, w.acc);
  TC_HIP(hipGetLastError());
  // after the item split: kOutRec keeps its unit counts where the raw items were
  TC_TRY(launch_light<kOut>(a, w, o, s));
  prof_stage("heavy");
  TC_TRY(launch_bins<kOut>(a, w, o, s));
  prof_stage("finish");
  return TC_OK;
}

// Unit counts and offsets of triangle finding live in the raw-item buffer,
// which is dead once the items are split by bin: rcap int32 counts, then
// rcap + 1 int64 offsets (12 rcap + 8 <= 16 rcap bytes for rcap >= 2).
Out unit_out(CountWs& w) {
  Out o{};
  char* base = reinterpret_cast<char*>(w.items_raw);
  o.ucnt = reinterpret_cast<int32_t*>(base);
  o.uoff = reinterpret_cast<int64_t*>(base + ((4 * w.rcap + 7) & ~int64_t(7)));
  return o;
}

}  // namespace

int count_params(const tc_tuning* t, bool cover, int64_t nnz, CountParams* out) {
  CountParams p;
  p.light_max = kLightMax;
  p.dn_light = kDnLight;
  p.bm_member = 4;
  // cover count: 8 words per task (R-MAT S24 71.3 -> 69.7 ms, S20 3.71 ->
  // 3.63 ms, S22 within 0.5%); the comparator keeps 16
  p.bm_desc = cover ? 8 : 16;
  // work items of 2^14 elements below 2^24 entries, where the heavy work is
  // too small to fill the chip in 2^19-element items (R-MAT S14 0.708 ->
  // 0.682 ms, S16 0.886 -> 0.842, Chung-Lu n = 10^5 0.844 -> 0.834; S18
  // unchanged)
  p.item_log2 = nnz < (int64_t(1) << 24) ? 14 : kElemChunkLog;
  p.tl_sparsity = 64;
  // Bin 0 (tables of 2 KB): on smaller graphs its items are short (about 500
  // elements at R-MAT S20) and two waves per block with half the blocks
  // finish sooner, taking the items round robin (the claim counter's
  // same-address atomics and the spread of finish times over a 4-item claim
  // cost 0.1 ms of 0.42 at S20); on large graphs (2400 elements per item at
  // S24) the items vary more and one wave per block with claims does
  // (round robin loses 2.4 ms there).
  p.bin0_mode = cover && nnz < (int64_t(1) << 27) ? 2 : 1;
  // The table bins one after another or side by side on forked streams:
  // side by side, bin 0's many small blocks can take the CUs before a
  // larger bin's and the stage time varies from call to call; the cover
  // count runs faster and steadier in sequence (R-MAT S20 heavy stage 2.04
  // ms against a median of 2.28 ms side by side, S24 within 1.5%), the
  // comparator, whose work is spread over the small bins, side by side.
  p.bins_mode = cover ? 1 : 2;
  // an anchor with more than 1024 task descriptors skips the smallest-table
  // bin: its items would be streamed by one wave each (R-MAT S22 15.9 ->
  // 14.5 ms, S20 3.89 -> 3.72 ms; S24, 72.0 ms without the limit, 72.4)
  p.bin0_max_desc = 1024;
  // A down-class pair (x, w) may stream the shorter of Up(w) and Hfwd(x)
  // when Up(w) is long (w then holds one task descriptor per vertex of
  // Up(w)).  On for graphs of at least 2^26 entries: with the layout's
  // degree-ordered levels, R-MAT S24 67.8 -> 66.7 ms and S22 14.59 -> 14.31
  // ms at 256; at S20 it gains nothing (3.77 -> 3.76 ms).
  p.up_anchor_min = cover && nnz >= (int64_t(1) << 26) ? 256 : -1;
  // Four degree groups per level from 2^26 entries (R-MAT S24 8% fewer
  // streamed elements, 2 ms faster overall), two below, where the layout's
  // twelve groups cost more than the shorter forward lists gain (S20 3.61
  // -> 3.72 ms).
  p.degree_groups = nnz >= (int64_t(1) << 26) ? 4 : 2;
  if (t) {
    if (t->light_max) p.light_max = t->light_max;
    if (t->dn_light) p.dn_light = t->dn_light;
    if (t->bitmap_member_words) p.bm_member = t->bitmap_member_words;
    if (t->bitmap_desc_words) p.bm_desc = t->bitmap_desc_words;
    if (t->item_log2) p.item_log2 = t->item_log2;
    if (t->bin0_mode) p.bin0_mode = t->bin0_mode;
    if (t->bins_mode) p.bins_mode = t->bins_mode;
    if (t->twolevel_sparsity) p.tl_sparsity = t->twolevel_sparsity;
    if (t->bin0_max_desc) p.bin0_max_desc = t->bin0_max_desc;
    if (t->up_anchor_min) p.up_anchor_min = t->up_anchor_min;
    if (t->degree_groups) p.degree_groups = t->degree_groups;
  }
  if (p.light_max < 1 || p.light_max > kLightMax)
    return fail(TC_ERR_INVALID_ARG, "tuning: light_max must be in 1..%d", kLightMax);
  if (p.dn_light < 1) return fail(TC_ERR_INVALID_ARG, "tuning: dn_light must be >= 1");
  if (p.bm_member < 1 || p.bm_member > 1024 || p.bm_desc < 1 || p.bm_desc > 1024)
    return fail(TC_ERR_INVALID_ARG, "tuning: bitmap word factors must be in 1..1024");
  if (p.item_log2 < 12 || p.item_log2 > 24) return fail(TC_ERR_INVALID_ARG, "tuning: item_log2 must be in 12..24");
  if (p.tl_sparsity < -1) return fail(TC_ERR_INVALID_ARG, "tuning: twolevel_sparsity must be >= 1, or -1");
  if (p.bin0_max_desc < -1) return fail(TC_ERR_INVALID_ARG, "tuning: bin0_max_desc must be >= 1, or -1");
  // w must be a heavy anchor (a probe set above every light bound)
  if (p.degree_groups != 2 && p.degree_groups != 4)
    return fail(TC_ERR_INVALID_ARG, "tuning: degree_groups must be 2 or 4");
  if (p.up_anchor_min != -1 && p.up_anchor_min < kLightMax)
    return fail(TC_ERR_INVALID_ARG, "tuning: up_anchor_min must be >= %d, or -1", kLightMax);
  if (p.bin0_mode < 1 || p.bin0_mode > 2 || p.bins_mode < 1 || p.bins_mode > 2)
    return fail(TC_ERR_INVALID_ARG, "tuning: bin0_mode and bins_mode must be 1 or 2");
  *out = p;
  return TC_OK;
}

CountWs count_reserve(Carver& c, int64_t n, int64_t nnz) {
  CountWs w;
  w.ndesc = c.take<int32_t>(n + 1);
  w.vinfo = c.take<uint8_t>(n + 1);
  w.so = c.take<int64_t>(n + 2);
  // a vertex has at most deg(x) descriptors and a descriptor at most two
  // tasks, so 2 nnz bounds the stream records of heavy anchors (front) plus
  // the tasks of light anchors (back), and the work items, for any input
  w.rcap = 2 * nnz + 2;
  w.sbeg = c.take<int64_t>(w.rcap);
  w.slen = c.take<int32_t>(w.rcap);
  w.soth = c.take<int32_t>(w.rcap);
  w.sx = c.take<int32_t>(w.rcap);
  w.items_raw = c.take<int4>(w.rcap);
  w.items = c.take<int4>(w.rcap);
  // descriptors are at most nnz, so chunks at most nnz / kResChunk + 1
  w.nchunk_cap = nnz / kResChunk + 2;
  w.cx0 = c.take<int32_t>(w.nchunk_cap + 1);
  w.ccnt = c.take<int4>(w.nchunk_cap);
  w.lpre = c.take<int64_t>(w.nchunk_cap + 1);
  w.samp = c.take<int32_t>(nnz / kSampStride + 2);
  w.pm = c.take<uint4>(n + 1);
  w.tl_words = c.take<uint32_t>(nnz + 1);
  w.tl_l1 = c.take<uint32_t>(nnz + 1);
  w.acc = c.take<unsigned long long>(kAccSlots);
  w.stats = c.take<int64_t>(24);
  // scans over vertices, over chunks and over the work units of triangle finding (<= rcap)
  w.scratch = c.take<char>(scan_ws_bytes(std::max(n + w.nchunk_cap + 1, w.rcap)) + 256);
  return w;
}

int forward_meta_run(const tc_csr* g, VMeta* meta, hipStream_t s) {
  if (g->n == 0) return TC_OK;
  forward_meta_kernel<<<grid_for(g->n, kThreads, 16384), kThreads, 0, s>>>(g->row_offsets, g->cols, g->n, meta);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int count_run(const CountArgs& a, CountWs& w, int64_t* triangles, int64_t* h_count, hipStream_t s) {
  const int64_t n = a.g->n;
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.acc), 0, kAccSlots, s));
  TC_TRY(fill_i64(w.stats, 0, 24, s));
  prof_stage("plan");
  if (n > 0) {
    Out o = unit_out(w);
    o.pv = a.per_vertex_out;
    o.order = a.order;
    if (!a.cover) TC_TRY((launch_all<false, kOutNone>(a, w, o, s)));
    else if (a.record_units) TC_TRY((launch_all<true, kOutRec>(a, w, o, s)));
    else if (a.per_vertex) TC_TRY((launch_all<true, kOutPV>(a, w, o, s)));
    else TC_TRY((launch_all<true, kOutNone>(a, w, o, s)));
  }
  finish_kernel<<<1, 1, 0, s>>>(w.acc, w.so, n, w.lpre, w.nchunk_cap, triangles, h_count, w.stats);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int list_run(const CountArgs& a, CountWs& w, int32_t* tri, int64_t cap, int64_t* triangles, int64_t* h_count,
             hipStream_t s) {
  CountArgs ra = a;
  ra.record_units = true;
  ra.per_vertex = false;
  TC_TRY(count_run(ra, w, triangles, h_count, s));
  if (a.g->n == 0 || cap == 0) return TC_OK;
  prof_stage("emit");
  // pass two: every work unit writes its triangles at the scanned offset of
  // its count (the number of units is read back first)
  int64_t host[2] = {0, 0};
  TC_HIP(hipMemcpyAsync(&host[0], w.acc + kAccItems, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipMemcpyAsync(&host[1], w.lpre + w.nchunk_cap, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  const int64_t units = host[0] + host[1];
  if (units < 0 || units > w.rcap) return TC_ERR_HIP;
  Out o = unit_out(w);
  o.tri = tri;
  o.cap = cap;
  o.order = a.order;
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(o.ucnt, const_cast<int64_t*>(o.uoff), units, sc, s));
  }
  TC_TRY(fill_i64(reinterpret_cast<int64_t*>(w.acc + kAccBinNext), 0, kBins, s));
  TC_TRY(launch_light<kOutEmit>(a, w, o, s));
  return launch_bins<kOutEmit>(a, w, o, s);
}

}  // namespace tc
