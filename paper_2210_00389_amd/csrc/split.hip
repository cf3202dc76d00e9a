// split.hip -- level-class layout of the adjacency and the cover-edge list.
//
// Alg. 1 selects the horizontal edges (L(u) = L(v), u < v) and tests every
// common neighbour w of a cover edge against L(w) = L(u).  BFS levels of
// adjacent vertices differ by at most one (the parity argument of Lemma 1),
// so relative to its row a neighbour is in one of three classes -- one level
// up, same level, one level down.
//
// This pass rewrites every row as [Up | Same | Down], each part ascending (a
// stable partition of the sorted row), and records per vertex the class
// bounds and the start of Hfwd(x) = {v in Same(x) : v > x}, the cover edges
// leaving x.  The counting kernels then evaluate the paper's test
// structurally (see count.hip).
//
// Two layouts share the row engine:
//   * identity: same vertex ids, classes from the given int32 levels (any
//     level function; used for the explicit cover-edge list);
//   * relabelled (for counting): vertices renumbered by (virtual level,
//     degree group, id), columns rewritten to the new ids, classes read off
//     the new id ranges.  The method only compares ids inside one
//     (component, level) class, and any total order there gives the same H
//     (as a set), T and per-vertex counts; each level becomes a contiguous
//     id range, which keeps the probe sets of the counting kernels inside a
//     small id window.
//
// Rows of up to kShort entries are handled by one thread each; longer rows of
// up to kMidCap entries by one wave, of up to kBigCap by one block, each held
// in registers between the counting and the scatter; longer rows are cut into
// segments of kSeg entries handled by one wave each (counts, then a per-row
// prefix over its segments, then a stable ballot scatter).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kShort = 32;
constexpr int kSeg = 2048;
constexpr int kRounds = 4;  // 64-entry rounds of a long row loaded at once
// Rows longer than kShort: up to kMidCap entries one wave each, up to
// kBigCap one block of 256 threads each, held in registers; longer rows in
// kSeg-entry segments, one wave each (a count pass that keeps the gathered
// ids, a per-row prefix, a scatter pass).
constexpr int kMidR = 8;                         // registers per lane, wave per row
constexpr int kMidCap = kMidR * 64;              // 512
constexpr int kBigWaves = 4;                     // block of 256 threads per row
constexpr int kBigR = 16;
constexpr int kBigCap = kBigWaves * kBigR * 64;  // 4096
static_assert(kBigCap >= kSeg, "a segmented row has at least one full segment");
enum RowCat { kRowShort = 0, kRowMid = 1, kRowBig = 2, kRowHuge = 3 };

// ---------------------------------------------------------- layouts
// A row is written as [Up | Same | Down], each ascending in the output
// numbering.  In the relabelled numbering every level is itself split in
// G id ranges by vertex degree (deg_group: G = 4 on large graphs, G = 2 on
// the others), each in input id order, so each class region is G ascending
// runs: the layout is a stable partition of the sorted input row into
// NG = 3 G groups, group
//   class * G + degree group   (class 0 up, 1 same, 2 down)
// (the identity layout has G = 1).  Group codes take 4 bits.
constexpr int kMaxDegGroups = 4;
constexpr int kMaxGroups = 3 * kMaxDegGroups;
constexpr int kNoGroup = 15;
constexpr int kCodeBits = 4;
static_assert(kNoGroup >= kMaxGroups && kNoGroup < (1 << kCodeBits), "group codes fit in kCodeBits");

// Degree group of a vertex of degree d among G groups per level: the
// same-level lists point from lower to higher groups, so the vertices of
// largest degree get the shortest forward lists.
template <int G>
__device__ __forceinline__ int deg_group(int64_t d) {
  static_assert(G == 2 || G == 4, "two or four degree groups per level");
  if constexpr (G == 4) return (d > 511) + (d > 2047) + (d > 8191);
  else return d > 2048 ? 1 : 0;
}

// A layout maps output row i to an input row and groups its entries:
//   ctx(i)          per-row context
//   cls(c, w, v)    group of input entry w; v gets the value written out
//   recls(c, v)     the same group, from the output value v
template <int NG>
struct alignas(8) RowCtxT {
  int64_t ib, ie, ob;  // input range, output begin
  int32_t self;        // the row's own id in the output numbering
  int32_t key;         // the row's (virtual) level
  int32_t b[NG - 1];   // relabelled: first id of groups 1 .. NG - 1 (ascending)
};
static_assert(sizeof(RowCtxT<kMaxGroups>) == 80, "row contexts are stored as whole int64 words");

struct IdentityLayout {
  static constexpr int kG = 1;  // one degree group: groups 0 up, 1 same, 2 down
  using Ctx = RowCtxT<3>;
  const int64_t* off;
  const int32_t* L;
  __device__ __forceinline__ Ctx ctx(int64_t i) const {
    Ctx c{};
    c.ib = off[i];
    c.ie = off[i + 1];
    c.ob = c.ib;
    c.self = static_cast<int32_t>(i);
    c.key = L[i];
    return c;
  }
  __device__ __forceinline__ int recls(const Ctx& c, int32_t v) const {
    const int lv = L[v];
    return lv < c.key ? 0 : (lv == c.key ? 1 : 2);
  }
  __device__ __forceinline__ int cls(const Ctx& c, int32_t w, int32_t& v) const {
    v = w;
    return recls(c, w);
  }
};

template <int G>
struct RelabelLayout {
  static constexpr int kG = G;
  static constexpr int NG = 3 * G;
  using Ctx = RowCtxT<NG>;
  const int64_t* off;    // input row offsets
  const int64_t* noff;   // output row offsets
  const int32_t* order;  // new id -> old id
  const int32_t* perm;   // old id -> new id
  const int32_t* L;
  const uint32_t* comp0;
  int32_t d0;
  const int64_t* gstart;  // first new id of each (virtual level, degree group) group: G vl + group
  __device__ __forceinline__ Ctx ctx(int64_t i) const {
    Ctx c{};
    const int32_t x = order[i];
    c.ib = off[x];
    c.ie = off[x + 1];
    c.ob = noff[i];
    c.self = static_cast<int32_t>(i);
    const int vl = L[x] + (((comp0[x >> 5] >> (x & 31)) & 1u) ? 0 : d0);
    c.key = vl;
    // groups of levels vl - 1, vl, vl + 1 (those of level -1 are empty: id 0)
#pragma unroll
    for (int j = 1; j < NG; ++j) {
      const int64_t gi = static_cast<int64_t>(G) * (vl - 1) + j;
      c.b[j - 1] = static_cast<int32_t>(gstart[gi > 0 ? gi : 0]);
    }
    return c;
  }
  // every neighbour lies in the level above, the same or the level below
  __device__ __forceinline__ int recls(const Ctx& c, int32_t v) const {
    int g = 0;
#pragma unroll
    for (int j = 0; j < NG - 1; ++j) g += v >= c.b[j];
    return g;
  }
  __device__ __forceinline__ int cls(const Ctx& c, int32_t w, int32_t& v) const {
    v = perm[w];
    return recls(c, v);
  }
};

template <int G>
__device__ __forceinline__ bool is_same(int g) { return g >= G && g < 2 * G; }

template <int G, class Ctx>
__device__ __forceinline__ VMeta row_meta(const Ctx& c, const int (&cnt)[3 * G], int slt) {
  int up = 0, same = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    up += cnt[g];
    same += cnt[G + g];
  }
  return VMeta{c.ob, up, up + slt, up + same, static_cast<int32_t>(c.ie - c.ib), {c.key, 0}};
}

// Rows of at most kShort entries: one thread; the row and the groups of its
// entries are loaded into registers first (all gathers in flight at once),
// then counted and scattered.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_short_kernel(Lay lay, const int32_t* cols, int64_t n, int32_t* out,
                                                             VMeta* meta, int32_t* nseg, int32_t* rcat) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const Ctx c = lay.ctx(i);
    const int32_t deg = static_cast<int32_t>(c.ie - c.ib);
    if (deg > kShort) {
      const int cat = deg <= kMidCap ? kRowMid : (deg <= kBigCap ? kRowBig : kRowHuge);
      rcat[i] = cat;
      nseg[i] = cat == kRowHuge ? (deg + kSeg - 1) / kSeg : 0;
      continue;
    }
    rcat[i] = kRowShort;
    nseg[i] = 0;
    int32_t wv[kShort];
#pragma unroll
    for (int q = 0; q < kShort; ++q) wv[q] = q < deg ? cols[c.ib + q] : 0;
    int32_t vv[kShort];
    int kc[kShort];
#pragma unroll
    for (int q = 0; q < kShort; ++q) {
      vv[q] = 0;
      kc[q] = q < deg ? lay.cls(c, wv[q], vv[q]) : kNoGroup;
    }
    int cnt[NG] = {};
    int slt = 0;
#pragma unroll
    for (int q = 0; q < kShort; ++q) {
#pragma unroll
      for (int g = 0; g < NG; ++g) cnt[g] += kc[q] == g;
      slt += is_same<G>(kc[q]) & (vv[q] < c.self);
    }
    int pos[NG];
    pos[0] = 0;
#pragma unroll
    for (int g = 1; g < NG; ++g) pos[g] = pos[g - 1] + cnt[g - 1];
#pragma unroll
    for (int q = 0; q < kShort; ++q) {
      if (kc[q] == kNoGroup) continue;
      int at = 0;
#pragma unroll
      for (int g = 0; g < NG; ++g)
        if (kc[q] == g) at = pos[g]++;
      out[c.ob + at] = vv[q];
    }
    meta[i] = row_meta<G>(c, cnt, slt);
  }
}

// Row lists of the two staged categories from their packed scan, as row
// contexts: the kernels that lay these rows out then start with one load
// instead of the chain of dependent loads ctx() makes.
template <class Lay>
__global__ void row_list_kernel(Lay lay, const int32_t* rcat, int64_t n, const int64_t* pre, typename Lay::Ctx* mid_ctx,
                                typename Lay::Ctx* big_ctx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = rcat[i];
    if (c == kRowMid) mid_ctx[pre[i] & 0xFFFFFFFFll] = lay.ctx(i);
    else if (c == kRowBig) big_ctx[pre[i] >> 32] = lay.ctx(i);
  }
}

// A wave's part of a row: up to R * 64 entries from part_begin, held in
// registers (lane l has entries part_begin + u * 64 + l); -1 past the end.
template <int R, class Ctx>
__device__ __forceinline__ void load_part(const int32_t* cols, const Ctx& c, int part_begin, int32_t (&wv)[R]) {
  const int lim = static_cast<int>(c.ie - c.ib) - part_begin;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int j = u * kWave + lane();
    wv[u] = j < lim ? cols[c.ib + part_begin + j] : -1;
  }
}

// Group counts of a wave's part (or of a row), 16 bits per field, four
// fields per word: field f (groups 0 .. NG - 1, then same-below-x) is
// bits 16 (f % 4) of w[f / 4].  Parts add field by field.
template <int NG>
struct CountsT {
  static constexpr int kWords = (NG + 1 + 3) / 4;
  uint64_t w[kWords];
};
constexpr uint64_t kF16 = 0xFFFF;

// A wave-uniform 64-bit value, kept in scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <int NG>
__device__ __forceinline__ void unpack(const CountsT<NG>& k, int (&cnt)[NG], int& slt) {
#pragma unroll
  for (int g = 0; g < NG; ++g) cnt[g] = static_cast<int>((k.w[g >> 2] >> (16 * (g & 3))) & kF16);
  slt = static_cast<int>((k.w[NG >> 2] >> (16 * (NG & 3))) & kF16);
}

// Groups of a part (kCodeBits bits per entry in *kp) and its output ids.
template <class Lay, int R>
__device__ __forceinline__ CountsT<3 * Lay::kG> classify_part(const Lay& lay, const typename Lay::Ctx& c, const int32_t (&wv)[R],
                                                int32_t (&vv)[R], uint64_t* kp, int nr = R) {
  constexpr int G = Lay::kG, NG = 3 * G;
  static_assert(kCodeBits * R <= 64, "group codes are packed in one 64-bit word");
  uint64_t k3 = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    vv[u] = 0;
    if (u >= nr) {  // past the part (uniform): no entries
      k3 |= static_cast<uint64_t>(kNoGroup) << (kCodeBits * u);
      continue;
    }
    const int k = wv[u] >= 0 ? lay.cls(c, wv[u], vv[u]) : kNoGroup;
    k3 |= static_cast<uint64_t>(k) << (kCodeBits * u);
  }
  uint64_t cnt[NG] = {};
  uint64_t slt = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (u >= nr) break;
    const int k = static_cast<int>((k3 >> (kCodeBits * u)) & kNoGroup);
#pragma unroll
    for (int g = 0; g < NG; ++g) cnt[g] += __popcll(__ballot(k == g));
    slt += __popcll(__ballot(is_same<G>(k) & (vv[u] < c.self)));
  }
  *kp = k3;
  CountsT<NG> out{};
#pragma unroll
  for (int g = 0; g < NG; ++g) out.w[g >> 2] |= cnt[g] << (16 * (g & 3));
  out.w[NG >> 2] |= slt << (16 * (NG & 3));
  return out;
}

// Scatter of a part: group g continues at p[g] (absolute output position);
// entries keep their order inside each group.
template <int R, int NG>
__device__ __forceinline__ void write_part(const int32_t (&vv)[R], uint64_t k3, int64_t (&p)[NG],
                                           int32_t* out, int nr = R) {
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (u >= nr) break;
    const int k = static_cast<int>((k3 >> (kCodeBits * u)) & kNoGroup);
    uint64_t m[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) m[g] = __ballot(k == g);
    // each lane picks its group's next slot and its rank among the group's
    // earlier lanes, so the round is one store instruction
    int64_t at = 0;
    uint64_t mine = 0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      at = k == g ? p[g] : at;
      mine = k == g ? m[g] : mine;
      p[g] += __popcll(m[g]);
    }
    if (k != kNoGroup) out[at + __popcll(mine & lt)] = vv[u];
  }
}

// Absolute group starts of a row from its counts, plus the offsets `before`
// (counts of earlier parts of the same row) inside each group.
template <int NG>
__device__ __forceinline__ void group_starts(int64_t base, const int (&tot)[NG], const int (&before)[NG],
                                             int64_t (&p)[NG]) {
  int64_t run = base;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    p[g] = run + before[g];
    run += tot[g];
  }
}

// Rows of up to R * 64 entries, one wave each.  The wave loads the context
// and the columns of its next row before it groups and writes the current
// one, so the memory latencies of two rows overlap.
template <class Lay, int R>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void lay_mid_kernel(Lay lay, const int32_t* cols, const typename Lay::Ctx* rows,
                                                           const int64_t* count, int32_t* out, VMeta* meta) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  static_assert(R * kWave < (1 << 16), "part counts are packed in 16-bit fields");
  const int64_t nrows = *count & 0xFFFFFFFFll;
  const int64_t nw = (int64_t)gridDim.x * (kThreads / kWave);
  // one row per wave: a wave-uniform index lets the row contexts load into
  // scalar registers
  int64_t r = (int64_t)blockIdx.x * (kThreads / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (r >= nrows) return;
  Ctx c = rows[r];
  int32_t wv[R];
  load_part<R>(cols, c, 0, wv);
  for (;;) {
    const int64_t rn = r + nw;
    const bool more = rn < nrows;
    Ctx cn = c;
    if (more) cn = rows[rn];
    int32_t vv[R];
    uint64_t k3;
    const int nr = static_cast<int>((c.ie - c.ib + kWave - 1) / kWave);  // rounds of this row
    const CountsT<NG> pk = classify_part<Lay, R>(lay, c, wv, vv, &k3, nr);
    int32_t wn[R];
    if (more) load_part<R>(cols, cn, 0, wn);
    int cnt[NG], slt;
    unpack(pk, cnt, slt);
    if (lane() == 0) meta[c.self] = row_meta<G>(c, cnt, slt);
    const int zero[NG] = {};
    int64_t p[NG];
    group_starts(c.ob, cnt, zero, p);
    write_part<R>(vv, k3, p, out, nr);
    if (!more) break;
    r = rn;
    c = cn;
#pragma unroll
    for (int u = 0; u < R; ++u) wv[u] = wn[u];
  }
}

// Rows of up to WPR * R * 64 entries, one block of WPR waves each; wave q
// holds entries [q * R * 64, (q + 1) * R * 64) and the waves' group counts
// are combined through LDS.
template <class Lay, int WPR, int R>
__global__ __launch_bounds__(WPR * kWave) __attribute__((amdgpu_waves_per_eu(5))) void lay_block_kernel(Lay lay, const int32_t* cols, const typename Lay::Ctx* rows,
                                                                const int64_t* count, int32_t* out, VMeta* meta) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  constexpr int kPart = R * kWave;
  static_assert(WPR * kPart < (1 << 16), "row counts are packed in 16-bit fields");
  __shared__ uint64_t s_w[WPR][CountsT<NG>::kWords];
  const int wave = threadIdx.x / kWave;
  const int64_t nrows = *count >> 32;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const Ctx c = rows[r];
    int32_t wv[R], vv[R];
    uint64_t k3;
    load_part<R>(cols, c, wave * kPart, wv);
    // rounds of this wave's part (0 past the row's end)
    const int64_t plen = (c.ie - c.ib) - static_cast<int64_t>(wave) * kPart;
    const int nr = plen <= 0 ? 0 : static_cast<int>(plen >= kPart ? R : (plen + kWave - 1) / kWave);
    const CountsT<NG> pk = classify_part<Lay, R>(lay, c, wv, vv, &k3, nr);
    if (lane() == 0) {
#pragma unroll
      for (int i = 0; i < CountsT<NG>::kWords; ++i) s_w[wave][i] = pk.w[i];
    }
    __syncthreads();
    CountsT<NG> before{}, tot{};
    for (int q = 0; q < WPR; ++q) {
#pragma unroll
      for (int i = 0; i < CountsT<NG>::kWords; ++i) {
        const uint64_t x = s_w[q][i];
        if (q < wave) before.w[i] += x;
        tot.w[i] += x;
      }
    }
#pragma unroll
    for (int i = 0; i < CountsT<NG>::kWords; ++i) {  // the same in every lane of the wave
      before.w[i] = uniform64(before.w[i]);
      tot.w[i] = uniform64(tot.w[i]);
    }
    int cnt[NG], slt, bef[NG], bslt;
    unpack(tot, cnt, slt);
    unpack(before, bef, bslt);
    if (threadIdx.x == 0) meta[c.self] = row_meta<G>(c, cnt, slt);
    int64_t p[NG];
    group_starts(c.ob, cnt, bef, p);
    write_part<R>(vv, k3, p, out, nr);
    __syncthreads();  // s_w is rewritten for the next row
  }
}

__global__ void seg_vtx_kernel(const int32_t* nseg, const int64_t* seg_off, int64_t n, int32_t* seg_vtx) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[x];
    const int64_t s0 = seg_off[x];
    for (int i = 0; i < k; ++i) seg_vtx[s0 + i] = static_cast<int32_t>(x);
  }
}

// Per segment of a segmented row: NG + 1 counts (the groups, then
// same-below-x), NG output positions.

// One wave per segment of a long row: group counts of the segment; the
// output ids are kept (stash) for the scatter pass.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_seg_count_kernel(Lay lay, const int32_t* cols, int64_t n,
                                                                 const int64_t* seg_off, const int32_t* seg_vtx,
                                                                 int32_t* seg_cnt, int32_t* stash) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  constexpr int kSegCnt = NG + 1;  // per segment: the group counts, then same-below-x
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t i = seg_vtx[sg];
    const Ctx c = lay.ctx(i);
    const int64_t s = sg - seg_off[i];
    const int64_t b = c.ib + s * kSeg;
    const int64_t e = min(c.ie, b + kSeg);
    int cnt[NG] = {};
    int slt = 0;
    for (int64_t j0 = b; j0 < e; j0 += kRounds * kWave) {
      int32_t wv[kRounds];
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        const int64_t j = j0 + u * kWave + lane();
        wv[u] = j < e ? cols[j] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        int k = kNoGroup;
        int32_t v = 0;
        if (wv[u] >= 0) {
          k = lay.cls(c, wv[u], v);
          stash[j0 + u * kWave + lane()] = v;  // the scatter pass reads the ids back instead of gathering again
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) cnt[g] += __popcll(__ballot(k == g));
        slt += __popcll(__ballot(is_same<G>(k) & (v < c.self)));
      }
    }
    if (lane() < kSegCnt) {
      int x = slt;
#pragma unroll
      for (int g = 0; g < NG; ++g)
        if (lane() == g) x = cnt[g];
      seg_cnt[kSegCnt * sg + lane()] = x;
    }
  }
}

// Per segmented row: the row record, and per segment the absolute output
// position of each of its groups.
template <class Lay>
__global__ void lay_seg_prefix_kernel(Lay lay, int64_t n, const int32_t* nseg, const int64_t* seg_off,
                                      const int32_t* seg_cnt, int64_t* seg_pre, VMeta* meta) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  constexpr int kSegCnt = NG + 1;  // per segment: the group counts, then same-below-x
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[i];
    if (k == 0) continue;
    const int64_t s0 = seg_off[i];
    int tot[NG] = {};
    int slt = 0;
    for (int j = 0; j < k; ++j) {
      const int32_t* sc = seg_cnt + kSegCnt * (s0 + j);
#pragma unroll
      for (int g = 0; g < NG; ++g) tot[g] += sc[g];
      slt += sc[NG];
    }
    const Ctx c = lay.ctx(i);
    meta[i] = row_meta<G>(c, tot, slt);
    int64_t p[NG];
    const int zero[NG] = {};
    group_starts(c.ob, tot, zero, p);
    for (int j = 0; j < k; ++j) {
      const int32_t* sc = seg_cnt + kSegCnt * (s0 + j);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        seg_pre[NG * (s0 + j) + g] = p[g];
        p[g] += sc[g];
      }
    }
  }
}

// One wave per segment: stable scatter of the segment's entries.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_seg_write_kernel(Lay lay, const int32_t* stash, int64_t n,
                                                                 const int64_t* seg_off, const int32_t* seg_vtx,
                                                                 const int64_t* seg_pre, int32_t* out) {
  constexpr int G = Lay::kG, NG = 3 * G;
  using Ctx = typename Lay::Ctx;
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t i = seg_vtx[sg];
    const Ctx c = lay.ctx(i);
    const int64_t s = sg - seg_off[i];
    const int64_t b = c.ib + s * kSeg;
    const int64_t e = min(c.ie, b + kSeg);
    int64_t p[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) p[g] = seg_pre[NG * sg + g];
    for (int64_t j0 = b; j0 < e; j0 += kRounds * kWave) {
      int32_t vv[kRounds];
      uint64_t k3 = 0;
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        const int64_t j = j0 + u * kWave + lane();
        vv[u] = j < e ? stash[j] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRounds; ++u)
        k3 |= static_cast<uint64_t>(vv[u] >= 0 ? lay.recls(c, vv[u]) : kNoGroup) << (kCodeBits * u);
      write_part<kRounds>(vv, k3, p, out);
    }
  }
}

// Blocks for a kernel that needs at most `need` of them, at most `cap`.
inline unsigned capped_grid(int64_t need, int64_t cap) {
  return static_cast<unsigned>(need < 1 ? 1 : (need < cap ? need : cap));
}

template <class Lay>
int layout_run(const Lay& lay, const int32_t* cols, int64_t n, int64_t nnz, SplitWs& w, hipStream_t s) {
  const unsigned gv = grid_for(n, kThreads, 16384);
  // the row classes hold at most nnz / (least row length) rows: a small
  // graph launches only the blocks its mid, block and segment rows can use
  const int64_t wpb = kThreads / kWave;
  const int64_t mid_rows = nnz / (kShort + 1), big_rows = nnz / (kMidCap + 1);
  const int64_t segs = nnz / kSeg + nnz / (kBigCap + 1) + 1;
  const unsigned gmid = capped_grid((mid_rows + wpb - 1) / wpb, static_cast<int64_t>(num_cus()) * 8);
  const unsigned gbig = capped_grid(big_rows, static_cast<int64_t>(num_cus()) * 4);
  const unsigned gw = capped_grid((segs + wpb - 1) / wpb, static_cast<int64_t>(num_cus()) * 8);
  lay_short_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, cols, n, w.scols, w.meta, w.nseg, w.rcat);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive_pair(w.rcat, kRowMid, kRowBig, w.cat_pre, n, sc, s));
  }
  typename Lay::Ctx* mid_ctx = reinterpret_cast<typename Lay::Ctx*>(w.mid_ctx);
  typename Lay::Ctx* big_ctx = reinterpret_cast<typename Lay::Ctx*>(w.big_ctx);
  row_list_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, w.rcat, n, w.cat_pre, mid_ctx, big_ctx);
  lay_mid_kernel<Lay, kMidR><<<gmid, kThreads, 0, s>>>(lay, cols, mid_ctx,
                                                                                      w.cat_pre + n, w.scols, w.meta);
  lay_block_kernel<Lay, kBigWaves, kBigR><<<gbig, kBigWaves * kWave, 0, s>>>(
      lay, cols, big_ctx, w.cat_pre + n, w.scols, w.meta);
  TC_HIP(hipGetLastError());
  Carver sc(w.scratch);
  TC_TRY(scan_exclusive<int32_t>(w.nseg, w.seg_off, n, sc, s));
  seg_vtx_kernel<<<gv, kThreads, 0, s>>>(w.nseg, w.seg_off, n, w.seg_vtx);
  lay_seg_count_kernel<Lay><<<gw, kThreads, 0, s>>>(lay, cols, n, w.seg_off, w.seg_vtx, w.seg_cnt, w.stash);
  lay_seg_prefix_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, n, w.nseg, w.seg_off, w.seg_cnt, w.seg_pre, w.meta);
  lay_seg_write_kernel<Lay><<<gw, kThreads, 0, s>>>(lay, w.stash, n, w.seg_off, w.seg_vtx, w.seg_pre, w.scols);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

// ------------------------------------------------------- relabelling
// Virtual level: L(v) in r0's component, L(v) + d0 elsewhere.
__device__ __forceinline__ int vlevel(const int32_t* L, const uint32_t* comp0, int32_t d0, int64_t v) {
  return L[v] + (((comp0[v >> 5] >> (v & 31)) & 1u) ? 0 : d0);
}

// Relabel group of a vertex: G * virtual level + degree group.
template <int G>
__device__ __forceinline__ int vgroup(const int64_t* off, const int32_t* L, const uint32_t* comp0, int32_t d0,
                                      int64_t v) {
  return G * vlevel(L, comp0, d0, v) + deg_group<G>(off[v + 1] - off[v]);
}

template <int G>
__global__ __launch_bounds__(kThreads) void vl_hist_kernel(const int64_t* off, const int32_t* L,
                                                           const uint32_t* comp0, int32_t d0, int64_t n,
                                                           int32_t ngroups, int32_t* cnt) {
  constexpr int kLds = 1024;
  __shared__ int32_t h[kLds];
  const bool local = ngroups <= kLds;
  if (local)
    for (int i = threadIdx.x; i < ngroups; i += kThreads) h[i] = 0;
  __syncthreads();
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int gr = vgroup<G>(off, L, comp0, d0, v);
    if (local) atomicAdd(&h[gr], 1);
    else atomicAdd(&cnt[gr], 1);
  }
  __syncthreads();
  if (local)
    for (int i = threadIdx.x; i < ngroups; i += kThreads)
      if (h[i]) atomicAdd(&cnt[i], h[i]);
}

template <int G>
__global__ void vl_keys_kernel(const int64_t* off, const int32_t* L, const uint32_t* comp0, int32_t d0, int64_t n,
                               uint64_t* keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = (static_cast<uint64_t>(vgroup<G>(off, L, comp0, d0, v)) << 32) | static_cast<uint64_t>(v);
}

__global__ void order_kernel(const uint64_t* sorted, int64_t n, const int64_t* off, int32_t* order, int32_t* perm,
                             int32_t* ndeg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = static_cast<int32_t>(sorted[i] & 0xFFFFFFFFull);
    order[i] = x;
    perm[x] = static_cast<int32_t>(i);
    ndeg[i] = static_cast<int32_t>(off[x + 1] - off[x]);
  }
}

// ------------------------------------------------------- H list
__global__ void hcount_kernel(const VMeta* meta, int64_t n, int32_t* hc) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    hc[x] = meta[x].sfe - meta[x].hfb;
}

// Rows with at most kShort cover edges: one thread; longer: one wave.
__global__ __launch_bounds__(kThreads) void hlist_kernel(const VMeta* meta, const int32_t* cols, int64_t n,
                                                         const int64_t* h_off, int64_t cap, int32_t* h_u,
                                                         int32_t* h_v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += stride) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb;
    if (hf == 0 || hf > kShort) continue;
    const int64_t src = m.begin + m.hfb, dst = h_off[x];
    for (int i = 0; i < hf && dst + i < cap; ++i) {
      h_u[dst + i] = static_cast<int32_t>(x);
      h_v[dst + i] = cols[src + i];
    }
  }
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = stride / kWave;
  for (int64_t x = wid; x < n; x += nw) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb;
    if (hf <= kShort) continue;
    const int64_t src = m.begin + m.hfb, dst = h_off[x];
    for (int i = lane(); i < hf && dst + i < cap; i += kWave) {
      h_u[dst + i] = static_cast<int32_t>(x);
      h_v[dst + i] = cols[src + i];
    }
  }
}

__global__ void copy_total_kernel(const int64_t* h_off, int64_t n, int64_t* out) { *out = h_off[n]; }

}  // namespace

SplitWs split_reserve(Carver& c, int64_t n, int64_t nnz) {
  SplitWs w;
  w.meta = c.take<VMeta>(n + 1);
  w.scols = c.take<int32_t>(nnz + kColPad);
  w.res = c.take<uint32_t>(1);
  w.nseg = c.take<int32_t>(n + 1);
  w.seg_off = c.take<int64_t>(n + 2);
  // Segmented rows have deg > kBigCap entries and ceil(deg / kSeg) <= deg / kSeg + deg / kBigCap segments.
  const int64_t max_segs = nnz / kSeg + nnz / kBigCap + 2;
  w.seg_vtx = c.take<int32_t>(max_segs + 1);
  w.seg_cnt = c.take<int32_t>((kMaxGroups + 1) * (max_segs + 1));  // sized for the most groups
  w.seg_pre = c.take<int64_t>(kMaxGroups * (max_segs + 1));
  w.ctr = c.take<int64_t>(4);
  w.rcat = c.take<int32_t>(n + 1);
  w.cat_pre = c.take<int64_t>(n + 1);
  constexpr int kCtxWords = sizeof(RowCtxT<kMaxGroups>) / sizeof(int64_t);  // the largest context
  w.mid_ctx = c.take<int64_t>(kCtxWords * (std::min(n, nnz / (kShort + 1)) + 2));
  w.big_ctx = c.take<int64_t>(kCtxWords * (nnz / (kMidCap + 1) + 2));
  w.stash = c.take<int32_t>(nnz + 1);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1));
  return w;
}

int split_run(const tc_csr* g, const int32_t* L, bool full_levels, SplitWs& w, hipStream_t s) {
  (void)full_levels;
  if (g->n == 0) return TC_OK;
  IdentityLayout lay{g->row_offsets, L};
  return layout_run(lay, g->cols, g->n, g->nnz, w, s);
}

RelabelWs relabel_reserve(Carver& c, int64_t n, int64_t max_vlevels) {
  RelabelWs w;
  w.order = c.take<int32_t>(n + 1);
  w.perm = c.take<int32_t>(n + 1);
  w.off = c.take<int64_t>(n + 2);
  // up to kMaxDegGroups groups per virtual level, plus the (empty) groups of the level after the last
  w.lstart_cnt = c.take<int32_t>(kMaxDegGroups * (max_vlevels + 2) + 1);
  w.lstart = c.take<int64_t>(kMaxDegGroups * (max_vlevels + 2) + 1);
  w.keys = c.take<uint64_t>(n + 1);
  w.keys_tmp = c.take<uint64_t>(n + 1);
  w.deg = c.take<int32_t>(n + 1);
  const size_t a = radix_ws_bytes(n), b = scan_ws_bytes(n + 2);
  w.scratch = c.take<char>(a > b ? a : b);
  return w;
}

namespace {

template <int G>
int relabel_groups(const tc_csr* g, const int32_t* L, const uint32_t* comp0, int32_t d0, int32_t nvl,
                   RelabelWs& w, SplitWs& sp, hipStream_t s) {
  const int64_t n = g->n;
  const unsigned gv = grid_for(n, kThreads, 16384);
  // New ids: by virtual level, inside a level by degree group (deg_group),
  // each group in id order.  The counting test compares ids only inside one
  // level, and any total order there gives the same H (as a set), T and
  // per-vertex counts: a triangle with one horizontal edge is counted at
  // that edge, an all-horizontal one {a, b, c} once, at its first edge with
  // its last vertex as apex.  Ordering by degree keeps the forward
  // same-level lists of the vertices of large degree short (the same-class
  // work sum over H of min(a, b) at R-MAT S22 is 6% below that of a single
  // split at degree 2048); on graphs under 2^26 entries two groups (a split
  // at degree 2048) lay out faster and count as fast.
  const int32_t ngroups = G * (nvl + 1);
  TC_TRY(fill_i32(w.lstart_cnt, 0, ngroups + 1, s));
  // few blocks: each adds its LDS histogram to the shared counts once
  vl_hist_kernel<G><<<grid_for(n, kThreads, static_cast<unsigned>(num_cus() * 2)), kThreads, 0, s>>>(
      g->row_offsets, L, comp0, d0, n, ngroups, w.lstart_cnt);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.lstart_cnt, w.lstart, ngroups, sc, s));
  }
  vl_keys_kernel<G><<<gv, kThreads, 0, s>>>(g->row_offsets, L, comp0, d0, n, w.keys);
  int bits = 0;
  while ((int64_t(1) << bits) < ngroups) ++bits;
  uint64_t* sorted = w.keys;
  TC_TRY(radix_sort_u64(w.keys, w.keys_tmp, n, 32, 32 + bits, w.scratch, s, &sorted));
  order_kernel<<<gv, kThreads, 0, s>>>(sorted, n, g->row_offsets, w.order, w.perm, w.deg);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.deg, w.off, n, sc, s));
  }
  RelabelLayout<G> lay{g->row_offsets, w.off, w.order, w.perm, L, comp0, d0, w.lstart};
  return layout_run(lay, g->cols, n, g->nnz, sp, s);
}

}  // namespace

int relabel_run(const tc_csr* g, const int32_t* L, const uint32_t* comp0, int32_t d0, int32_t nvl,
                int degree_groups, RelabelWs& w, SplitWs& sp, hipStream_t s) {
  if (g->n == 0) return TC_OK;
  if (degree_groups == 4) return relabel_groups<4>(g, L, comp0, d0, nvl, w, sp, s);
  if (degree_groups == 2) return relabel_groups<2>(g, L, comp0, d0, nvl, w, sp, s);
  return fail(TC_ERR_INVALID_ARG, "relabel: degree_groups must be 2 or 4");
}

int hlist_run(const tc_csr* g, const VMeta* meta, const int32_t* cols, int64_t* h_off, int32_t* h_u, int32_t* h_v,
              int64_t cap, int64_t* h_count, char* scratch, hipStream_t s) {
  const int64_t n = g->n;
  if (n == 0) {
    TC_TRY(fill_i64(h_off, 0, 1, s));
    if (h_count) TC_TRY(fill_i64(h_count, 0, 1, s));
    return TC_OK;
  }
  Carver sc(scratch);
  int32_t* hc = sc.take<int32_t>(n + 1);
  hcount_kernel<<<grid_for(n, kThreads, 16384), kThreads, 0, s>>>(meta, n, hc);
  TC_TRY(scan_exclusive<int32_t>(hc, h_off, n, sc, s));
  if (h_u)
    hlist_kernel<<<static_cast<unsigned>(num_cus() * 8), kThreads, 0, s>>>(meta, cols, n, h_off, cap, h_u, h_v);
  if (h_count) copy_total_kernel<<<1, 1, 0, s>>>(h_off, n, h_count);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
