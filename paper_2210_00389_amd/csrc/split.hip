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
//   * relabelled (for counting): vertices renumbered by (virtual level, id),
//     columns rewritten to the new ids, classes read off the new id ranges.
//     Within one (component, level) class the new order is the old order,
//     and the method only compares ids inside such a class, so H and every
//     count are unchanged; each level becomes a contiguous id range, which
//     keeps the probe sets of the counting kernels inside a small id window.
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
// A layout maps output row i to an input row and classifies its entries:
//   ctx(i)          per-row context
//   cls(c, w, v)    class of input entry w (0 up, 1 same, 2 down); v gets
//                   the value written to the output row
//   recls(c, v)     the same class, from the output value v
struct RowCtx {
  int64_t ib, ie, ob;  // input range, output begin
  int32_t self;        // the row's own id in the output numbering
  int32_t key;         // the row's (virtual) level
  int64_t lo, hi;      // same-level id window (relabelled layout)
};

struct IdentityLayout {
  const int64_t* off;
  const int32_t* L;
  __device__ __forceinline__ RowCtx ctx(int64_t i) const {
    RowCtx c;
    c.ib = off[i];
    c.ie = off[i + 1];
    c.ob = c.ib;
    c.self = static_cast<int32_t>(i);
    c.key = L[i];
    c.lo = c.hi = 0;
    return c;
  }
  __device__ __forceinline__ int cls(const RowCtx& c, int32_t w, int32_t& v) const {
    v = w;
    const int lw = L[w];
    return lw < c.key ? 0 : (lw == c.key ? 1 : 2);
  }
  // class of an entry from its output value
  __device__ __forceinline__ int recls(const RowCtx& c, int32_t v) const {
    const int lv = L[v];
    return lv < c.key ? 0 : (lv == c.key ? 1 : 2);
  }
};

struct RelabelLayout {
  const int64_t* off;    // input row offsets
  const int64_t* noff;   // output row offsets
  const int32_t* order;  // new id -> old id
  const int32_t* perm;   // old id -> new id
  const int32_t* L;
  const uint32_t* comp0;
  int32_t d0;
  const int64_t* lstart;
  __device__ __forceinline__ RowCtx ctx(int64_t i) const {
    RowCtx c;
    const int32_t x = order[i];
    c.ib = off[x];
    c.ie = off[x + 1];
    c.ob = noff[i];
    c.self = static_cast<int32_t>(i);
    const int vl = L[x] + (((comp0[x >> 5] >> (x & 31)) & 1u) ? 0 : d0);
    c.key = vl;
    c.lo = lstart[vl];
    c.hi = lstart[vl + 1];
    return c;
  }
  __device__ __forceinline__ int cls(const RowCtx& c, int32_t w, int32_t& v) const {
    v = perm[w];
    return recls(c, v);
  }
  __device__ __forceinline__ int recls(const RowCtx& c, int32_t v) const { return v < c.lo ? 0 : (v < c.hi ? 1 : 2); }
};

// Rows of at most kShort entries: one thread; the row and the classes of its
// entries are loaded into registers first (all gathers in flight at once),
// then counted and scattered.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_short_kernel(Lay lay, const int32_t* cols, int64_t n, int32_t* out,
                                                             VMeta* meta, int32_t* nseg, int32_t* rcat) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const RowCtx c = lay.ctx(i);
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
    for (int q = 0; q < kShort; ++q) kc[q] = q < deg ? lay.cls(c, wv[q], vv[q]) : 3;
    int up = 0, same = 0, slt = 0;
#pragma unroll
    for (int q = 0; q < kShort; ++q) {
      up += kc[q] == 0;
      same += kc[q] == 1;
      slt += (kc[q] == 1) & (vv[q] < c.self);
    }
    int pu = 0, ps = up, pd = up + same;
#pragma unroll
    for (int q = 0; q < kShort; ++q) {
      if (kc[q] == 3) continue;
      const int pos = kc[q] == 0 ? pu++ : (kc[q] == 1 ? ps++ : pd++);
      out[c.ob + pos] = vv[q];
    }
    meta[i] = VMeta{c.ob, up, up + slt, up + same, deg, {c.key, 0}};
  }
}

// Row lists of the two staged categories from their packed scan, as row
// contexts: the kernels that lay these rows out then start with one load
// instead of the chain of dependent loads ctx() makes.
template <class Lay>
__global__ void row_list_kernel(Lay lay, const int32_t* rcat, int64_t n, const int64_t* pre, RowCtx* mid_ctx,
                                RowCtx* big_ctx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = rcat[i];
    if (c == kRowMid) mid_ctx[pre[i] & 0xFFFFFFFFll] = lay.ctx(i);
    else if (c == kRowBig) big_ctx[pre[i] >> 32] = lay.ctx(i);
  }
}

// A wave's part of a row: up to R * 64 entries from part_begin, held in
// registers (lane l has entries part_begin + u * 64 + l); -1 past the end.
template <int R>
__device__ __forceinline__ void load_part(const int32_t* cols, const RowCtx& c, int part_begin, int32_t (&wv)[R]) {
  const int lim = static_cast<int>(c.ie - c.ib) - part_begin;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int j = u * kWave + lane();
    wv[u] = j < lim ? cols[c.ib + part_begin + j] : -1;
  }
}

// Classes of a part (2 bits per entry in *kp, 3 = none) and its output ids;
// returns the part's counts packed as up | same << 16 | same-below-x << 32
// | down << 48 (each < 2^16).
template <class Lay, int R>
__device__ __forceinline__ uint64_t classify_part(const Lay& lay, const RowCtx& c, const int32_t (&wv)[R],
                                                  int32_t (&vv)[R], uint32_t* kp) {
  uint32_t k2 = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    vv[u] = 0;
    const int k = wv[u] >= 0 ? lay.cls(c, wv[u], vv[u]) : 3;
    k2 |= static_cast<uint32_t>(k) << (2 * u);
  }
  uint64_t up = 0, same = 0, slt = 0, down = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const uint32_t k = (k2 >> (2 * u)) & 3u;
    up += __popcll(__ballot(k == 0));
    same += __popcll(__ballot(k == 1));
    slt += __popcll(__ballot((k == 1) & (vv[u] < c.self)));
    down += __popcll(__ballot(k == 2));
  }
  *kp = k2;
  return up | (same << 16) | (slt << 32) | (down << 48);
}

// Scatter of a part: the class regions continue at pu / ps / pd (absolute
// output positions); entries keep their order inside each class.
template <int R>
__device__ __forceinline__ void write_part(const int32_t (&vv)[R], uint32_t k2, int64_t pu, int64_t ps, int64_t pd,
                                           int32_t* out) {
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const uint32_t k = (k2 >> (2 * u)) & 3u;
    const uint64_t mu = __ballot(k == 0), ms = __ballot(k == 1), md = __ballot(k == 2);
    if (k == 0) out[pu + __popcll(mu & lt)] = vv[u];
    else if (k == 1) out[ps + __popcll(ms & lt)] = vv[u];
    else if (k == 2) out[pd + __popcll(md & lt)] = vv[u];
    pu += __popcll(mu);
    ps += __popcll(ms);
    pd += __popcll(md);
  }
}

constexpr uint64_t kF16 = 0xFFFF;

// Rows of up to R * 64 entries, one wave each.  The wave loads the context
// and the columns of its next row before it classifies and writes the
// current one, so the memory latencies of two rows overlap.
template <class Lay, int R>
__global__ __launch_bounds__(kThreads) void lay_mid_kernel(Lay lay, const int32_t* cols, const RowCtx* rows,
                                                           const int64_t* count, int32_t* out, VMeta* meta) {
  static_assert(R * kWave < (1 << 16), "part counts are packed in 16-bit fields");
  const int64_t nrows = *count & 0xFFFFFFFFll;
  const int64_t nw = (int64_t)gridDim.x * (kThreads / kWave);
  int64_t r = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  if (r >= nrows) return;
  RowCtx c = rows[r];
  int32_t wv[R];
  load_part<R>(cols, c, 0, wv);
  for (;;) {
    const int64_t rn = r + nw;
    const bool more = rn < nrows;
    RowCtx cn = c;
    if (more) cn = rows[rn];
    int32_t vv[R];
    uint32_t k2;
    const uint64_t pk = classify_part<Lay, R>(lay, c, wv, vv, &k2);
    int32_t wn[R];
    if (more) load_part<R>(cols, cn, 0, wn);
    const int up = static_cast<int>(pk & kF16), same = static_cast<int>((pk >> 16) & kF16);
    const int slt = static_cast<int>((pk >> 32) & kF16);
    const int deg = static_cast<int>(c.ie - c.ib);
    if (lane() == 0) meta[c.self] = VMeta{c.ob, up, up + slt, up + same, deg, {c.key, 0}};
    write_part<R>(vv, k2, c.ob, c.ob + up, c.ob + up + same, out);
    if (!more) break;
    r = rn;
    c = cn;
#pragma unroll
    for (int u = 0; u < R; ++u) wv[u] = wn[u];
  }
}

// Rows of up to WPR * R * 64 entries, one block of WPR waves each; wave q
// holds entries [q * R * 64, (q + 1) * R * 64) and the waves' class counts
// are combined through LDS.
template <class Lay, int WPR, int R>
__global__ __launch_bounds__(WPR * kWave) void lay_block_kernel(Lay lay, const int32_t* cols, const RowCtx* rows,
                                                                const int64_t* count, int32_t* out, VMeta* meta) {
  constexpr int kPart = R * kWave;
  static_assert(WPR * kPart < (1 << 16), "row counts are packed in 16-bit fields");
  __shared__ uint64_t s_pk[WPR];
  const int wave = threadIdx.x / kWave;
  const int64_t nrows = *count >> 32;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const RowCtx c = rows[r];
    int32_t wv[R], vv[R];
    uint32_t k2;
    load_part<R>(cols, c, wave * kPart, wv);
    const uint64_t pk = classify_part<Lay, R>(lay, c, wv, vv, &k2);
    if (lane() == 0) s_pk[wave] = pk;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int q = 0; q < WPR; ++q) {
      const uint64_t x = s_pk[q];
      if (q < wave) before += x;
      tot += x;
    }
    const int64_t up = static_cast<int64_t>(tot & kF16), same = static_cast<int64_t>((tot >> 16) & kF16);
    const int64_t slt = static_cast<int64_t>((tot >> 32) & kF16);
    const int deg = static_cast<int>(c.ie - c.ib);
    if (threadIdx.x == 0)
      meta[c.self] = VMeta{c.ob, static_cast<int>(up), static_cast<int>(up + slt), static_cast<int>(up + same), deg,
                           {c.key, 0}};
    write_part<R>(vv, k2, c.ob + static_cast<int64_t>(before & kF16),
                  c.ob + up + static_cast<int64_t>((before >> 16) & kF16),
                  c.ob + up + same + static_cast<int64_t>((before >> 48) & kF16), out);
    __syncthreads();  // s_pk is rewritten for the next row
  }
}

__global__ void seg_vtx_kernel(const int32_t* nseg, const int64_t* seg_off, int64_t n, int32_t* seg_vtx) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[x];
    const int64_t s0 = seg_off[x];
    for (int i = 0; i < k; ++i) seg_vtx[s0 + i] = static_cast<int32_t>(x);
  }
}

// One wave per segment of a long row: class counts of the segment.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_seg_count_kernel(Lay lay, const int32_t* cols, int64_t n,
                                                                 const int64_t* seg_off, const int32_t* seg_vtx,
                                                                 int32_t* seg_cnt, int32_t* stash) {
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t i = seg_vtx[sg];
    const RowCtx c = lay.ctx(i);
    const int64_t s = sg - seg_off[i];
    const int64_t b = c.ib + s * kSeg;
    const int64_t e = min(c.ie, b + kSeg);
    int up = 0, same = 0, slt = 0;
    for (int64_t j0 = b; j0 < e; j0 += kRounds * kWave) {
      int32_t wv[kRounds];
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        const int64_t j = j0 + u * kWave + lane();
        wv[u] = j < e ? cols[j] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        int k = 3;
        int32_t v = 0;
        if (wv[u] >= 0) {
          k = lay.cls(c, wv[u], v);
          stash[j0 + u * kWave + lane()] = v;  // the scatter pass reads the ids back instead of gathering again
        }
        up += __popcll(__ballot(k == 0));
        same += __popcll(__ballot(k == 1));
        slt += __popcll(__ballot((k == 1) & (v < c.self)));
      }
    }
    if (lane() == 0) {
      seg_cnt[3 * sg + 0] = up;
      seg_cnt[3 * sg + 1] = same;
      seg_cnt[3 * sg + 2] = slt;
    }
  }
}

// Per long row: prefix of its segments' counts, and the row record.
template <class Lay>
__global__ void lay_seg_prefix_kernel(Lay lay, int64_t n, const int32_t* nseg, const int64_t* seg_off,
                                      const int32_t* seg_cnt, int32_t* seg_pre, VMeta* meta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[i];
    if (k == 0) continue;
    const int64_t s0 = seg_off[i];
    int up = 0, same = 0, slt = 0;
    for (int j = 0; j < k; ++j) {
      const int64_t sg = s0 + j;
      seg_pre[3 * sg + 0] = up;
      seg_pre[3 * sg + 1] = same;
      up += seg_cnt[3 * sg + 0];
      same += seg_cnt[3 * sg + 1];
      slt += seg_cnt[3 * sg + 2];
    }
    const RowCtx c = lay.ctx(i);
    meta[i] = VMeta{c.ob, up, up + slt, up + same, static_cast<int32_t>(c.ie - c.ib), {c.key, 0}};
  }
}

// One wave per segment: stable scatter of the segment's entries.
template <class Lay>
__global__ __launch_bounds__(kThreads) void lay_seg_write_kernel(Lay lay, const int32_t* stash, int64_t n,
                                                                 const int64_t* seg_off, const int32_t* seg_vtx,
                                                                 const int32_t* seg_pre, const VMeta* meta,
                                                                 int32_t* out) {
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const uint64_t lt = lanemask_lt();
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t i = seg_vtx[sg];
    const RowCtx c = lay.ctx(i);
    const int64_t s = sg - seg_off[i];
    const int64_t b = c.ib + s * kSeg;
    const int64_t e = min(c.ie, b + kSeg);
    const VMeta m = meta[i];
    int64_t pu = seg_pre[3 * sg + 0];
    int64_t ps = m.up + seg_pre[3 * sg + 1];
    int64_t pd = m.sfe + (s * kSeg - seg_pre[3 * sg + 0] - seg_pre[3 * sg + 1]);
    for (int64_t j0 = b; j0 < e; j0 += kRounds * kWave) {
      int32_t vv[kRounds];
      int kc[kRounds];
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        const int64_t j = j0 + u * kWave + lane();
        vv[u] = j < e ? stash[j] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRounds; ++u) kc[u] = vv[u] >= 0 ? lay.recls(c, vv[u]) : 3;
#pragma unroll
      for (int u = 0; u < kRounds; ++u) {
        const int k = kc[u];
        const uint64_t mu = __ballot(k == 0), ms = __ballot(k == 1), md = __ballot(k == 2);
        if (k == 0) out[c.ob + pu + __popcll(mu & lt)] = vv[u];
        else if (k == 1) out[c.ob + ps + __popcll(ms & lt)] = vv[u];
        else if (k == 2) out[c.ob + pd + __popcll(md & lt)] = vv[u];
        pu += __popcll(mu);
        ps += __popcll(ms);
        pd += __popcll(md);
      }
    }
  }
}

template <class Lay>
int layout_run(const Lay& lay, const int32_t* cols, int64_t n, SplitWs& w, hipStream_t s) {
  const unsigned gv = grid_for(n, kThreads, 16384);
  const unsigned gw = static_cast<unsigned>(num_cus() * 8);
  lay_short_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, cols, n, w.scols, w.meta, w.nseg, w.rcat);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive_pair(w.rcat, kRowMid, kRowBig, w.cat_pre, n, sc, s));
  }
  RowCtx* mid_ctx = reinterpret_cast<RowCtx*>(w.mid_ctx);
  RowCtx* big_ctx = reinterpret_cast<RowCtx*>(w.big_ctx);
  row_list_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, w.rcat, n, w.cat_pre, mid_ctx, big_ctx);
  lay_mid_kernel<Lay, kMidR><<<static_cast<unsigned>(num_cus() * 8), kThreads, 0, s>>>(lay, cols, mid_ctx,
                                                                                      w.cat_pre + n, w.scols, w.meta);
  lay_block_kernel<Lay, kBigWaves, kBigR><<<static_cast<unsigned>(num_cus() * 4), kBigWaves * kWave, 0, s>>>(
      lay, cols, big_ctx, w.cat_pre + n, w.scols, w.meta);
  TC_HIP(hipGetLastError());
  Carver sc(w.scratch);
  TC_TRY(scan_exclusive<int32_t>(w.nseg, w.seg_off, n, sc, s));
  seg_vtx_kernel<<<gv, kThreads, 0, s>>>(w.nseg, w.seg_off, n, w.seg_vtx);
  lay_seg_count_kernel<Lay><<<gw, kThreads, 0, s>>>(lay, cols, n, w.seg_off, w.seg_vtx, w.seg_cnt, w.stash);
  lay_seg_prefix_kernel<Lay><<<gv, kThreads, 0, s>>>(lay, n, w.nseg, w.seg_off, w.seg_cnt, w.seg_pre, w.meta);
  lay_seg_write_kernel<Lay><<<gw, kThreads, 0, s>>>(lay, w.stash, n, w.seg_off, w.seg_vtx, w.seg_pre, w.meta,
                                                    w.scols);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

// ------------------------------------------------------- relabelling
// Virtual level: L(v) in r0's component, L(v) + d0 elsewhere.
__device__ __forceinline__ int vlevel(const int32_t* L, const uint32_t* comp0, int32_t d0, int64_t v) {
  return L[v] + (((comp0[v >> 5] >> (v & 31)) & 1u) ? 0 : d0);
}

__global__ __launch_bounds__(kThreads) void vl_hist_kernel(const int32_t* L, const uint32_t* comp0, int32_t d0,
                                                           int64_t n, int32_t nvl, int32_t* cnt) {
  constexpr int kLds = 1024;
  __shared__ int32_t h[kLds];
  const bool local = nvl <= kLds;
  if (local)
    for (int i = threadIdx.x; i < nvl; i += kThreads) h[i] = 0;
  __syncthreads();
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int vl = vlevel(L, comp0, d0, v);
    if (local) atomicAdd(&h[vl], 1);
    else atomicAdd(&cnt[vl], 1);
  }
  __syncthreads();
  if (local)
    for (int i = threadIdx.x; i < nvl; i += kThreads)
      if (h[i]) atomicAdd(&cnt[i], h[i]);
}

__global__ void vl_keys_kernel(const int32_t* L, const uint32_t* comp0, int32_t d0, int64_t n, uint64_t* keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = (static_cast<uint64_t>(vlevel(L, comp0, d0, v)) << 32) | static_cast<uint64_t>(v);
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
  w.seg_cnt = c.take<int32_t>(3 * max_segs + 3);
  w.seg_pre = c.take<int32_t>(3 * max_segs + 3);
  w.ctr = c.take<int64_t>(4);
  w.rcat = c.take<int32_t>(n + 1);
  w.cat_pre = c.take<int64_t>(n + 1);
  static_assert(sizeof(RowCtx) == 6 * sizeof(int64_t), "row contexts are stored as six int64 words");
  w.mid_ctx = c.take<int64_t>(6 * (std::min(n, nnz / (kShort + 1)) + 2));
  w.big_ctx = c.take<int64_t>(6 * (nnz / (kMidCap + 1) + 2));
  w.stash = c.take<int32_t>(nnz + 1);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1));
  return w;
}

int split_run(const tc_csr* g, const int32_t* L, bool full_levels, SplitWs& w, hipStream_t s) {
  (void)full_levels;
  if (g->n == 0) return TC_OK;
  IdentityLayout lay{g->row_offsets, L};
  return layout_run(lay, g->cols, g->n, w, s);
}

RelabelWs relabel_reserve(Carver& c, int64_t n, int64_t max_vlevels) {
  RelabelWs w;
  w.order = c.take<int32_t>(n + 1);
  w.perm = c.take<int32_t>(n + 1);
  w.off = c.take<int64_t>(n + 2);
  w.lstart_cnt = c.take<int32_t>(max_vlevels + 2);
  w.lstart = c.take<int64_t>(max_vlevels + 3);
  w.keys = c.take<uint64_t>(n + 1);
  w.keys_tmp = c.take<uint64_t>(n + 1);
  w.deg = c.take<int32_t>(n + 1);
  const size_t a = radix_ws_bytes(n), b = scan_ws_bytes(n + 2);
  w.scratch = c.take<char>(a > b ? a : b);
  return w;
}

int relabel_run(const tc_csr* g, const int32_t* L, const uint32_t* comp0, int32_t d0, int32_t nvl, RelabelWs& w,
                SplitWs& sp, hipStream_t s) {
  const int64_t n = g->n;
  if (n == 0) return TC_OK;
  const unsigned gv = grid_for(n, kThreads, 16384);
  TC_TRY(fill_i32(w.lstart_cnt, 0, nvl + 1, s));
  // few blocks: each adds its LDS histogram to the shared counts once
  vl_hist_kernel<<<grid_for(n, kThreads, static_cast<unsigned>(num_cus() * 2)), kThreads, 0, s>>>(
      L, comp0, d0, n, nvl, w.lstart_cnt);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.lstart_cnt, w.lstart, nvl, sc, s));
  }
  vl_keys_kernel<<<gv, kThreads, 0, s>>>(L, comp0, d0, n, w.keys);
  int bits = 0;
  while ((int64_t(1) << bits) < nvl) ++bits;
  uint64_t* sorted = w.keys;
  TC_TRY(radix_sort_u64(w.keys, w.keys_tmp, n, 32, 32 + bits, w.scratch, s, &sorted));
  order_kernel<<<gv, kThreads, 0, s>>>(sorted, n, g->row_offsets, w.order, w.perm, w.deg);
  TC_HIP(hipGetLastError());
  {
    Carver sc(w.scratch);
    TC_TRY(scan_exclusive<int32_t>(w.deg, w.off, n, sc, s));
  }
  RelabelLayout lay{g->row_offsets, w.off, w.order, w.perm, L, comp0, d0, w.lstart};
  return layout_run(lay, g->cols, n, sp, s);
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
