// split.hip -- level-class layout of the adjacency and the cover-edge list.
//
// Alg. 1 selects the horizontal edges (L(u) = L(v), u < v) and tests every
// common neighbour w of a cover edge against L(w) = L(u).  Because BFS levels
// of adjacent vertices differ by at most one (the parity argument of
// Lemma 1), the level of a neighbour relative to its row is one of three
// classes -- one up, same, one down -- and L mod 4 (2 bits per vertex, 4 MB
// for 16.7 M vertices, so it stays in L2) is enough to tell them apart.
//
// This pass rewrites every row as [Up | Same | Down], each part still
// ascending (a stable partition), and records per vertex the class bounds and
// the start of Hfwd(x) = {v in Same(x) : v > x}, the cover edges leaving x.
// The counting kernels then evaluate the test structurally: a common
// neighbour found in two Up lists or two Down lists is on another level, and
// one found in two Same lists is counted only when it lies above v.
//
// Rows of up to kShort entries are handled by one thread each; longer rows
// are cut into segments of kSeg entries handled by one wave each (counts,
// then a per-row prefix over its segments, then a stable ballot scatter).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kShort = 32;
constexpr int kSeg = 2048;

// class of neighbour w of row x: 0 = up, 1 = same, 2 = down
struct FullLevels {
  const int32_t* L;
  __device__ __forceinline__ int row(int64_t x) const { return L[x]; }
  __device__ __forceinline__ int cls(int rowkey, int32_t w) const {
    int lw = L[w];
    return lw < rowkey ? 0 : (lw == rowkey ? 1 : 2);
  }
};

struct Residues {
  const uint32_t* res;
  __device__ __forceinline__ int get(int64_t v) const {
    return static_cast<int>((res[v >> 4] >> ((v & 15) * 2)) & 3u);
  }
  __device__ __forceinline__ int row(int64_t x) const { return get(x); }
  __device__ __forceinline__ int cls(int rowkey, int32_t w) const {
    int d = (get(w) - rowkey) & 3;  // 0 same, 1 down, 3 up
    return d == 0 ? 1 : (d == 3 ? 0 : 2);
  }
};

__global__ void pack_res_kernel(const int32_t* L, int64_t n, uint32_t* res) {
  const int64_t words = (n + 15) / 16;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t r = 0;
    const int64_t v0 = i * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (v0 + j < n) r |= (static_cast<uint32_t>(L[v0 + j]) & 3u) << (2 * j);
    res[i] = r;
  }
}

template <class C>
__global__ __launch_bounds__(kThreads) void split_short_kernel(const int64_t* off, const int32_t* cols,
                                                               int64_t n, C cl, int32_t* scols,
                                                               VMeta* meta, int32_t* nseg) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = off[x], e = off[x + 1];
    const int32_t deg = static_cast<int32_t>(e - b);
    if (deg > kShort) {
      nseg[x] = (deg + kSeg - 1) / kSeg;
      continue;
    }
    nseg[x] = 0;
    const int rk = deg ? cl.row(x) : 0;
    int up = 0, same = 0, slt = 0;
    for (int64_t j = b; j < e; ++j) {
      int32_t w = cols[j];
      int c = cl.cls(rk, w);
      up += c == 0;
      same += c == 1;
      slt += (c == 1) & (w < x);
    }
    int pu = 0, ps = up, pd = up + same;
    for (int64_t j = b; j < e; ++j) {
      int32_t w = cols[j];
      int c = cl.cls(rk, w);
      int pos = c == 0 ? pu++ : (c == 1 ? ps++ : pd++);
      scols[b + pos] = w;
    }
    meta[x] = VMeta{b, up, up + slt, up + same, deg, {0, 0}};
  }
}

__global__ void seg_vtx_kernel(const int32_t* nseg, const int64_t* seg_off, int64_t n, int32_t* seg_vtx) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[x];
    const int64_t s0 = seg_off[x];
    for (int i = 0; i < k; ++i) seg_vtx[s0 + i] = static_cast<int32_t>(x);
  }
}

template <class C>
__global__ __launch_bounds__(kThreads) void seg_count_kernel(const int64_t* off, const int32_t* cols,
                                                             int64_t n, C cl, const int64_t* seg_off,
                                                             const int32_t* seg_vtx, int32_t* seg_cnt) {
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t x = seg_vtx[sg];
    const int64_t s = sg - seg_off[x];
    const int64_t b = off[x] + s * kSeg;
    const int64_t e = min(off[x + 1], b + kSeg);
    const int rk = cl.row(x);
    int up = 0, same = 0, slt = 0;
    for (int64_t j0 = b; j0 < e; j0 += kWave) {
      const int64_t j = j0 + lane();
      int c = 3;
      int32_t w = 0;
      if (j < e) {
        w = cols[j];
        c = cl.cls(rk, w);
      }
      up += __popcll(__ballot(c == 0));
      same += __popcll(__ballot(c == 1));
      slt += __popcll(__ballot((c == 1) & (w < x)));
    }
    if (lane() == 0) {
      seg_cnt[3 * sg + 0] = up;
      seg_cnt[3 * sg + 1] = same;
      seg_cnt[3 * sg + 2] = slt;
    }
  }
}

__global__ void seg_prefix_kernel(const int64_t* off, int64_t n, const int32_t* nseg, const int64_t* seg_off,
                                  const int32_t* seg_cnt, int32_t* seg_pre, VMeta* meta) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int k = nseg[x];
    if (k == 0) continue;
    const int64_t s0 = seg_off[x];
    int up = 0, same = 0, slt = 0;
    for (int i = 0; i < k; ++i) {
      const int64_t sg = s0 + i;
      seg_pre[3 * sg + 0] = up;
      seg_pre[3 * sg + 1] = same;
      up += seg_cnt[3 * sg + 0];
      same += seg_cnt[3 * sg + 1];
      slt += seg_cnt[3 * sg + 2];
    }
    const int32_t deg = static_cast<int32_t>(off[x + 1] - off[x]);
    meta[x] = VMeta{off[x], up, up + slt, up + same, deg, {0, 0}};
  }
}

template <class C>
__global__ __launch_bounds__(kThreads) void seg_write_kernel(const int64_t* off, const int32_t* cols,
                                                             int64_t n, C cl, const int64_t* seg_off,
                                                             const int32_t* seg_vtx, const int32_t* seg_pre,
                                                             const VMeta* meta, int32_t* scols) {
  const int64_t nsegs = seg_off[n];
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t sg = wid; sg < nsegs; sg += nw) {
    const int32_t x = seg_vtx[sg];
    const int64_t s = sg - seg_off[x];
    const int64_t rb = off[x];
    const int64_t b = rb + s * kSeg;
    const int64_t e = min(off[x + 1], b + kSeg);
    const VMeta mx = meta[x];
    const int rk = cl.row(x);
    int64_t pu = seg_pre[3 * sg + 0];
    int64_t ps = mx.up + seg_pre[3 * sg + 1];
    int64_t pd = mx.sfe + (s * kSeg - seg_pre[3 * sg + 0] - seg_pre[3 * sg + 1]);
    const uint64_t lt = lanemask_lt();
    for (int64_t j0 = b; j0 < e; j0 += kWave) {
      const int64_t j = j0 + lane();
      int c = 3;
      int32_t w = 0;
      if (j < e) {
        w = cols[j];
        c = cl.cls(rk, w);
      }
      const uint64_t mu = __ballot(c == 0), ms = __ballot(c == 1), md = __ballot(c == 2);
      if (c == 0) scols[rb + pu + __popcll(mu & lt)] = w;
      else if (c == 1) scols[rb + ps + __popcll(ms & lt)] = w;
      else if (c == 2) scols[rb + pd + __popcll(md & lt)] = w;
      pu += __popcll(mu);
      ps += __popcll(ms);
      pd += __popcll(md);
    }
  }
}

// ------------------------------------------------------- H list
__global__ void hcount_kernel(const VMeta* meta, int64_t n, int32_t* hc) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x)
    hc[x] = meta[x].sfe - meta[x].hfb;
}

// Rows with at most 32 cover edges: one thread; longer: one wave.
__global__ __launch_bounds__(kThreads) void hlist_kernel(const int64_t* off, const VMeta* meta,
                                                         const int32_t* cols, int64_t n,
                                                         const int64_t* h_off, int64_t cap, int32_t* h_u,
                                                         int32_t* h_v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += stride) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb;
    if (hf == 0 || hf > kShort) continue;
    const int64_t src = off[x] + m.hfb, dst = h_off[x];
    for (int i = 0; i < hf && dst + i < cap; ++i) {
      h_u[dst + i] = static_cast<int32_t>(x);
      h_v[dst + i] = cols[src + i];
    }
  }
  // long rows, one wave each
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = stride / kWave;
  for (int64_t x = wid; x < n; x += nw) {
    const VMeta m = meta[x];
    const int hf = m.sfe - m.hfb;
    if (hf <= kShort) continue;
    const int64_t src = off[x] + m.hfb, dst = h_off[x];
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
  w.scols = c.take<int32_t>(nnz + 1);
  w.res = c.take<uint32_t>((n + 15) / 16 + 1);
  w.nseg = c.take<int32_t>(n + 1);
  w.seg_off = c.take<int64_t>(n + 2);
  const int64_t max_segs = nnz / (kShort + 1) + 1;  // every long row has > kShort entries
  w.seg_vtx = c.take<int32_t>(max_segs + 1);
  w.seg_cnt = c.take<int32_t>(3 * max_segs + 3);
  w.seg_pre = c.take<int32_t>(3 * max_segs + 3);
  w.ctr = c.take<int64_t>(4);
  w.scratch = c.take<char>(scan_ws_bytes(n + 1));
  return w;
}

int split_run(const tc_csr* g, const int32_t* L, bool full_levels, SplitWs& w, hipStream_t s) {
  const int64_t n = g->n;
  if (n == 0) return TC_OK;
  const unsigned gv = grid_for(n, kThreads, 16384);
  const unsigned gw = static_cast<unsigned>(num_cus() * 8);
  if (full_levels) {
    FullLevels cl{L};
    split_short_kernel<<<gv, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.scols, w.meta, w.nseg);
  } else {
    pack_res_kernel<<<grid_for((n + 15) / 16, kThreads, 16384), kThreads, 0, s>>>(L, n, w.res);
    Residues cl{w.res};
    split_short_kernel<<<gv, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.scols, w.meta, w.nseg);
  }
  TC_HIP(hipGetLastError());
  Carver sc(w.scratch);
  TC_TRY(scan_exclusive<int32_t>(w.nseg, w.seg_off, n, sc, s));
  seg_vtx_kernel<<<gv, kThreads, 0, s>>>(w.nseg, w.seg_off, n, w.seg_vtx);
  if (full_levels) {
    FullLevels cl{L};
    seg_count_kernel<<<gw, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.seg_off, w.seg_vtx, w.seg_cnt);
  } else {
    Residues cl{w.res};
    seg_count_kernel<<<gw, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.seg_off, w.seg_vtx, w.seg_cnt);
  }
  seg_prefix_kernel<<<gv, kThreads, 0, s>>>(g->row_offsets, n, w.nseg, w.seg_off, w.seg_cnt, w.seg_pre,
                                            w.meta);
  if (full_levels) {
    FullLevels cl{L};
    seg_write_kernel<<<gw, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.seg_off, w.seg_vtx,
                                             w.seg_pre, w.meta, w.scols);
  } else {
    Residues cl{w.res};
    seg_write_kernel<<<gw, kThreads, 0, s>>>(g->row_offsets, g->cols, n, cl, w.seg_off, w.seg_vtx,
                                             w.seg_pre, w.meta, w.scols);
  }
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int hlist_run(const tc_csr* g, const VMeta* meta, const int32_t* cols, int64_t* h_off, int32_t* h_u,
              int32_t* h_v, int64_t cap, int64_t* h_count, char* scratch, hipStream_t s) {
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
    hlist_kernel<<<static_cast<unsigned>(num_cus() * 8), kThreads, 0, s>>>(g->row_offsets, meta, cols, n,
                                                                          h_off, cap, h_u, h_v);
  if (h_count) copy_total_kernel<<<1, 1, 0, s>>>(h_off, n, h_count);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tc
