// tc_api.hip -- the C ABI declared in include/tc.h: argument checks,
// workspace carving, stage sequencing.  No device memory is allocated here.
#include <stdint.h>
#include <string.h>

#include "tc_internal.h"

using namespace tc;

namespace {

constexpr int64_t kMaxN = 0x7FFFFFFFLL;

int check_csr(const tc_csr* g, const char* fn) {
  if (!g) return fail(TC_ERR_INVALID_ARG, "%s: graph is NULL", fn);
  if (g->n < 0 || g->nnz < 0) return fail(TC_ERR_INVALID_ARG, "%s: negative n or nnz", fn);
  if (g->n > kMaxN) return fail(TC_ERR_TOO_LARGE, "%s: n = %lld exceeds 2^31 - 1", fn, (long long)g->n);
  if (g->n > 0 && !g->row_offsets) return fail(TC_ERR_INVALID_ARG, "%s: row_offsets is NULL", fn);
  if (g->nnz > 0 && !g->cols) return fail(TC_ERR_INVALID_ARG, "%s: cols is NULL", fn);
  if (g->n == 0 && g->nnz != 0) return fail(TC_ERR_INVALID_ARG, "%s: nnz > 0 with n = 0", fn);
  return TC_OK;
}

// The count kernels keep a list length below 2^29 beside a flag bit in each
// stream record, so the counting calls refuse graphs in which a vertex could
// reach degree 2^29.  A degree is at most n - 1 and at most nnz / 2 (every
// edge is stored in both rows): only graphs beyond both bounds are refused.
constexpr int64_t kMaxListLen = int64_t(1) << 29;

int check_degree_bound(const tc_csr* g, const char* fn) {
  if (g->n - 1 >= kMaxListLen && g->nnz / 2 >= kMaxListLen)
    return fail(TC_ERR_TOO_LARGE, "%s: n - 1 and nnz / 2 both reach 2^29, so a degree could exceed the longest list "
                "a stream record holds", fn);
  return TC_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need, const char* fn) {
  if (ws_bytes < need)
    return fail(TC_ERR_WORKSPACE, "%s: workspace of %zu bytes, %zu needed", fn, ws_bytes, need);
  if (need > 0 && !ws) return fail(TC_ERR_INVALID_ARG, "%s: workspace is NULL", fn);
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(TC_ERR_INVALID_ARG, "%s: workspace not 256-byte aligned", fn);
  return TC_OK;
}

// ------------------------------------------------------- workspace plans
struct CountPlan {
  int64_t* stats;
  int32_t* L;
  uint32_t* comp0;  // r0's component (kept from the BFS for the relabelling)
  char* region;     // BFS first, then relabelled layout + count
  BfsWs bfs;
  RelabelWs relabel;
  SplitWs split;
  CountWs count;
  int64_t* pv_new;  // per-vertex counts in relabelled ids
  size_t bytes;
};

CountPlan plan_count(void* base, int64_t n, int64_t nnz) {
  CountPlan p;
  Carver c(base);
  p.stats = c.take<int64_t>(24);
  p.L = c.take<int32_t>(n + 1);
  p.comp0 = c.take<uint32_t>((n + 31) / 32 + 1);
  p.region = c.take<char>(0);
  const size_t head = c.used();
  Carver a(p.region);
  p.bfs = bfs_reserve(a, n);
  p.bfs.comp0 = p.comp0;
  Carver b(p.region);
  p.relabel = relabel_reserve(b, n, 2 * n + 2);
  p.split = split_reserve(b, n, nnz);
  p.count = count_reserve(b, n, nnz);
  p.count.stats = p.stats;
  p.pv_new = b.take<int64_t>(n + 1);
  p.bytes = head + (a.used() > b.used() ? a.used() : b.used());
  return p;
}

__global__ void pv_back_kernel(const int64_t* pv_new, const int32_t* order, int64_t n, int64_t* pv) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    pv[order[i]] = pv_new[i];
}

struct BaselinePlan {
  int64_t* stats;
  VMeta* meta;
  int32_t* cols;  // padded copy of the caller's columns
  CountWs count;
  size_t bytes;
};

BaselinePlan plan_baseline(void* base, int64_t n, int64_t nnz) {
  BaselinePlan p;
  Carver c(base);
  p.stats = c.take<int64_t>(24);
  p.meta = c.take<VMeta>(n + 1);
  p.cols = c.take<int32_t>(nnz + kColPad);
  p.count = count_reserve(c, n, nnz);
  p.count.stats = p.stats;
  p.bytes = c.used();
  return p;
}

struct CoverPlan {
  SplitWs split;
  int64_t* h_off;
  char* hscratch;
  size_t bytes;
};

CoverPlan plan_cover(void* base, int64_t n, int64_t nnz) {
  CoverPlan p;
  Carver c(base);
  p.split = split_reserve(c, n, nnz);
  p.h_off = c.take<int64_t>(n + 2);
  p.hscratch = c.take<char>(scan_ws_bytes(n + 1) + (n + 1) * sizeof(int32_t) + 512);
  p.bytes = c.used();
  return p;
}

size_t bfs_bytes(int64_t n) {
  Carver c(nullptr);
  bfs_reserve(c, n);
  return c.used();
}

__global__ void stats_kernel(int64_t* stats, int64_t n, int64_t nnz, int64_t levels) {
  stats[0] = n;
  stats[1] = nnz;
  stats[3] = levels;
}

int maybe_validate(const tc_csr* g, uint32_t flags, void* ws, hipStream_t s) {
  if (!(flags & TC_VALIDATE)) return TC_OK;
  return validate_run(g, ws, s);
}

struct CallScope {
  explicit CallScope(hipStream_t s) { prof_begin_call(s); }
  ~CallScope() { prof_end_call(); }
};

}  // namespace

extern "C" {

size_t tc_workspace_bytes(int op, int64_t n, int64_t nnz, int32_t num_graphs) {
  if (n < 0 || nnz < 0 || num_graphs < 0) return 0;
  size_t b = 0;
  switch (op) {
    case TC_OP_BUILD_CSR: b = build_ws_bytes(n, nnz); break;
    case TC_OP_BFS_LEVELS: b = bfs_bytes(n); break;
    case TC_OP_COVER_EDGES: b = plan_cover(nullptr, n, nnz).bytes; break;
    case TC_OP_COUNT: {
      const size_t a = plan_count(nullptr, n, nnz).bytes, sm = small_ws_bytes(n, nnz);
      b = a > sm ? a : sm;
      break;
    }
    case TC_OP_COUNT_BATCH: b = batch_ws_bytes(n, nnz, num_graphs); break;
    case TC_OP_EDGE_BASELINE: b = plan_baseline(nullptr, n, nnz).bytes; break;
    case TC_OP_VALIDATE: b = validate_ws_bytes(n, nnz); break;
    case TC_OP_SELECT_ROOT: b = select_root_ws_bytes(n); break;
    default: return 0;
  }
  const size_t v = validate_ws_bytes(n, nnz);
  return b > v ? b : v;
}

int tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, int64_t* row_offsets,
                 int32_t* cols, int64_t* nnz_out, void* ws, size_t ws_bytes, tc_stream_t stream) {
  if (n < 0 || num_pairs < 0) return fail(TC_ERR_INVALID_ARG, "tc_build_csr: negative size");
  if (n > kMaxN) return fail(TC_ERR_TOO_LARGE, "tc_build_csr: n exceeds 2^31 - 1");
  if (!row_offsets || !nnz_out) return fail(TC_ERR_INVALID_ARG, "tc_build_csr: NULL output");
  if (num_pairs > 0 && (!src || !dst || !cols)) return fail(TC_ERR_INVALID_ARG, "tc_build_csr: NULL pairs/cols");
  TC_TRY(check_ws(ws, ws_bytes, build_ws_bytes(n, num_pairs), "tc_build_csr"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  prof_stage("build_csr");
  return build_run(n, num_pairs, src, dst, row_offsets, cols, nnz_out, ws, ws_bytes, s);
}

int tc_validate_csr(const tc_csr* g, void* ws, size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_validate_csr"));
  TC_TRY(check_ws(ws, ws_bytes, validate_ws_bytes(g->n, g->nnz), "tc_validate_csr"));
  return validate_run(g, ws, static_cast<hipStream_t>(stream));
}

int tc_bfs_levels(const tc_csr* g, int64_t root, uint32_t flags, int32_t* levels, int32_t* num_levels, void* ws,
                  size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_bfs_levels"));
  if (root >= g->n || root < -1) return fail(TC_ERR_INVALID_ARG, "tc_bfs_levels: root %lld out of range", (long long)root);
  if (g->n > 0 && !levels) return fail(TC_ERR_INVALID_ARG, "tc_bfs_levels: levels is NULL");
  TC_TRY(check_ws(ws, ws_bytes, tc_workspace_bytes(TC_OP_BFS_LEVELS, g->n, g->nnz, 0), "tc_bfs_levels"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  TC_TRY(maybe_validate(g, flags, ws, s));
  Carver c(ws);
  BfsWs w = bfs_reserve(c, g->n);
  prof_stage("bfs");
  return bfs_run(g, root, levels, num_levels, w, s);
}

int tc_cover_edges(const tc_csr* g, const int32_t* levels, int32_t* h_u, int32_t* h_v, int64_t* h_count, void* ws,
                   size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_cover_edges"));
  if (!h_count || (g->n > 0 && !levels) || (g->nnz > 0 && (!h_u || !h_v)))
    return fail(TC_ERR_INVALID_ARG, "tc_cover_edges: NULL argument");
  TC_TRY(check_ws(ws, ws_bytes, plan_cover(nullptr, g->n, g->nnz).bytes, "tc_cover_edges"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  if (g->n == 0) return fill_i64(h_count, 0, 1, s);
  CoverPlan p = plan_cover(ws, g->n, g->nnz);
  prof_stage("split");
  TC_TRY(split_run(g, levels, true, p.split, s));
  prof_stage("hlist");
  return hlist_run(g, p.split.meta, p.split.scols, p.h_off, h_u, h_v, g->nnz / 2, h_count, p.hscratch, s);
}

namespace {

// BFS, relabel and layout, then the count or (list) triangle finding into
// tri[3 * cap].
int cover_call(const tc_csr* g, int64_t root, uint32_t flags, int64_t* triangles, int64_t* h_count, int32_t* levels,
               int64_t* per_vertex, bool list, int32_t* tri, int64_t cap, void* ws, hipStream_t s,
               const CountParams& prm) {
  const bool pv = flags & TC_PER_VERTEX;
  TC_TRY(maybe_validate(g, flags, ws, s));
  CountPlan p = plan_count(ws, g->n, g->nnz);
  int32_t* L = levels ? levels : p.L;
  int32_t nl = 0, d0 = 0;
  prof_stage("bfs");
  TC_TRY(bfs_run(g, root, L, &nl, p.bfs, s, &d0));
  tc_csr rg = *g;  // the relabelled graph
  if (g->n > 0) {
    prof_stage("relabel");
    TC_TRY(relabel_run(g, L, p.comp0, d0, d0 + nl + 1, prm.degree_groups, p.relabel, p.split, s));
    rg.row_offsets = p.relabel.off;
    rg.cols = p.split.scols;
  }
  if (pv) TC_TRY(fill_i64(p.pv_new, 0, g->n, s));
  CountArgs a;
  a.g = &rg;
  a.prm = prm;
  a.cols = p.split.scols;
  a.meta = p.split.meta;
  a.cover = true;
  a.per_vertex = pv;
  a.per_vertex_out = p.pv_new;
  a.order = p.relabel.order;
  if (list) TC_TRY(list_run(a, p.count, tri, cap, triangles, h_count, s));
  else TC_TRY(count_run(a, p.count, triangles, h_count, s));
  if (pv && g->n > 0) {
    pv_back_kernel<<<grid_for(g->n, 256, 16384), 256, 0, s>>>(p.pv_new, p.relabel.order, g->n, per_vertex);
    TC_HIP(hipGetLastError());
  }
  stats_kernel<<<1, 1, 0, s>>>(p.stats, g->n, g->nnz, nl);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace

int tc_count_tuned(const tc_csr* g, int64_t root, uint32_t flags, const tc_tuning* tuning, int64_t* triangles,
                   int64_t* h_count, int32_t* levels, int64_t* per_vertex, void* ws, size_t ws_bytes,
                   tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_count"));
  TC_TRY(check_degree_bound(g, "tc_count"));
  if (!triangles) return fail(TC_ERR_INVALID_ARG, "tc_count: triangles is NULL");
  if (root >= g->n || root < -1) return fail(TC_ERR_INVALID_ARG, "tc_count: root %lld out of range", (long long)root);
  const bool pv = flags & TC_PER_VERTEX;
  if (pv && g->n > 0 && !per_vertex) return fail(TC_ERR_INVALID_ARG, "tc_count: per_vertex is NULL");
  const size_t need = tc_workspace_bytes(TC_OP_COUNT, g->n, g->nnz, 0);
  TC_TRY(check_ws(ws, ws_bytes, need, "tc_count"));
  int64_t small_n = TC_SMALL_MAX_N, small_nnz = TC_SMALL_MAX_NNZ;
  if (tuning) {
    if (tuning->small_max_n) small_n = tuning->small_max_n;
    if (tuning->small_max_nnz) small_nnz = tuning->small_max_nnz;
  }
  CountParams prm;
  TC_TRY(count_params(tuning, true, g->nnz, &prm));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  if (!pv && small_path_fits(g->n, g->nnz, small_n, small_nnz)) {
    TC_TRY(maybe_validate(g, flags, ws, s));
    return small_count_run(g, root, triangles, h_count, levels, ws, ws_bytes, s);
  }
  return cover_call(g, root, flags, triangles, h_count, levels, per_vertex, false, nullptr, 0, ws, s, prm);
}

int tc_count(const tc_csr* g, int64_t root, uint32_t flags, int64_t* triangles, int64_t* h_count, int32_t* levels,
             int64_t* per_vertex, void* ws, size_t ws_bytes, tc_stream_t stream) {
  return tc_count_tuned(g, root, flags, nullptr, triangles, h_count, levels, per_vertex, ws, ws_bytes, stream);
}

int tc_list_triangles(const tc_csr* g, int64_t root, uint32_t flags, int32_t* tri, int64_t cap, int64_t* triangles,
                      int64_t* h_count, int32_t* levels, void* ws, size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_list_triangles"));
  TC_TRY(check_degree_bound(g, "tc_list_triangles"));
  if (!triangles) return fail(TC_ERR_INVALID_ARG, "tc_list_triangles: triangles is NULL");
  if (cap < 0 || (cap > 0 && !tri)) return fail(TC_ERR_INVALID_ARG, "tc_list_triangles: bad output buffer");
  if (flags & TC_PER_VERTEX) return fail(TC_ERR_INVALID_ARG, "tc_list_triangles: TC_PER_VERTEX not supported");
  if (root >= g->n || root < -1)
    return fail(TC_ERR_INVALID_ARG, "tc_list_triangles: root %lld out of range", (long long)root);
  const size_t need = plan_count(nullptr, g->n, g->nnz).bytes;
  TC_TRY(check_ws(ws, ws_bytes, need, "tc_list_triangles"));
  CountParams prm;
  TC_TRY(count_params(nullptr, true, g->nnz, &prm));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  return cover_call(g, root, flags, triangles, h_count, levels, nullptr, true, tri, cap, ws, s, prm);
}

int tc_select_root(const tc_csr* g, int32_t num_candidates, uint32_t flags, int64_t* root_out,
                   int64_t* candidates_out, int64_t* h_out, void* ws, size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_select_root"));
  if (!root_out) return fail(TC_ERR_INVALID_ARG, "tc_select_root: root_out is NULL");
  if (num_candidates < 1 || num_candidates > TC_MAX_ROOT_CANDIDATES)
    return fail(TC_ERR_INVALID_ARG, "tc_select_root: num_candidates %d outside 1..%d", num_candidates,
                TC_MAX_ROOT_CANDIDATES);
  TC_TRY(check_ws(ws, ws_bytes, tc_workspace_bytes(TC_OP_SELECT_ROOT, g->n, g->nnz, 0), "tc_select_root"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  TC_TRY(maybe_validate(g, flags, ws, s));
  if (g->n == 0) {
    *root_out = -1;
    return TC_OK;
  }
  prof_stage("select_root");
  return select_root_run(g, num_candidates, root_out, candidates_out, h_out, ws, s);
}

int tc_edge_support(const tc_csr* g, const int32_t* tri, int64_t num_triangles, int32_t* support,
                    tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_edge_support"));
  if (num_triangles < 0 || (num_triangles > 0 && !tri)) return fail(TC_ERR_INVALID_ARG, "tc_edge_support: bad list");
  if (g->nnz > 0 && !support) return fail(TC_ERR_INVALID_ARG, "tc_edge_support: support is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  prof_stage("support");
  return support_run(g, tri, num_triangles, support, s);
}

int tc_count_edge_baseline(const tc_csr* g, uint32_t flags, int64_t* triangles, void* ws, size_t ws_bytes,
                           tc_stream_t stream) {
  return tc_count_edge_baseline_tuned(g, flags, nullptr, triangles, ws, ws_bytes, stream);
}

int tc_count_edge_baseline_tuned(const tc_csr* g, uint32_t flags, const tc_tuning* tuning, int64_t* triangles,
                                 void* ws, size_t ws_bytes, tc_stream_t stream) {
  TC_TRY(check_csr(g, "tc_count_edge_baseline"));
  TC_TRY(check_degree_bound(g, "tc_count_edge_baseline"));
  if (!triangles) return fail(TC_ERR_INVALID_ARG, "tc_count_edge_baseline: triangles is NULL");
  CountParams prm;
  TC_TRY(count_params(tuning, false, g->nnz, &prm));
  const size_t need = plan_baseline(nullptr, g->n, g->nnz).bytes;
  TC_TRY(check_ws(ws, ws_bytes, need, "tc_count_edge_baseline"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  TC_TRY(maybe_validate(g, flags, ws, s));
  BaselinePlan p = plan_baseline(ws, g->n, g->nnz);
  prof_stage("forward_lists");
  TC_TRY(forward_meta_run(g, p.meta, s));
  if (g->nnz > 0)
    TC_HIP(hipMemcpyAsync(p.cols, g->cols, g->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  CountArgs a;
  a.g = g;
  a.prm = prm;
  a.cols = p.cols;
  a.meta = p.meta;
  a.cover = false;
  a.per_vertex = false;
  a.per_vertex_out = nullptr;
  TC_TRY(count_run(a, p.count, triangles, nullptr, s));
  stats_kernel<<<1, 1, 0, s>>>(p.stats, g->n, g->nnz, 0);
  TC_HIP(hipGetLastError());
  return TC_OK;
}

int tc_count_batch(const tc_batch* b, const tc_tuning* tuning, uint32_t flags, int64_t* triangles,
                   int64_t* h_count, int32_t* levels, void* ws, size_t ws_bytes, tc_stream_t stream) {
  if (!b || !triangles) return fail(TC_ERR_INVALID_ARG, "tc_count_batch: NULL argument");
  if (b->num_graphs < 0 || b->total_vertices < 0 || b->total_nnz < 0)
    return fail(TC_ERR_INVALID_ARG, "tc_count_batch: negative size");
  if (b->max_graph_vertices > TC_BATCH_MAX_N)
    return fail(TC_ERR_TOO_LARGE, "tc_count_batch: a graph has more than %d vertices", TC_BATCH_MAX_N);
  if (b->num_graphs > 0 && (!b->vbase || !b->row_offsets || (b->total_nnz > 0 && !b->cols)))
    return fail(TC_ERR_INVALID_ARG, "tc_count_batch: NULL batch array");
  TC_TRY(check_ws(ws, ws_bytes, batch_ws_bytes(b->total_vertices, b->total_nnz, b->num_graphs), "tc_count_batch"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScope scope(s);
  prof_stage("batch");
  return batch_run(b, tuning, flags, triangles, h_count, levels, ws, ws_bytes, s);
}

const char* tc_status_string(int status) {
  switch (status) {
    case TC_OK: return "ok";
    case TC_ERR_INVALID_ARG: return "invalid argument";
    case TC_ERR_WORKSPACE: return "workspace too small";
    case TC_ERR_NOT_SORTED: return "row not sorted";
    case TC_ERR_DUPLICATE: return "duplicate entry";
    case TC_ERR_SELF_LOOP: return "self loop";
    case TC_ERR_NOT_SYMMETRIC: return "not symmetric";
    case TC_ERR_OUT_OF_RANGE: return "id out of range";
    case TC_ERR_TOO_LARGE: return "too large";
    case TC_ERR_HIP: return "HIP runtime error";
    case TC_ERR_BAD_OFFSETS: return "bad row offsets";
    default: return "unknown status";
  }
}

const char* tc_last_error(void) { return last_error(); }

void tc_profile_enable(int on) { prof_enable(on); }

int tc_profile_read(tc_profile* out) {
  if (!out) return fail(TC_ERR_INVALID_ARG, "tc_profile_read: NULL");
  return prof_read(out);
}

int tc_read_stats(const void* ws, tc_stats* out, tc_stream_t stream) {
  if (!ws || !out) return fail(TC_ERR_INVALID_ARG, "tc_read_stats: NULL");
  memset(out, 0, sizeof *out);
  hipStream_t s = static_cast<hipStream_t>(stream);
  TC_HIP(hipMemcpyAsync(out, ws, sizeof(tc_stats), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  return TC_OK;
}

}  // extern "C"
