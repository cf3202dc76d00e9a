/*
 * tc.h -- C ABI of libtc, exact triangle counting through cover edges on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Bader, Li, Ganeshan, Gundogdu, Lew, Alvarado Rodriguez, Du,
 * "Triangle Counting Through Cover-Edges" (arXiv 2210.00389).
 *   - BFS levels L(v) (Def. 2), one BFS per component in the scan order of
 *     Alg. 1;
 *   - the horizontal edges H = {(u,v) : L(u) = L(v), u < v}, a cover-edge set
 *     (Def. 1, Lemma 1, Thm. 1);
 *   - T = sum over (u,v) in H of |{w in N(u) ∩ N(v) : L(w) != L(u) or w > v}|
 *     (Alg. 1, counting test; exact by Lemma 2 and Thm. 2).
 *
 * Conventions for every entry point:
 *   - Graphs are simple and undirected, in CSR form: row_offsets is int64
 *     [n+1] with row_offsets[0] = 0, cols is int32 [nnz], every row strictly
 *     ascending, no self loops, and (u,v) present iff (v,u) present.  nnz is
 *     twice the edge count m.  Vertex ids are the integers 0..n-1, and "u < v"
 *     in the method is integer order on these ids.
 *   - Pointers marked "device" are HIP device (or managed) memory; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer; the
 *     library allocates and frees no device memory and keeps no state
 *     between calls except the thread-local error text, the profiling
 *     switch, per-device auxiliary streams and events (created on first use,
 *     for table bins run side by side), one small pinned host buffer per
 *     calling thread (the BFS state read back between groups of levels) and
 *     the static device array of tc_count_batch_noalloc.
 *   - `ws` is a caller-provided device workspace of at least
 *     tc_workspace_bytes(op, ...) bytes, 256-byte aligned.  Its contents on
 *     entry are ignored; on return they are scratch.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it in order; device outputs are valid once the stream has been
 *     synchronised.  Entry points that return a value through a host pointer
 *     synchronise the stream themselves, as documented per function.
 *   - Return value: TC_OK (0) or a negative tc_status.  No entry point aborts
 *     or throws; tc_last_error() gives a thread-local description of the last
 *     failure.  Structural checks of the input graph (sorted, duplicate-free,
 *     loop-free, symmetric, ids in range) run only when TC_VALIDATE is set in
 *     `flags` (the check synchronises `stream`); without it a non-simple graph
 *     gives unspecified counts (never an out-of-bounds access as long as ids
 *     are in range and offsets are monotone).
 *   - All counts are exact 64-bit integers; results do not depend on the
 *     scheduling of the GPU or on the tuning parameters.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* tc_stream_t; /* a hipStream_t */

typedef enum tc_status {
  TC_OK = 0,
  TC_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad root, ... */
  TC_ERR_WORKSPACE = -2,     /* ws_bytes smaller than tc_workspace_bytes() */
  TC_ERR_NOT_SORTED = -3,    /* a row is not ascending (TC_VALIDATE) */
  TC_ERR_DUPLICATE = -4,     /* a row repeats an id (TC_VALIDATE) */
  TC_ERR_SELF_LOOP = -5,     /* u in N(u) (TC_VALIDATE) */
  TC_ERR_NOT_SYMMETRIC = -6, /* v in N(u) but u not in N(v) (TC_VALIDATE) */
  TC_ERR_OUT_OF_RANGE = -7,  /* an id outside [0, n) */
  TC_ERR_TOO_LARGE = -8,     /* n or nnz beyond the int32-id / int64 limits, or
                                a degree that could reach 2^29 (counting calls) */
  TC_ERR_HIP = -9,           /* a HIP runtime call failed */
  TC_ERR_BAD_OFFSETS = -10   /* row_offsets not monotone or not from 0 to nnz */
} tc_status;

/* flags */
#define TC_VALIDATE 1u       /* check the CSR structure before counting */
#define TC_PER_VERTEX 2u     /* tc_count: also fill per_vertex */

/* Workspace query operations. */
typedef enum tc_op {
  TC_OP_BUILD_CSR = 1,
  TC_OP_BFS_LEVELS = 2,
  TC_OP_COVER_EDGES = 3,
  TC_OP_COUNT = 4,
  TC_OP_COUNT_BATCH = 5,
  TC_OP_EDGE_BASELINE = 6,
  TC_OP_VALIDATE = 7,
  TC_OP_SELECT_ROOT = 8
} tc_op;

/* A graph in CSR form (all pointers device). */
typedef struct tc_csr {
  int64_t n;                  /* vertices, 0 <= n <= 2^31 - 1 */
  int64_t nnz;                /* directed entries = 2 m */
  const int64_t* row_offsets; /* [n + 1] */
  const int32_t* cols;        /* [nnz] */
} tc_csr;

/* Many independent graphs side by side (all pointers device).  Graph g owns
 * the vertices vbase[g] .. vbase[g+1]-1 of the concatenated vertex range;
 * row_offsets indexes the concatenated cols array; cols hold LOCAL ids
 * (0 .. n_g - 1) of the same graph. */
typedef struct tc_batch {
  int32_t num_graphs;         /* G >= 0 */
  int64_t total_vertices;     /* vbase[G] */
  int64_t total_nnz;          /* row_offsets[total_vertices] */
  const int64_t* vbase;       /* [G + 1], vbase[0] = 0 */
  const int64_t* row_offsets; /* [total_vertices + 1] */
  const int32_t* cols;        /* [total_nnz] */
  int32_t max_graph_vertices; /* max_g n_g (host value, bounds the per-graph
                                 on-chip state); must be <= TC_BATCH_MAX_N */
} tc_batch;

#define TC_BATCH_MAX_N 65536

/* Tuning knobs; a NULL tc_tuning* (or a zero field) means the compiled-in
 * default.  None of them changes a result, only how the work is scheduled.
 * The autotuner of the Python package picks them per batch shape
 * (tc_count_batch) or per graph class (tc_count_tuned). */
typedef struct tc_tuning {
  /* tc_count_batch */
  int32_t batch_block;        /* threads per block of the counting kernel:
                                 64 (one block per piece, not persistent),
                                 256 (default) or 512 */
  int32_t batch_piece;        /* CSR entries per work piece (>= 1024,
                                 default 16384) */
  int32_t batch_blocks_per_cu;/* resident blocks per CU of the persistent
                                 counting kernel (0 = as many as LDS allows) */
  /* tc_count_tuned: which path a graph takes */
  int32_t small_max_n;        /* a graph with 0 < n <= small_max_n and
                                 nnz <= small_max_nnz is levelled and counted
                                 by the batched kernels as a batch of one
                                 (one workgroup, no host synchronisation);
                                 default TC_SMALL_MAX_N, -1 = never; capped
                                 at TC_BATCH_MAX_N */
  int32_t small_max_nnz;      /* default TC_SMALL_MAX_NNZ */
  /* tc_count_tuned and tc_count_edge_baseline_tuned: the intersection stage
   * (every anchor's tasks either merged in registers or streamed against an
   * on-chip table of its probe set) */
  int32_t light_max;          /* anchors with a probe set of at most this many
                                 ids are merged in registers (1..32, default
                                 32) ... */
  int32_t dn_light;           /* ... and, in the cover count, at most this many
                                 down-neighbours (>= 1, default 32) */
  int32_t bitmap_member_words;/* a heavy anchor's table is a bitmap over its
                                 probe set's id window when the bitmap's words
                                 are at most bitmap_member_words * |P| + 64
                                 (default 4) ... */
  int32_t bitmap_desc_words;  /* ... or bitmap_desc_words * its task count
                                 (default 8 for the cover count, 16 for the
                                 comparator); else a hash table (1..1024) */
  int32_t item_log2;          /* work items hold about 2^item_log2 streamed
                                 elements (12..24, default 14 below 2^24
                                 entries, else 19) */
  int32_t bin0_mode;          /* smallest-table bin: 1 = blocks claim items,
                                 2 = items round robin (default 2 for the
                                 cover count below 2^27 entries, else 1) */
  int32_t bins_mode;          /* table bins 1 = one after another, 2 = side by
                                 side on forked streams (default 1 for the
                                 cover count, 2 for the comparator) */
  int32_t twolevel_sparsity;  /* a probe set too large for an LDS bitmap or
                                 hash table gets a two-level table (block bits
                                 in LDS, member words in global memory); one
                                 that would fill the 128 KB hash table gets it
                                 too when its id window is at least this many
                                 times its size (default 64, -1 = never) */
  int32_t bin0_max_desc;      /* an anchor with more task descriptors than
                                 this skips the smallest-table bin (its items
                                 are streamed by one wave each there):
                                 default 1024, -1 = no limit */
  int32_t up_anchor_min;      /* cover count, a pair (x, w) with w one level
                                 below x and Hfwd(x) non-empty: x streams Up(w)
                                 against its table, unless |Up(w)| exceeds both
                                 up_anchor_min and |Hfwd(x)|; then w streams
                                 Hfwd(x) against the Up part of its table
                                 (>= 32; -1 = x always; default 256 for
                                 graphs of at least 2^26 entries, else -1) */
  int32_t degree_groups;      /* cover count: the relabel orders each level by
                                 this many degree groups (2: degree up to 2048,
                                 then the rest; 4: up to 511, 512-2047,
                                 2048-8191, 8192 and above); default 4 for
                                 graphs of at least 2^26 entries, else 2 */
} tc_tuning;

#define TC_SMALL_MAX_N 65536
#define TC_SMALL_MAX_NNZ 262144

/* Bytes of workspace `op` needs for a graph with n vertices and nnz entries
 * (for TC_OP_BUILD_CSR, nnz = number of input pairs; for TC_OP_COUNT_BATCH,
 * n and nnz are the batch totals and num_graphs its graph count).  Returns 0
 * for an unknown op or negative sizes. */
size_t tc_workspace_bytes(int op, int64_t n, int64_t nnz, int32_t num_graphs);

/* Builds a simple undirected CSR from raw pairs (data layout of the input of
 * Sec. III: CSR with both orientations).  Pairs (src[i], dst[i]) with
 * src[i] == dst[i] are dropped; every other pair contributes both (s,d) and
 * (d,s); repeats are merged; rows come out sorted ascending.
 *   n                vertex count (ids must lie in [0, n); else
 *                    TC_ERR_OUT_OF_RANGE)
 *   num_pairs        length of src / dst (device int32)
 *   row_offsets      device int64 [n + 1] (output)
 *   cols             device int32, capacity 2 * num_pairs (output)
 *   nnz_out          host int64 (output); the call synchronises `stream`.
 */
int tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                 int64_t* row_offsets, int32_t* cols, int64_t* nnz_out, void* ws,
                 size_t ws_bytes, tc_stream_t stream);

/* Checks the CSR structure (offsets monotone from 0 to nnz, ids in range,
 * rows strictly ascending, no loops, symmetric).  Returns TC_OK or the first
 * violated property's status.  Synchronises `stream`. */
int tc_validate_csr(const tc_csr* g, void* ws, size_t ws_bytes, tc_stream_t stream);

/* BFS levels as in Alg. 1 (Def. 2): a BFS from `root` (root < 0: the vertex
 * of largest degree, smallest id on ties), then, in increasing id order,
 * one more BFS from every vertex not yet reached, so each further component
 * is levelled from its smallest id.  Isolated vertices get level 0.
 *   levels       device int32 [n] (output)
 *   num_levels   host int32 (nullable): the largest level count of any one
 *                BFS (max level + 1; 0 for n = 0)
 * Synchronises `stream`: the BFS state is read back once per group of up to
 * six levels from the root, and, if vertices with edges are left
 * unreached, once per group of up to four levels of the remaining
 * components. */
int tc_bfs_levels(const tc_csr* g, int64_t root, uint32_t flags, int32_t* levels,
                  int32_t* num_levels, void* ws, size_t ws_bytes, tc_stream_t stream);

/* The horizontal edges of a given level function (Alg. 1, edge selection;
 * Thm. 1): every (u, v) with u < v and levels[u] == levels[v], in
 * lexicographic order.  `levels` may be any int32 array (not only BFS
 * levels).
 *   h_u, h_v     device int32, capacity nnz / 2 each (output)
 *   h_count      device int64 [1] (output): |H|
 * Asynchronous. */
int tc_cover_edges(const tc_csr* g, const int32_t* levels, int32_t* h_u, int32_t* h_v,
                   int64_t* h_count, void* ws, size_t ws_bytes, tc_stream_t stream);

/* Cover-edge triangle count (Alg. 1): levels as in tc_bfs_levels, H, then
 * the count over H with the paper's test.
 *   triangles    device int64 [1] (output): T
 *   h_count      device int64 [1] (nullable output): |H|
 *   levels       device int32 [n] (nullable output): the BFS levels used
 *   per_vertex   device int64 [n] (output iff flags & TC_PER_VERTEX): the
 *                number of triangles through each vertex (sums to 3T)
 * Synchronises `stream` during the BFS as tc_bfs_levels does; the rest
 * (relabelling, layout, count) is asynchronous.  Graphs within the
 * small-graph bounds (TC_SMALL_MAX_N vertices, TC_SMALL_MAX_NNZ entries)
 * take the path of tc_count_tuned, which never synchronises.  A graph in
 * which a vertex could reach degree 2^29 (n - 1 and nnz / 2 both at least
 * 2^29) gives TC_ERR_TOO_LARGE: the count keeps list lengths below 2^29
 * (tc_list_triangles and tc_count_edge_baseline share the limit). */
int tc_count(const tc_csr* g, int64_t root, uint32_t flags, int64_t* triangles,
             int64_t* h_count, int32_t* levels, int64_t* per_vertex, void* ws,
             size_t ws_bytes, tc_stream_t stream);

/* tc_count with tuning knobs (NULL = the defaults of tc_count).  A graph
 * within the small-graph bounds of `tuning` is levelled in one workgroup's
 * LDS and counted by the kernels of tc_count_batch, with no host
 * synchronisation; T, |H| and the levels are the same on either path
 * (TC_PER_VERTEX always takes the general path).  After the small-graph
 * path tc_read_stats reports n, nnz and |H| only. */
int tc_count_tuned(const tc_csr* g, int64_t root, uint32_t flags, const tc_tuning* tuning,
                   int64_t* triangles, int64_t* h_count, int32_t* levels, int64_t* per_vertex,
                   void* ws, size_t ws_bytes, tc_stream_t stream);

/* Triangle finding (the paper counts and finds triangles; Alg. 1 visits each
 * triangle exactly once, at one horizontal edge and one apex): the same
 * levels, H and count as tc_count, then every triangle written once.
 * Two passes: the count records how many triangles each unit of work finds,
 * a prefix sum turns those into output offsets, and a second pass over the
 * same work writes each triangle at its unit's offset.
 *   tri          device int32 [3 * cap] (output): min(T, cap) triangles, each
 *                as its three vertex ids in ascending order; the order of the
 *                triangles is unspecified (it may differ between calls), the
 *                set is exact.  If cap < T, which cap triangles are written
 *                is unspecified: call tc_count first for T, or pass cap >= T.
 *                May be NULL when cap = 0.
 *   cap          capacity of `tri` in triangles (>= 0)
 *   triangles    device int64 [1] (output): T
 *   h_count      device int64 [1] (nullable output): |H|
 *   levels       device int32 [n] (nullable output): the BFS levels used
 * flags: TC_VALIDATE only (TC_PER_VERTEX is rejected).  Workspace: the
 * tc_count size (TC_OP_COUNT).  Synchronises `stream` during the BFS as
 * tc_bfs_levels does and once between the two passes. */
int tc_list_triangles(const tc_csr* g, int64_t root, uint32_t flags, int32_t* tri, int64_t cap,
                      int64_t* triangles, int64_t* h_count, int32_t* levels, void* ws,
                      size_t ws_bytes, tc_stream_t stream);

/* Root choice for a small cover-edge set: the paper's goal is the
 * cover-edge set with the smallest k = |H| / m, and H depends on the BFS
 * root.  The candidates are the num_candidates vertices of largest degree
 * (smallest id first on ties); for each, the levels of tc_bfs_levels with
 * that root are computed and |H| is counted; the candidate with the
 * smallest |H| is returned (the earlier one on ties).  Pass it as `root` to
 * tc_count or tc_list_triangles (T does not depend on the root, Thm. 2).
 *   num_candidates  1 .. TC_MAX_ROOT_CANDIDATES (fewer if n is smaller)
 *   root_out        host int64 (output): the chosen root (-1 if n = 0)
 *   candidates_out  host int64 [num_candidates] (nullable output)
 *   h_out           host int64 [num_candidates] (nullable output): |H| of
 *                   each candidate, in candidate order
 * Workspace: TC_OP_SELECT_ROOT.  Synchronises `stream`. */
#define TC_MAX_ROOT_CANDIDATES 64
int tc_select_root(const tc_csr* g, int32_t num_candidates, uint32_t flags, int64_t* root_out,
                   int64_t* candidates_out, int64_t* h_out, void* ws, size_t ws_bytes,
                   tc_stream_t stream);

/* Triangles per edge (the support of a k-truss decomposition) from a list
 * of triangles such as tc_list_triangles writes: support[e] = number of
 * listed triangles containing the edge of CSR entry e; both orientations of
 * an edge hold the same value.  support is cleared first.  A triple with an
 * id outside [0, n) is skipped; a triple whose pair is not an edge adds
 * nothing for that pair.
 *   tri          device int32 [3 * num_triangles]
 *   support      device int32 [nnz] (output)
 * Asynchronous; needs no workspace. */
int tc_edge_support(const tc_csr* g, const int32_t* tri, int64_t num_triangles, int32_t* support,
                    tc_stream_t stream);

/* Comparator: the plain direction-oriented edge iterator (related-work
 * section: every edge (u, v) with u < v counts the w in N(u) ∩ N(v) with
 * w > v), on the same intersection kernels as tc_count.
 *   triangles    device int64 [1] (output)
 * Asynchronous. */
int tc_count_edge_baseline(const tc_csr* g, uint32_t flags, int64_t* triangles, void* ws,
                           size_t ws_bytes, tc_stream_t stream);
/* The comparator with the intersection-stage knobs of tc_tuning (NULL = the
 * defaults of tc_count_edge_baseline). */
int tc_count_edge_baseline_tuned(const tc_csr* g, uint32_t flags, const tc_tuning* tuning,
                                 int64_t* triangles, void* ws, size_t ws_bytes, tc_stream_t stream);

/* Cover-edge counts of many small graphs in one persistent launch: per graph,
 * the levels of tc_bfs_levels (root = largest degree), H and T.
 *   triangles    device int64 [G] (output); -1 for a graph of more than
 *                TC_BATCH_MAX_N vertices, which is skipped (its levels are
 *                not written)
 *   h_count      device int64 [G] (nullable output); -1 as for triangles
 *   levels       device int32 [total_vertices] (nullable output)
 * flags: TC_VALIDATE checks the batch first -- vbase rising from 0 to
 * total_vertices, every n_g within TC_BATCH_MAX_N (else TC_ERR_TOO_LARGE) and
 * within max_graph_vertices (else TC_ERR_INVALID_ARG), offsets monotone from
 * 0 to total_nnz, and each graph a simple undirected CSR in its local ids
 * (the statuses of tc_validate_csr); the check synchronises `stream`.
 * Without TC_VALIDATE the call issues no host synchronisation (capturable in
 * a hipGraph), and a max_graph_vertices above TC_BATCH_MAX_N is still
 * rejected before any device work. */
int tc_count_batch(const tc_batch* b, const tc_tuning* tuning, uint32_t flags,
                   int64_t* triangles, int64_t* h_count, int32_t* levels, void* ws,
                   size_t ws_bytes, tc_stream_t stream);

/* tc_count_batch for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * results are those of tc_count_batch (same kernels); the scratch that
 * tc_count_batch takes from `ws` lives instead in a static device array of
 * tc_noalloc_scratch_bytes() bytes (32 MiB) that each GPU holds until the
 * process ends.  The call allocates and frees nothing.
 *   - A batch needing more scratch than that (tc_workspace_bytes(
 *     TC_OP_COUNT_BATCH, ...) above the array's size) gives TC_ERR_TOO_LARGE
 *     before any device work; about 1.3 G entries in total fit.
 *   - TC_VALIDATE is not supported (TC_ERR_INVALID_ARG): check a batch with
 *     tc_count_batch first.
 *   - Every call on one GPU shares that GPU's array: calls that overlap on
 *     one GPU (other streams, other threads) race and give unspecified
 *     results; serialise them.  No stream synchronisation is issued. */
int tc_count_batch_noalloc(const tc_batch* b, const tc_tuning* tuning, uint32_t flags,
                           int64_t* triangles, int64_t* h_count, int32_t* levels,
                           tc_stream_t stream);
size_t tc_noalloc_scratch_bytes(void);

/* Text of a status code (static storage). */
const char* tc_status_string(int status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* tc_last_error(void);

/* Profiling: when enabled, every entry point records a HIP event before and
 * after each of its stages on `stream`; tc_profile_read synchronises the
 * stream of the last call and returns, for the calling thread's last call,
 * the number of stages and for each its name and elapsed milliseconds. */
#define TC_PROFILE_MAX_STAGES 32
typedef struct tc_profile {
  int32_t num_stages;
  char names[TC_PROFILE_MAX_STAGES][24];
  float ms[TC_PROFILE_MAX_STAGES];
} tc_profile;

void tc_profile_enable(int on);
int tc_profile_read(tc_profile* out);

/* Work statistics of the calling thread's last tc_count /
 * tc_count_edge_baseline call (read back from the workspace; synchronises
 * `stream`).  Element counts are exact and drive the algorithmic-byte figures
 * of the roofline. */
typedef struct tc_stats {
  int64_t n, nnz;
  int64_t h;               /* |H| (baseline: number of edges u < v) */
  int64_t num_levels;      /* BFS level count (baseline: 0) */
  int64_t stream_elems;    /* list elements streamed by the intersections */
  int64_t light_tasks;     /* tasks on the per-task merge path */
  int64_t heavy_items;     /* work items of the anchored (LDS hash) path */
  int64_t heavy_desc;      /* stream records of heavy anchors (anchored path) */
  int64_t heavy_elems;     /* list elements streamed by the anchored kernel */
  int64_t heavy_builds;    /* probe-set elements inserted into on-chip tables */
  int64_t light_elems;     /* list elements streamed by the per-task merges */
  int64_t bin_elems[4];    /* anchored-kernel elements per table bin (2 KB,
                              32 KB, 128 KB, row search) */
  int64_t bin_items[4];    /* work items per table bin */
  int64_t descriptors;     /* per-vertex task descriptors examined */
  int64_t twolevel_elems;  /* anchored-kernel elements probed in two-level
                              tables (block bits in LDS, member words in
                              global memory; part of bin 2's) */
} tc_stats;

int tc_read_stats(const void* ws, tc_stats* out, tc_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
