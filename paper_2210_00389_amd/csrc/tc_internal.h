// tc_internal.h -- interfaces between the libtc sources.
#pragma once

#include "tc_common.h"

namespace tc {

void clear_error();
const char* last_error();
int prof_read(tc_profile* out);
void prof_enable(int on);

// ---------------------------------------------------------------- BFS
struct BfsWs {
  uint32_t* vis;     // visited bitmap [n/32 + 1]
  uint32_t* bms;     // three rotating frontier bitmaps
  int32_t* big;      // long frontier rows of the current level
  int32_t* parent;   // union-find over the unreached vertices
  int64_t* part;     // per-block (count, entries) of the last step
  char* st;          // device state of the running BFS
  unsigned long long* key;
  int64_t* root;
  uint32_t* comp0;  // optional (caller-owned, n/32+1 words): r0's component
};
BfsWs bfs_reserve(Carver& c, int64_t n);
// *first_levels (nullable) receives the level count of the BFS from r0.
int bfs_run(const tc_csr* g, int64_t root, int32_t* L, int32_t* num_levels, BfsWs& w,
            hipStream_t s, int32_t* first_levels = nullptr);

// Root choice by |H| over the vertices of largest degree (root_select.hip).
constexpr int kMaxRootCandidates = 64;
size_t select_root_ws_bytes(int64_t n);
int select_root_run(const tc_csr* g, int num, int64_t* root_out, int64_t* cand_out, int64_t* h_out, void* ws,
                    hipStream_t s);

// ------------------------------------------------------ radix sort
// LSD radix sort of 64-bit keys on bits [bit_lo, bit_hi), 8 bits per pass,
// stable.  Returns the buffer holding the result (keys or tmp).
size_t radix_ws_bytes(int64_t N);
int radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t N, int bit_lo, int bit_hi, char* scratch,
                   hipStream_t s, uint64_t** result);

// ------------------------------------------------ level-class layout
// Per vertex x, relative to row_offsets[x] in the re-laid-out columns:
//   Up    = [0, up)    neighbours one level closer to the root
//   Same  = [up, sfe)  neighbours on the same level; Hfwd = [hfb, sfe) are
//                      those with a larger id (the cover edges (x, v), x < v)
//   Down  = [sfe, deg) neighbours one level further
// Each class is ascending.  For the comparator the same record describes the
// plain forward lists: up = 0, hfb = first neighbour > x, sfe = deg.
// `begin` repeats row_offsets[x] so that one 32-byte read resolves a vertex.
struct alignas(32) VMeta {
  int64_t begin;
  int32_t up, hfb, sfe, deg;
  int32_t pad[2];
};

struct SplitWs {
  VMeta* meta;
  int32_t* scols;     // re-laid-out columns [nnz]
  uint32_t* res;      // packed 2-bit level residues (L mod 4)
  int32_t* nseg;      // per vertex: segments of a long row
  int64_t* seg_off;   // scan of nseg
  int32_t* seg_vtx;   // segment -> vertex
  int32_t* seg_cnt;   // per segment: six group counts and same-below-x (x7)
  int64_t* seg_pre;   // per segment: output position of each group (x6)
  int64_t* ctr;
  int32_t* rcat;      // per vertex: row category (short, mid, big, segmented)
  int64_t* cat_pre;   // packed scans of the mid (low half) / big (high half) categories
  int64_t* mid_ctx;   // per-row contexts of each category (seven words per row)
  int64_t* big_ctx;
  int32_t* stash;     // output ids of segmented rows, in input order [nnz]
  char* scratch;
};
SplitWs split_reserve(Carver& c, int64_t n, int64_t nnz);
// full_levels: classify by comparing int32 levels (any level function);
// otherwise use packed residues (requires |L(u) - L(v)| <= 1 on edges).
int split_run(const tc_csr* g, const int32_t* L, bool full_levels, SplitWs& w, hipStream_t s);

// Relabelled layout for counting: vertices renumbered by (virtual level,
// degree group, id) where the virtual level is L(v) in r0's component and
// L(v) + D0 elsewhere (D0 = level count from r0).  The method only ever
// compares ids of one (component, level) class, and any total order there
// gives the same cover edges (as a set), T, per-vertex counts and triangle
// set.  Each level becomes a contiguous id range.
struct RelabelWs {
  int32_t* order;     // new id -> old id
  int32_t* perm;      // old id -> new id
  int64_t* off;       // relabelled row offsets [n + 1]
  int32_t* lstart_cnt;  // histogram of (virtual level, degree group) groups
  int64_t* lstart;    // first new id of each group
  uint64_t* keys;
  uint64_t* keys_tmp;
  int32_t* deg;
  char* scratch;
};
RelabelWs relabel_reserve(Carver& c, int64_t n, int64_t max_vlevels);
// Writes the relabelled rows into split.scols and records into split.meta
// (indexed by new ids); fills w.off, w.order, w.perm.
// degree_groups: 2 or 4 degree groups per level (see tc_tuning).
int relabel_run(const tc_csr* g, const int32_t* L, const uint32_t* comp0, int32_t d0, int32_t max_vl,
                int degree_groups, RelabelWs& w, SplitWs& sp, hipStream_t s);

// Explicit horizontal-edge list from the layout: h_off = scan of
// (sfe - hfb), then (x, scols[..]) for every cover edge, lexicographic.
// At most `cap` entries are written (the caller's capacity); h_off[n] and
// *h_count report the full count.
int hlist_run(const tc_csr* g, const VMeta* meta, const int32_t* cols, int64_t* h_off,
              int32_t* h_u, int32_t* h_v, int64_t cap, int64_t* h_count, char* scratch,
              hipStream_t s);

// ------------------------------------------------------------ count
// Column buffers handed to count_run hold at least this many readable
// entries past nnz (the streaming kernel loads whole chunks).
constexpr int kColPad = 64;

struct CountWs {
  int32_t* ndesc;      // per vertex: descriptors [n + 1]
  uint8_t* vinfo;      // per vertex: heavy flag, table bin and kind
  int64_t* so;         // exclusive scan of ndesc [n + 1]
  // stream records of heavy anchors (compacted) and their work items
  int64_t* sbeg;       // [rcap]
  int32_t* slen;       // length | flags
  int32_t* soth;       // the vertex whose list is streamed
  int32_t* sx;         // light tasks: the anchor
  int4* items_raw;     // (anchor, first record lo/hi, count | bin | kind) [rcap]
  int4* items;         // the same grouped by bin [rcap]
  int32_t* cx0;        // first vertex of every descriptor chunk
  int4* ccnt;          // per chunk: heavy records, light tasks, items
  int64_t* lpre;       // scan of the per-chunk light task counts
  int32_t* samp;       // every 32nd layout column, for the searches of the resolution
  uint4* pm;           // per vertex: the record fields the resolution reads of a neighbour, in 16 bytes [n + 1]
  uint32_t* tl_words;  // member words of two-level anchors, at their rows' positions [nnz + 1]
  uint32_t* tl_l1;     // LDS part (block bits, prefix counts) of two-level tables, likewise [nnz + 1]
  int64_t nchunk_cap;
  int64_t rcap;
  unsigned long long* acc;
  int64_t* stats;      // tc_stats mirror
  char* scratch;
};
CountWs count_reserve(Carver& c, int64_t n, int64_t nnz);

// Scheduling choices of the count (none changes a result): see tc_tuning.
struct CountParams {
  int light_max;   // anchors with a probe set of at most this many ids are light (<= 32)
  int dn_light;    // ... and (cover count) at most this many down-neighbours
  int bm_member;   // bitmap table when its words <= bm_member * |P| + 64 ...
  int bm_desc;     // ... or <= bm_desc * (descriptors of the anchor); else hash
  int item_log2;   // work items hold about 2^item_log2 streamed elements
  int bin0_mode;   // 1: blocks claim items; 2: items round robin
  int bins_mode;   // 1: table bins one after another; 2: side by side
  int tl_sparsity; // largest hash bin: two-level table instead when window >= this * |P| (-1: never)
  int bin0_max_desc; // anchors with more descriptors skip the smallest-table bin (-1: no limit)
  int up_anchor_min; // down-class pair (x, w): w anchors it when |Up(w)| > this and > |Hfwd(x)| (-1: never)
  int degree_groups; // cover count: degree groups per level of the relabel (2 or 4)
};
// The defaults, overridden by the non-zero fields of `t` (nullable);
// TC_ERR_INVALID_ARG for a value out of range.
int count_params(const tc_tuning* t, bool cover, int64_t nnz, CountParams* out);

struct CountArgs {
  const tc_csr* g;
  CountParams prm;
  const int32_t* cols;  // layout columns [nnz + kColPad] (cover: split; comparator: copy)
  const VMeta* meta;
  bool cover;           // cover edges (three classes) or the comparator
  bool per_vertex;
  int64_t* per_vertex_out;
  const int32_t* order = nullptr;  // layout id -> caller id (cover layout)
  bool record_units = false;       // first pass of triangle finding
};
int count_run(const CountArgs& a, CountWs& w, int64_t* triangles, int64_t* h_count,
              hipStream_t s);
// Triangle finding (cover layout): count_run recording per-unit counts, a
// scan, and a second pass writing min(T, cap) triangles to tri[3 * cap] as
// ascending caller ids.  Synchronises the stream once (unit count).
int list_run(const CountArgs& a, CountWs& w, int32_t* tri, int64_t cap, int64_t* triangles, int64_t* h_count,
             hipStream_t s);
// Triangles per edge from a triangle list: support[e] for both CSR entries
// of each of the three edges of every listed triangle (cleared first).
int support_run(const tc_csr* g, const int32_t* tri, int64_t ntri, int32_t* support, hipStream_t s);

// Comparator layout: meta with up = 0, hfb = first neighbour > x, sfe = deg.
int forward_meta_run(const tc_csr* g, VMeta* meta, hipStream_t s);

// -------------------------------------------------------- CSR build
size_t build_ws_bytes(int64_t n, int64_t num_pairs);
int build_run(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
              int64_t* row_offsets, int32_t* cols, int64_t* nnz_out, void* ws, size_t ws_bytes,
              hipStream_t s);

size_t validate_ws_bytes(int64_t n, int64_t nnz);
int validate_run(const tc_csr* g, void* ws, hipStream_t s);
// Structure of a batch: vertex bases from 0 to total_vertices, every graph
// within TC_BATCH_MAX_N and max_graph_vertices, offsets monotone, and each
// graph a simple undirected CSR in its local ids.  Uses the first 256 bytes
// of ws; synchronises `s`.
int validate_batch_run(const tc_batch* b, void* ws, hipStream_t s);

// ------------------------------------------------------------ batch
// piece_min: the smallest work piece (CSR entries) the call may use; it
// sizes the piece slots of the workspace.
size_t batch_ws_bytes(int64_t total_n, int64_t total_nnz, int32_t num_graphs, int piece_min = 1024);
// root0 >= 0 replaces the default root of graph 0 (batches pass -1).
int batch_run(const tc_batch* b, const tc_tuning* t, uint32_t flags, int64_t* triangles,
              int64_t* h_count, int32_t* levels, void* ws, size_t ws_bytes, hipStream_t s,
              int32_t root0 = -1, int piece_min = 1024);

// One graph of at most TC_BATCH_MAX_N vertices counted by the batched
// kernels (one workgroup levels it in LDS, no host synchronisation): T,
// |H| and the levels of tc_count; stats carries n, nnz and |H| only.
size_t small_ws_bytes(int64_t n, int64_t nnz);
bool small_path_fits(int64_t n, int64_t nnz, int64_t max_n, int64_t max_nnz);
int small_count_run(const tc_csr* g, int64_t root, int64_t* triangles, int64_t* h_count, int32_t* levels,
                    void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace tc
