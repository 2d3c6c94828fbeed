// Internal definitions shared by the host API layer and the HIP kernels.
#pragma once

#include <atomic>
#include <cstddef>
#include <cstdint>

#include "../../include/grb.h"

namespace grb {

// ---- kernel geometry -------------------------------------------------
constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kPushTile = 1024;      // merge-path items (entries + edges) per push tile
constexpr int kCompactThreads = 1024;  // threads per compaction workgroup (16 waves)
constexpr int kCompactWords = 256;     // bitmap words per compaction workgroup
constexpr int kHeavyDeg = 2048;      // rows longer than this are split for pull
constexpr int kHeavyChunk = 1024;    // edges per split piece of a long row
constexpr int kExpandGrid = 1024;    // workgroups of the grid-stride expand kernels (4 per CU: all
                                     // resident at once, so a small level pays one dispatch round)
constexpr int kPushSplit = 256;      // BFS push: rows longer than this are cut in pieces of this size
constexpr int kSweepGrid = 4096;     // workgroups of the PageRank sweep (two rounds of 8 waves per SIMD)
constexpr int kWaveParts = kSweepGrid * kWavesPerBlock;  // balanced word runs of full sweeps
constexpr int kSweepUnroll = 4;      // PageRank: 64-position steps whose loads are issued together
constexpr int kUnroll = 4;         // 64-edge steps whose loads are issued together
constexpr int kMsMaxWordsPerPass = 8;  // batched BFS: query words (of 64) per pass, at most
constexpr int kPullRows = 4;       // BFS pull: rows per lane whose first loads overlap
constexpr int kCntStripes = 32;      // BFS: striped frontier counters (count, degree sum)
constexpr int kStatsCap = GRB_STATS_MAX;

// ---- matrix ----------------------------------------------------------
struct Csr {
  const int32_t *rp = nullptr;  // row_ptr[nrows + 1]
  const int32_t *ci = nullptr;  // col_idx[nnz]
  const void *val = nullptr;    // values[nnz] or nullptr (structure only)
  int vtype = -1;               // grb_type of val, -1 when val is null
  int64_t nrows = 0;
  int64_t ncols = 0;
  int64_t nnz = 0;
  // metadata from grb_matrix_prepare
  const int32_t *heavy = nullptr;      // split pieces: (row, begin) pairs
  int64_t nheavy = 0;                  // number of pieces
  const int32_t *heavy_rows = nullptr; // (row, first piece, piece count) triples
  int64_t nheavy_rows = 0;
  const int32_t *split = nullptr;      // (row, begin) pieces of rows longer than kPushSplit
  int64_t nsplit = 0;
  const int32_t *split_rows = nullptr; // (row, first piece, piece count) triples
  int64_t nsplit_rows = 0;
  // bitmap words cut into kWaveParts contiguous runs of about equal work
  // (edges of rows up to kPushSplit long plus a fixed cost per word), for
  // kernels that sweep every row: run p is words [wpart[p], wpart[p + 1])
  const int32_t *wpart = nullptr;
  // rows without entries (and the padding bits past nrows), one bit each
  const uint64_t *iso = nullptr;
  // first two column ids of every row (-1 where the row is shorter), read
  // with the row extents so that a pull settled by them never touches col_idx
  const int2 *first2 = nullptr;
  int64_t max_deg = 0;  // longest row (host copy, from prepare)
  bool negative = false;  // a stored value is negative or NaN (from prepare)
  bool valid() const { return rp != nullptr; }
};

}  // namespace grb

struct grb_matrix_s {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  grb::Csr a;   // CSR of A
  grb::Csr at;  // CSR of A^T (aliases a for symmetric matrices)
  bool symmetric = false;
  bool prepared = false;
  // levels of the last BFS on this matrix: a hint for how many level
  // launches to queue before the first read-back (speed only)
  std::atomic<int32_t> bfs_depth{0};
};

struct grb_vector_s {
  int64_t n = 0;
  grb_type type = GRB_BOOL;
  void *values = nullptr;      // n elements by index, or null (every entry is 1)
  uint64_t *bitmap = nullptr;  // presence words, or null
  int32_t *indices = nullptr;  // sorted present indices (capacity n), or null
  int32_t *count = nullptr;    // device int32: entries in `indices`
};

namespace grb {

// ---- device-side control block ------------------------------------------
struct Ctrl {
  int32_t count;    // entries in the current frontier list
  int32_t sumdeg;   // sum of their degrees in the push matrix
  int32_t ntiles;   // merge-path tiles for push
  int32_t ticket;   // compaction workgroup ticket counter
  int32_t nlev;     // levels (BFS) / rounds (SSSP) with a non-empty frontier
  int32_t dir;      // direction chosen by the last expand
  int32_t iters;    // PageRank iterations run
  int32_t converged;
  double D;         // PageRank: dangling mass of the current iterate
  double delta;     // PageRank: L1 change of the last iteration
  int32_t lists[3 * 5 * 32];  // BFS / SSSP: striped counters of the three frontier buffers
  int32_t bucket;             // bucketed SSSP: the bucket of the last round
  int32_t pushed[3];          // BFS: buffer's frontier came from a push of > 1 vertex
                              // (its vertices' parents are still open)
  double Dfz;                 // adaptive PageRank: dangling mass of the frozen vertices
  int64_t active;             // adaptive PageRank: vertices still active
  int32_t ticket_list;        // generic product: list preparation workgroup tickets
  int32_t error;              // batched BFS: a source id was out of range
  int32_t small_levels;       // BFS / SSSP: levels or rounds run by the multi-workgroup loop
  int32_t spilled;            // ... which then handed a frontier to the wide kernels
  int32_t pushed_sd[3];       // BFS: degree sum of the push that found the buffer's frontier
  int32_t pad32;
  int64_t pad[2];
};

// stats record per iteration: {frontier, sumdeg, direction, unused}
constexpr int kStatFields = 4;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline int64_t words_of(int64_t n) { return (n + 63) / 64; }

// While alive on a host thread, the library's read-backs use no pinned
// staging buffer they would have to allocate (plain copies instead).
class NoAllocScope {
 public:
  NoAllocScope();
  ~NoAllocScope();
  NoAllocScope(const NoAllocScope &) = delete;
  NoAllocScope &operator=(const NoAllocScope &) = delete;

 private:
  bool prev_;
};

// ---- direction of a generic product ----------------------------------------
// The automatic choice is taken on the device from the input's entry count
// and degree sum, which the product's first kernel leaves as per-workgroup
// partials (kMxvParts (count, degree sum) pairs); every later kernel of the
// product evaluates the rule itself, so no kernel waits on the host.
constexpr int kMxvParts = 256;     // workgroups of the generic product's first kernel
constexpr int kMxvPartThreads = 1024;
constexpr int kMxvListChunk = 4096;  // list entries per workgroup of the list preparation
struct DirGate {
  const int64_t *part = nullptr;  // 2 * kMxvParts partials (unused when forced)
  // the choice, left by the first kernel of the product that evaluated the
  // rule (0 until then; cleared by the first kernel), so that later kernels
  // read one word instead of the partials
  int32_t *decided = nullptr;
  int forced = 0;                 // grb_direction: 0 = automatic
  bool can_push = true, can_pull = true;
  int rule = 0, denom = 10;
  int64_t nnz = 0, n_in = 0;
};

// ---- kernel launch interfaces (implemented in grb_kernels.hip) -------------
struct CompactArgs {
  const uint64_t *nb = nullptr;  // bitmap to compact
  int64_t nw = 0;
  const int32_t *rp = nullptr;   // degrees come from this row_ptr (may be null)
  int32_t *list = nullptr;
  int32_t *degpre = nullptr;
  int32_t *rowstart = nullptr;   // row start (in rp) of each list entry
  int32_t *tiles = nullptr;
  uint64_t *status_cur = nullptr;
  uint64_t *status_next = nullptr;
  Ctrl *ctrl = nullptr;
  uint64_t *clear = nullptr;     // optional: bitmap zeroed word by word
  bool skip_if_empty = false;    // return at once when ctrl->count == 0
  bool gated = false;            // return at once unless `gate` picks push
  DirGate gate;
  int32_t *count_out = nullptr;  // optional: the list's length is also stored here
  int64_t nbits = 0;             // bits of the bitmap that count (0 = all nw * 64)
  // optional: every block's (entries, degree sum), computed by an earlier
  // kernel; the blocks' offsets then come from their prefix, with no look-back
  const int64_t *blk_part = nullptr;
};
int compact_blocks(int64_t nw);
void launch_compact(const CompactArgs &a, void *stream);

// Multi-workgroup level loop (high-diameter, low-degree graphs): a small grid
// of workgroups runs BFS levels (SSSP bucket rounds) back to back, separated
// by a barrier of its own (one arrival per workgroup on a shared counter,
// then a bounded wait), with the frontier as a queue in device memory.
// Everything one workgroup hands to another goes through device-coherent
// (agent-scope) atomics, loads and stores, so no L2 write-back is needed.
// State shared by the loop's workgroups:
constexpr int kCoopThreads = 256;
// workgroups of the loop: BFS levels carry few entries (the 3000 x 3000
// grid's frontier holds at most 3,000 vertices), bucket rounds more (a
// pending set of up to ~8,000 there), and a barrier costs more the more
// workgroups arrive (measured: 0.85 us for 16, 1.0 for 32)
constexpr int kCoopGridBfs = 16;
constexpr int kCoopGridSssp = 32;
constexpr int kCoopSegsMax = kCoopGridSssp * (kCoopThreads / 64);  // one queue segment per wave
constexpr int kCoopSeg = 256;          // queue entries per wave and level (more: spill)
constexpr int kCoopEdges = 65536;      // a frontier with more edges goes to the level kernel
// Each level's queue has one segment per wave of the loop; the wave that
// found the entries stores their count and degree sum (slot d & 1 for the
// frontier of level d).
struct CoopCtl {
  unsigned long long bar;  // arrivals (low 32 bits) | 1 + the barrier given up (high 32 bits)
  int32_t cnt[2][kCoopSegsMax];   // entries queued
  int32_t esum[2][kCoopSegsMax];  // BFS: their degree sum; bucketed SSSP: that of the near ones
  int32_t near[2][kCoopSegsMax];  // bucketed SSSP: entries below the round's limit
  int32_t far[2][kCoopSegsMax];   // bucketed SSSP: smallest bucket of the others (INT_MAX: none)
};
constexpr int64_t kCoopMaxLevels = int64_t(1) << 24;  // arrivals stay below 2^32
// A barrier not completed after this many ticks of the 100 MHz real-time
// clock (1 ms: a level of the loop takes microseconds) is given up; the
// frontier then continues with the level kernel.  Nothing waits unboundedly,
// also when some of the loop's workgroups are not resident.
constexpr uint64_t kCoopWaitTicks = 100000;

// BFS with one kernel per level (grb_bfs.hip).  Each of the three rotating
// frontier buffers has kCntStripes (count, degree sum) counter pairs.
// per stripe: frontier size, its degree sum, its rows longer than kPushSplit
constexpr int kCntFields = 3;
constexpr int kCntSlots = kCntFields * kCntStripes;
struct BfsArgs {
  int64_t n = 0, nw = 0, nnz = 0;
  Csr push;   // out-edges (CSR of A)
  Csr pull;   // in-edges (CSR of A^T)
  bool can_pull = true;
  bool same_csr = false;  // symmetric matrix: push and pull read one CSR
  uint64_t *visited = nullptr;
  uint64_t *fcur = nullptr, *fnxt = nullptr, *fclr = nullptr;
  int32_t *levels = nullptr, *parents = nullptr;
  int32_t *cnt_cur = nullptr, *cnt_nxt = nullptr, *cnt_clr = nullptr;
  Ctrl *ctrl = nullptr;
  int64_t *stats = nullptr;
  int32_t d = 0;
  int32_t rule = 0, denom = 10, forced = 0;
  // multi-workgroup loop: shared state and the two level queues (entries:
  // vertex, and row start | degree << 32; queue d & 1 at offset (d & 1) *
  // kCoopSegsMax * qseg, segment s of a queue at s * qseg)
  CoopCtl *coop = nullptr;
  int32_t *qv = nullptr;
  uint64_t *qe = nullptr;
  int32_t qseg = 0;
};
void launch_bfs_start(const BfsArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                      void *stream);
void launch_bfs_level(const BfsArgs &a, void *stream);
constexpr int kCoopMaxDeg = 64;  // graphs whose rows are at most this long use the loop
// BFS levels in kCoopGridBfs workgroups while the frontier fits the queues
// (kCoopSeg vertices per wave, kCoopEdges edges) and pushes; starts at level 0 after
// launch_bfs_start (which fills the first queue), then a hand-over kernel
// leaves a frontier that outgrew the loop (or a given-up barrier's next
// frontier) as the bitmap and counters of level ctrl->small_levels.
// Parents are left to the parents pass.
void launch_bfs_coop(const BfsArgs &a, int32_t source, int64_t max_levels, uint64_t *const F[3],
                     uint64_t wait_ticks, void *stream);
void launch_bfs_parents(const BfsArgs &a, void *stream);

// SSSP with one kernel per round (grb_sssp.hip); counters as BFS
struct SsspArgs {
  int64_t n = 0, nw = 0, nnz = 0;
  Csr push, pull;
  bool can_pull = true;
  bool same_csr = false;
  const float *wpush = nullptr, *wpull = nullptr;
  float *dist = nullptr;
  uint64_t *iso = nullptr;  // rows without in-edges (never improve in pull)
  uint64_t *fcur = nullptr, *fnxt = nullptr, *fclr = nullptr;
  // frontier distances: dist of the buffer's frontier vertices, +inf
  // elsewhere (the improved value of each vertex, for the next round)
  float *fd_cur = nullptr, *fd_nxt = nullptr, *fd_clr = nullptr;
  float delta = 0.0f;  // bucketed rounds: bucket width
  int32_t *cnt_cur = nullptr, *cnt_nxt = nullptr, *cnt_clr = nullptr;
  Ctrl *ctrl = nullptr;
  int64_t *stats = nullptr;
  int32_t d = 0;
  int32_t rule = 0, denom = 10, forced = 0;
  // bucketed rounds in the multi-workgroup loop: as BfsArgs
  CoopCtl *coop = nullptr;
  int32_t *qv = nullptr;
  uint64_t *qe = nullptr;
  int32_t qseg = 0;
};
void launch_sssp_start(const SsspArgs &a, int32_t source, uint64_t *f1, uint64_t *f2, float *fd1,
                       float *fd2, void *stream);
void launch_sssp_round(const SsspArgs &a, void *stream);

// Bucketed SSSP (near-far rounds, push only): per stripe the next round's
// near count, its degree sum, its rows with pieces, the smallest far bucket
// and the pending count
constexpr int kDeltaFields = 5;
constexpr int kDeltaSlots = kDeltaFields * kCntStripes;
void launch_sssp_delta_start(const SsspArgs &a, int32_t source, uint64_t *f1, uint64_t *f2,
                             void *stream);
void launch_sssp_delta_round(const SsspArgs &a, void *stream);
// bucket rounds in the multi-workgroup loop (kCoopGridSssp workgroups, the BFS
// loop's queues and limits), then a hand-over kernel that leaves a pending
// set that outgrew it (or a given-up barrier's next set) as the bitmap and
// counters of round ctrl->small_levels for the round kernel
void launch_sssp_delta_coop(const SsspArgs &a, int64_t max_rounds, uint64_t *const F[3],
                            uint64_t wait_ticks, void *stream);

struct PrArgs {
  int64_t n = 0, nw = 0;
  Csr pull;                    // CSR of A^T (in-edges)
  const int32_t *out_rp = nullptr;  // CSR row_ptr of A (out-degrees)
  void *p = nullptr;           // ranks (in place)
  const void *x = nullptr;     // p / outdeg of the current iterate
  void *xn = nullptr;          // next x
  void *heavy_part = nullptr;  // partial sums of the pieces of long rows
  double *blk_part = nullptr;  // per workgroup partials, kPrFields each
  int nblk = 0;                // workgroups of the SpMV kernel (kExpandGrid)
  int nblk_long = 0;           // workgroups of the long-row kernel
  Ctrl *ctrl = nullptr;
  int64_t *stats = nullptr;    // adaptive: per-iteration {active rows, their in-edges, pull}
  double alpha = 0.85;
  double tol = 0.0;
  // adaptive PageRank: bit v of act_cur = vertex v still updated in this
  // iteration, act_prev = in the previous one, act_nxt = in the next one
  // (written here); nullptr for plain PageRank
  uint64_t *act_cur = nullptr, *act_prev = nullptr, *act_nxt = nullptr;
  double eps = 0.0;  // freeze when |p' - p| <= eps * p
};
// per-workgroup partials of a PageRank iteration: L1 change, dangling mass
// of the updated vertices, dangling mass of the vertices frozen now,
// vertices active after the iteration, vertices and in-edges updated
constexpr int kPrFields = 6;
int pr_long_grid(int64_t nsplit_rows);  // workgroups of the long-row kernel
void launch_pr_init(int is_fp64, const PrArgs &a, void *stream);
void launch_pr_iter(int is_fp64, const PrArgs &a, void *stream);  // adaptive iff a.act_cur

// masked SpGEMM in the dot-product form, C = (A B^T) .* M (grb_mxm.hip)
constexpr int kMxmLds = 1024;  // entries of a row of A a wave keeps in LDS
constexpr size_t kMxmWs = 256; // workspace: the triangle counter
constexpr int kPairBits = 1 << 16;  // structure-only product: LDS bitmap columns per wave
constexpr int kPairTail = 256;      // ... and LDS entries of a row's part above them
constexpr int kPairLong = 128;      // rows of B streamed one at a time from this length
constexpr int kPairUnroll = 8;      // ... 64 x kPairUnroll entries per step
struct MxmArgs {
  int64_t nrows = 0;  // rows of M (and of A)
  Csr M, A, B;        // B is given by its rows (the columns of B^T)
  void *c = nullptr;  // nnz(M) results in M's entry order (write mode)
  unsigned long long *count = nullptr;  // count mode: the sum of all results
  int vt = 0;         // GRB_FP32 / GRB_FP64 (PLUS_TIMES), else PLUS_PAIR
};
void launch_mxm_dot(const MxmArgs &a, bool count, void *stream);

// generic helpers
void launch_first_two(const int32_t *rp, const int32_t *ci, int64_t nrows, int2 *out,
                      void *stream);
void launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, void *stream);
void launch_fill_bytes_pattern(void *p, int64_t count, int elem_size, const void *value,
                               void *stream);
void launch_popcount(const uint64_t *bm, int64_t nw, int64_t *out, void *stream);
// *flag (cleared first) = 1 if some value is negative or NaN (fp32 / fp64)
void launch_any_negative(const void *values, int vtype, int64_t n, int32_t *flag, void *stream);
void launch_vector_build(uint64_t *bitmap, void *values, int elem_size, int64_t n,
                         const int32_t *idx, const void *vals, int64_t count, uint64_t one,
                         void *stream);

// batched multi-source BFS (grb_msbfs.hip)
struct MsbfsArgs {
  int64_t n = 0, nw = 0, nnz = 0, k = 0;
  int W = 0;            // query words per vertex (k / 64 rounded up)
  int kt = 1;           // query words per pass (tile width)
  Csr push, pull;
  bool can_pull = true;
  int32_t *levels = nullptr;  // n x k, vertex-major
  uint64_t *V = nullptr;      // visited, n x W
  uint64_t *F = nullptr, *Fn = nullptr, *Fc = nullptr;      // frontier blocks
  uint64_t *act = nullptr, *actn = nullptr, *actc = nullptr;  // vertex has a frontier bit
  unsigned long long *cnt_cur = nullptr, *cnt_nxt = nullptr, *cnt_clr = nullptr, *cnt_base = nullptr;
  Ctrl *ctrl = nullptr;
  int64_t *stats = nullptr;
  int32_t d = 0;
  int32_t rule = 0, denom = 10, forced = 0;
  // continuous batching (sessions): per-query start level (discoveries at
  // level d are written as d + 1 - start[q]) and per-query-word "has a
  // frontier bit" words of the next level (cleared two levels ahead)
  const int32_t *start = nullptr;
  unsigned long long *alive_nxt = nullptr, *alive_clr = nullptr;
};
void launch_msbfs_start(const MsbfsArgs &a, const int32_t *sources, uint64_t *F1, uint64_t *F2,
                        uint64_t *act1, uint64_t *act2, void *stream);
void launch_msbfs_level(const MsbfsArgs &a, int grid_x, void *stream);
// sessions: every query idle (its bits set in V), blocks and counters cleared
void launch_msbfs_session_init(const MsbfsArgs &a, uint64_t *F1, uint64_t *F2, uint64_t *act1,
                               uint64_t *act2, unsigned long long *alive3, void *stream);
// sessions: queries lanes[i] start from sources[i] at level a.d (device
// arrays of `count` entries; clr[W] holds the joining queries' bits per word)
void launch_msbfs_session_join(const MsbfsArgs &a, const int32_t *lanes, const int32_t *sources,
                               int32_t count, const uint64_t *clr, int32_t *start,
                               unsigned long long *alive_cur, void *stream);
// sessions: out[i * n + v] = level of query lanes[i] at v, -1 where unvisited
void launch_msbfs_session_extract(const MsbfsArgs &a, const int32_t *lanes, int32_t count,
                                  int32_t *out, void *stream);

// connected components (grb_cc.hip): FastSV vectors in the workspace
struct CcArgs {
  int64_t n = 0, nw = 0;
  int32_t *f = nullptr, *f_old = nullptr, *gf = nullptr, *mngf = nullptr, *labels = nullptr;
  uint64_t *gf_bm = nullptr, *mngf_bm = nullptr;
  int64_t *changed = nullptr;  // per iteration: vertices whose grandparent changed
};
void launch_cc_init(const CcArgs &a, void *stream);
void launch_cc_step(const CcArgs &a, int32_t it, void *stream);  // hooking .. grandparents
void launch_cc_out(const CcArgs &a, void *stream);

// generic masked products (grb_mxv.hip)
struct MxvArgs {
  int64_t n_out = 0, n_in = 0, nw_out = 0, nw_in = 0, nnz = 0;
  Csr push;   // rows = input indices (CSR of A'^T)
  Csr pull;   // rows = output indices (CSR of A')
  bool can_push = true, can_pull = true;
  int semiring = 0;        // grb_semiring
  int accum = 0;           // grb_binop
  bool pick_vec = false;   // MIN_FIRST / MIN_SECOND: the product is the vector operand
  bool has_mask = false, mask_comp = false, mask_struct = false, replace = false;
  // operands
  const void *u_val = nullptr;
  const uint64_t *u_bm = nullptr;
  void *w_val = nullptr;
  uint64_t *w_bm = nullptr;
  const void *m_val = nullptr;
  const uint64_t *m_bm = nullptr;
  int m_type = 0;
  // sparse (list) forms: sorted present indices and their device-side count
  const int32_t *u_list = nullptr, *u_cnt = nullptr;  // input given as a list
  bool u_from_list = false;     // u_bm is built from u_list (the vector has no bitmap)
  const int32_t *m_list = nullptr, *m_cnt = nullptr;  // mask given only as a list
  int32_t *w_list = nullptr, *w_cnt = nullptr;        // output list to refresh
  const int32_t *w_list_in = nullptr, *w_cnt_in = nullptr;  // output given only as a list
  // workspace
  void *t_val = nullptr;
  uint64_t *t_bm = nullptr, *t_vb = nullptr;
  void *hp_val = nullptr;       // per pull piece partial value
  uint8_t *hp_has = nullptr;    // per pull piece: any contribution
  uint8_t *settled = nullptr;   // OR pull: long row settled by its first two entries (by row)
  int32_t *list = nullptr, *degpre = nullptr, *rowstart = nullptr, *tiles = nullptr;
  int64_t tiles_cap = 0;        // entries of `tiles`
  uint64_t *status = nullptr, *status_out = nullptr, *status_list = nullptr;
  int nblk = 0, nblk_out = 0, nblk_list = 0;
  int64_t *part = nullptr;      // direction partials of the first kernel
  // per compaction block of a bitmap input (nblk of them): entries and their
  // degree sum, left by the first kernel when the product may push
  int64_t *blk_part = nullptr;
  Ctrl *ctrl = nullptr;
  DirGate gate;
};
void launch_mxv(const MxvArgs &a, void *stream);

// vectors: sorted list (capacity n) -> presence bitmap (every word written);
// with a gate, only when the product pulls
void launch_list_to_bitmap(const int32_t *list, const int32_t *cnt, int64_t n, uint64_t *bm,
                           void *stream, const DirGate *gate = nullptr);
// vectors: presence bitmap of n bits -> sorted list and count, one workgroup
// (no workspace)
void launch_bitmap_to_list_small(const uint64_t *bm, int64_t n, int32_t *list, int32_t *cnt,
                                 void *stream);
// vectors: list entries 0..n-1 and count n
void launch_iota(int32_t *list, int64_t n, int32_t *cnt, void *stream);
// vectors: out[k] = values[list[k]] for k < *cnt (elem_size bytes per value)
void launch_gather_values(const void *values, int elem_size, const int32_t *list,
                          const int32_t *cnt, int64_t cap, void *out, void *stream);

}  // namespace grb
