// kernels.h -- internal interfaces between the library's translation units.
#pragma once
#include <mutex>

#include "common.h"

namespace rsb {

// The fixed device region of rsb_partition_noalloc on one GPU: its device
// address (looked up once per device), size, and the lock and free list of
// the calls that use it.
struct NoallocRegion {
  void *ptr = nullptr;
  size_t bytes = 0;
  hipError_t err = hipSuccess;
  std::mutex mu;
  Arena arena;
};
// Makes `device` current and returns its region (RSB_EDEVICE if the lookup fails).
NoallocRegion &noalloc_region(int device);

// Reference measurements (probe.hip).  hbm_probe_gbs: GB/s of a plain
// stream over `bytes` (kind 0 read, 1 copy counting both directions, 2
// write), average of `reps` launches after a warm-up.  spmv_alone_us:
// average time of y = L x alone on a level's sliced ELL (0 for the
// gather-scatter operator).
struct LevelView;
double hbm_probe_gbs(int kind, int64_t bytes, int reps, int device, Ctx &ctx);
double spmv_alone_us(const LevelView &L, bool fp32, int reps, Ctx &ctx);
// The same with every slice read from its 32-bit words.
double spmv_words_us(const LevelView &L, bool fp32, int reps, Ctx &ctx);

// ---------------------------------------------------------------------------
// Plain CSR on the device (output of the dual-graph builder).
// ---------------------------------------------------------------------------
struct DevCsr {
  int64_t n = 0, nnz = 0;
  DevBuf<int64_t> row_ptr;
  DevBuf<int32_t> col;
  DevBuf<int32_t> wgt;
};

void scan_exclusive(const int64_t *in, int64_t n, int64_t *out, int64_t *total, Ctx &ctx);
void scan_exclusive(const int32_t *in, int64_t n, int64_t *out, int64_t *total, Ctx &ctx);
void fill_i32(int32_t *p, int64_t n, int32_t v, Ctx &ctx);
void fill_f64(double *p, int64_t n, double v, Ctx &ctx);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits of the keys;
// with sync = false the result is only ordered on ctx.stream.
void sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int bits, Ctx &ctx,
                bool sync = true);

// Locality order of a graph (Cuthill-McKee: breadth-first levels from a
// pseudo-peripheral row, each level ordered by the least position of a
// neighbour in the level before, ties by row): perm[new row] = old row.  The
// CSR is rewritten in that order (columns relabelled).
void locality_order(DevCsr &g, DevBuf<int32_t> &perm, Ctx &ctx);

// Start values of opts->bfs_start for one mesh's dual graph (element order):
// warm[i] = (d_i - mean) / sd with d the number of edges from the pseudo-
// peripheral row (the row farthest from row 0, smallest index among the
// farthest), mean and sd over the rows the search reaches (exact integer
// sums); other entries are left as they are.
void bfs_start_values(const DevCsr &g, double *warm, Ctx &ctx);

// Dual graph of nelem elements with nv vertex ids each (device ids).
void build_dual_graph(const int64_t *d_ids, int64_t nelem, int nv, int graph, DevCsr &out,
                      Ctx &ctx);

// ---------------------------------------------------------------------------
// A bisection level: all segments (subgraphs still to be split) side by side.
//
// Rows of a level are the elements of all segments, each segment starting at a
// multiple of 64 and padded to a multiple of 64 with empty rows.  The
// Laplacian is stored as sliced ELL with slices of 64 rows: slice c holds
// `width_c` slot columns, slot k of row r at cols[chunk_ptr[c] + 64 k + r%64]
// as a packed (column, weight) word; unused slots are 0.  Columns are level
// row indices; cut edges to other segments are absent (induced subgraphs).
// ---------------------------------------------------------------------------
struct SegDev {
  int64_t row0;   // first row
  int32_t n;      // elements
  int32_t npad;   // rows (n rounded up to 64)
  int32_t P;      // parts this segment is divided into
  int32_t p0;     // first part id
  int32_t nlow;   // elements of the low child: floor(n * floor(P/2) / P)
  int32_t blk0, nblk, grp0, ngrp;
  int32_t mesh;   // input mesh of the segment
};

struct BlkDev {
  int64_t row0;   // first row of the tile
  int32_t nrows;  // rows in the tile (multiple of 64)
  int32_t seg;
  int32_t grp;
  int32_t pad;
};

struct GrpDev {
  int32_t seg, blk0, nblk, pad;
};

// Per-segment scalars of the eigen-solver (device resident).
struct SegState {
  double c, s;          // input vector transform: q = (w - c u0) * s
  double theta;         // Ritz value of the last cycle
  double tnorm;         // running estimate of ||T||
  double lq2;           // ||L q_j||^2 of the current step
  double alpha_tmp;     // alpha before the second Gram-Schmidt pass
  double res;           // residual norm of the last Ritz pair
  double rho;           // Rayleigh quotient of the last Ritz vector
  double invsqrt_nc;    // 1/sqrt(size of the solved component)
  int32_t k;            // Lanczos steps in the current cycle
  int32_t active;       // still iterating
  int32_t cycle_done;   // current cycle ended (length m or breakdown)
  int32_t need2;        // second Gram-Schmidt pass pending
  int32_t converged;    // tolerance met
  int32_t restarts;     // cycles run after the first
  int32_t strad;        // root row of the component being cut (-1: none)
  int32_t ncomp;        // components in the segment
  int32_t nlow2;        // low-side count inside the cut component
  int32_t solve;        // 1 if this segment has a component to cut
  int32_t flip;         // sign flip of the final vector
  int32_t first;        // row of the sign-deciding element
  int64_t steps;        // Lanczos or CG steps run (all cycles)
  int32_t cycles;       // cycles (Lanczos) or outer iterations (inverse iteration)
  int32_t cg_it;        // CG steps of the current solve
  double rr;            // CG: r^T r
  double cg_alpha, cg_beta;
  double cg_c;          // CG with AMG: u0 component removed from the preconditioned residual
  int32_t cg_done;      // CG solve finished
  int32_t j0;           // first Lanczos step of the current cycle (1, or nk + 1 after a thick restart)
  int32_t nk;           // Ritz pairs kept at the head of the current cycle's basis
  int32_t nnext;        // Ritz pairs formed at the end of the cycle (thick restart)
  int32_t refine;       // mixed precision: 1 = stopped where FP32 directions stall with
                        // the tolerance not met, 2 = continued with FP64 directions
  int32_t stall;        // consecutive cycles whose residual changed by <= 5%
  int32_t pair;         // two-step Lanczos: 0 none pending; 1 the last pair's block
                        // (W1, W2, factor R) awaits normalisation; 2 a one-column
                        // pair ended the cycle (W1 is the continuation); 3 the
                        // cycle's last vector awaits its second pass
  double r00, r01, r11; // two-step Lanczos: Cholesky factor of the last pair's block
};

// The Laplacian in gather-scatter form (Sec. 5: A_w = P^T Q Q^T P,
// L = diag(A_w 1) - A_w), on the weighted vertex-shared graph.  A group is
// one mesh vertex within one subgraph; row e's value of L x is the sum over
// its distinct vertices' groups g of (size_g x_e - U_g), U_g the sum of x
// over the group's rows.
constexpr uint32_t kGsNone = 0xFFFFFFFFu;  // slot without a group
constexpr int kGsMaxDeg = 64;              // most elements sharing one vertex

struct GsView {
  int nv = 0;                      // vertex slots per row; 0: sliced ELL operator
  const uint32_t *ev = nullptr;    // [nrows / 64][nv][64] group of each row slot
  const int32_t *deg = nullptr;    // [nrows] sum of the row's group sizes
  const uint32_t *gptr = nullptr;  // [ngroups + 1] offsets into gent (< 2^32 pairs)
  const int32_t *gent = nullptr;   // rows of every group, ascending
  const int32_t *gseg = nullptr;   // [ngroups] subgraph of the group
  double *U = nullptr;             // [ngroups] group sums of the vector multiplied
  int64_t ngroups = 0;
  int32_t only_seg = -1;           // >= 0: only that subgraph's groups (state slot 0)
};

// Vertex -> (element, slot) incidence of all meshes of a call, vertices in
// increasing id; a slot repeating an id already in its element is kGsNone.
struct GsBase {
  int nv = 0;
  int64_t nvert = 0, npairs = 0;
  DevBuf<int64_t> vptr;    // [nvert + 1]
  DevBuf<uint32_t> vent;   // [npairs] element * nv + slot, or kGsNone
};

struct GsLevel {
  int nv = 0;
  int64_t ngroups = 0, nent = 0;
  DevBuf<uint32_t> ev;
  DevBuf<int32_t> deg, gent, gseg;
  DevBuf<uint32_t> gptr;
  DevBuf<double> U;
};

struct Level {
  int64_t nrows = 0;     // padded rows
  int64_t nchunks = 0;   // nrows / 64
  int32_t nseg = 0;
  int32_t nblk = 0, ngrp = 0;
  int32_t rpt = 16;      // rows per thread of the streaming kernels (tile = 256 rpt)
  std::vector<SegDev> seg;
  std::vector<BlkDev> blk;
  std::vector<GrpDev> grp;
  DevBuf<SegDev> d_seg;
  DevBuf<BlkDev> d_blk;
  DevBuf<GrpDev> d_grp;
  DevBuf<int64_t> chunk_ptr;   // [nchunks + 1] word offsets
  DevBuf<uint32_t> cols;       // packed words
  DevBuf<int32_t> orig;        // row -> index in the concatenated input (-1: pad)
  DevBuf<int32_t> gid;         // row -> element id within its mesh
  int64_t words = 0;
  int64_t nnz = 0;             // off-diagonal nonzeros (non-padding words)
  DevBuf<uint32_t> pk;         // packed copy of the slices that fit (16-bit entries)
  DevBuf<int4> pmeta;          // [nchunks] window bases, or kPlainSlice
  DevBuf<int4> crlo, crhi;     // [nchunks] least / greatest column of each window
  DevBuf<TileStage> stage;     // [nchunks] at each tile's first slice (current tiles)
  DevBuf<int4> lmeta;          // [nchunks] LDS bases of the windows (current tiles)
  int64_t packed_slices = 0;   // slices read in the packed form
  int64_t packed_nnz = 0;      // nonzeros in those slices
  int64_t staged_tiles = 0;    // current tiles whose gathers are staged in LDS
  GsLevel gs;                  // gather-scatter operator, when selected
};

// Non-owning view of a level, or of some of its segments: vectors keep the
// level's row indexing (stride nrows), the tables may cover a subset.
struct LevelView {
  int64_t nrows = 0;
  int32_t nseg = 0, nblk = 0, ngrp = 0, rpt = 16;
  const SegDev *seg = nullptr;
  const BlkDev *blk = nullptr;
  const GrpDev *grp = nullptr;
  const int64_t *chunk_ptr = nullptr;
  const uint32_t *cols = nullptr;
  const uint32_t *pk = nullptr;
  const int4 *pmeta = nullptr;
  const TileStage *stage = nullptr;
  const int4 *lmeta = nullptr;
  const int32_t *gid = nullptr;
  const int32_t *orig = nullptr;
  int64_t nnz = 0;
  int64_t nchunks = 0, packed_slices = 0, packed_nnz = 0;
  GsView gs;
};

// Algorithmic bytes of a level's matrix as the row kernels read it: 4 per
// nonzero of a slice kept in 32-bit words, 2 per nonzero of a packed slice
// plus its 16 bytes of window bases.
inline double matrix_bytes(const LevelView &v) {
  const double pn = (double)v.packed_nnz;
  return 4.0 * ((double)v.nnz - pn) + 2.0 * pn + 16.0 * (double)v.packed_slices;
}

// Packed copy of a level's slices (or every slice marked kPlainSlice when
// packing is off): Level::pk, pmeta, packed_slices, packed_nnz.
void pack_level(Level &L, Ctx &ctx);

inline LevelView view_of(const Level &L) {
  LevelView v;
  v.nrows = L.nrows;
  v.nseg = L.nseg;
  v.nblk = L.nblk;
  v.ngrp = L.ngrp;
  v.rpt = L.rpt;
  v.seg = L.d_seg.get();
  v.blk = L.d_blk.get();
  v.grp = L.d_grp.get();
  v.chunk_ptr = L.chunk_ptr.get();
  v.cols = L.cols.get();
  v.pk = L.pk.get();
  v.pmeta = L.pmeta.get();
  v.stage = L.stage.get();
  v.lmeta = L.lmeta.get();
  v.nchunks = L.nchunks;
  v.packed_slices = L.packed_slices;
  v.packed_nnz = L.packed_nnz;
  v.gid = L.gid.get();
  v.orig = L.orig.get();
  v.nnz = L.nnz;
  if (L.gs.nv > 0) {
    v.gs.nv = L.gs.nv;
    v.gs.ev = L.gs.ev.get();
    v.gs.deg = L.gs.deg.get();
    v.gs.gptr = L.gs.gptr.get();
    v.gs.gent = L.gs.gent.get();
    v.gs.gseg = L.gs.gseg.get();
    v.gs.U = L.gs.U.get();
    v.gs.ngroups = L.gs.ngroups;
  }
  return v;
}

// Gather-scatter operator: the incidence of the call's meshes, vertices
// ordered by the least rank[e] of their elements (rank: element -> first
// level row; null: the element index), and its groups on one level.
void gs_base_build(const std::vector<const int64_t *> &ids, const std::vector<int64_t> &nelem,
                   int nv, const int32_t *rank, GsBase &B, Ctx &ctx);
void gs_level_build(const GsBase &B, const Level &L, int64_t nelem_total, GsLevel &G, Ctx &ctx);
// rank[orig[r]] = r for the live rows r of a level
void gs_rank_of_rows(const int32_t *orig, int64_t nrows, int32_t *rank, Ctx &ctx);
// y = L x on the rows of a level (FP64; vectors indexed by row).
void gs_apply(const GsView &g, int64_t nrows, const double *x, double *y, Ctx &ctx);

// Fill host block/group tables of a level from its segment table and
// upload all three tables.
void level_tables(Level &L, int rpt, Ctx &ctx);

// Tile of the streaming kernels: the built-in rows per thread, and the
// choice for one level (options, cache or timing trials; rebuilds the
// level's tables when it changes the tile).  work: the Lanczos workspace.
int default_rpt(int64_t nrows);
void choose_tile(Level &L, const rsb_opts &o, void *work, Ctx &ctx);

// Level 0 from per-mesh CSR graphs (segments in mesh order).  perm (optional,
// per mesh, device): row r of the CSR is element perm[r] of its mesh.
void level0_from_csr(Level &L, const std::vector<const DevCsr *> &g,
                     const std::vector<int32_t> &nparts, int rpt, Ctx &ctx,
                     const std::vector<const int32_t *> *perm = nullptr);

// ---------------------------------------------------------------------------
// Eigen-solver buffers for one level and one vector precision.
// ---------------------------------------------------------------------------
struct SolveDev {
  DevBuf<SegState> st;
  DevBuf<double> alpha, beta, h;         // [nseg][pstride]
  DevBuf<double> tvec;                   // [nseg][nkcap][pstride] Ritz coefficients
  DevBuf<double> tvals;                  // [nseg][nkcap] Ritz values
  DevBuf<double> arrow;                  // [nseg][pstride] couplings of kept Ritz vectors
  DevBuf<double> cdel;                   // [nseg][pstride] delayed second-pass coefficients
  int nkcap = 1;                         // Ritz vectors formed per cycle (1, or the kept count)
  DevBuf<double> part, gpart;            // [nblk][pstride], [ngrp][pstride]
  DevBuf<unsigned> gcnt, scnt;           // counters (zero between launches)
  DevBuf<int32_t> n_active;              // [4]: active count, stats
  DevBuf<int64_t> counters;              // [4]: segment steps
  int pstride = 0;
  int m = 0;
};

struct CompDev {
  DevBuf<int32_t> root;    // component root row of every row
  DevBuf<int32_t> size;    // component size at the root row
  DevBuf<int64_t> pre;     // exclusive prefix of sizes within a segment (at roots)
};

// Components of every segment and the part of each segment to cut.
void components_and_targets(Level &L, CompDev &C, SolveDev &S, Ctx &ctx);

// Lanczos solve of every segment with a component to cut.  Precision T of
// the vectors; FP64 scalars.  Result: y64[row] (unit norm on the component,
// zero elsewhere in the segment).  Returns the number of level-steps run.
struct KernelProfile {
  double ms = 0.0;       // summed device time of the profiled kernel
  double bytes = 0.0;    // its algorithmic bytes
  int64_t launches = 0;
};

struct LanczosParams {
  int m;
  int keep;              // 0: explicit restart; k > 0: thick restart keeping k Ritz pairs
  int max_restarts;
  double tol;
  int use_graph;
  uint64_t seed;
  KernelProfile *prof;   // non-null: time the step-j>=3 project kernel with events
  int64_t nnz;           // off-diagonal nonzeros of the level (for the byte count)
  double *y2_out;        // non-null (thick restart): the second Ritz vector, FP64
  const double *warm;    // non-null: warm start by element index (NaN: none)
  int pairs = 0;         // 1: thick restart runs steps j >= 3 two at a time
};
// work: lanczos_workspace_bytes(L.nrows, m, T is float, keep) bytes of device
// memory (FP64 u0, q_1, restart and work vectors; type-T directions q_2..q_m
// and two work vectors; FP64 kept Ritz vectors 2..keep when T is float).
// T = double: all FP64; T = float: mixed precision.
void solve_alloc(SolveDev &S, int nseg, int nblk, int ngrp, int m, int keep, Ctx &ctx);
size_t lanczos_workspace_bytes(int64_t rows, int m, bool fp32, int keep);
// Device time (ms) of one Lanczos step of the level with its current tile.
template <typename T>
double lanczos_trial_ms(const LevelView &L, int m, bool pairs, void *work, Ctx &ctx);
template <typename T>
int64_t lanczos_level(const LevelView &L, CompDev &C, SolveDev &S, const LanczosParams &p,
                      void *work, double *y64_out, Ctx &ctx);

// Block Lanczos of two vectors (method RSB_BLOCK, FP64): the Fiedler pair of
// every segment with a component to cut.  y64 receives y1, y2 (if non-null)
// y2 (zero without a second direction); S.tvals holds the pair's Ritz values
// (second: 1e300 without a second direction), S.st the Fiedler vector's
// Rayleigh quotient, residual, cycles and convergence.  Returns the block
// steps launched.
constexpr int kBkMaxM = 48;  // largest basis of a block Lanczos cycle
struct BlockParams {
  int m;                 // basis vectors per cycle (even): m / 2 blocks
  int keep;              // 0: explicit restart from the pair; k > 0 (even): thick restart
  int max_restarts;
  double tol;
  uint64_t seed;
  const double *warm;    // non-null: warm start of column 0 by element index (NaN: none)
  int sweep;             // > 0: a pair within sweep_gap is rotated to the start's projection
  double sweep_gap;
};
int64_t block_level(const LevelView &L, CompDev &C, SolveDev &S, const BlockParams &p,
                    double *y64, double *y2, Ctx &ctx);

// Aggregation multigrid hierarchy of a bisection level (preconditioner of
// the inverse-iteration solves).  Level 0 aliases the level's packed sliced
// ELL; coarse levels own sliced-ELL column and weight words.
struct MatDevHost {
  const int64_t *chunk_ptr = nullptr;
  const uint32_t *packed = nullptr;  // level 0
  const int32_t *col = nullptr;      // coarse levels
  const uint32_t *wgt = nullptr;
};

struct AmgLevelDev {
  int64_t n = 0;                 // rows (coarse levels: padded to a multiple of 64)
  int64_t words = 0;             // slots of a coarse level
  MatDevHost mat;
  const int32_t *gid = nullptr;  // global id carried by every row
  DevBuf<int32_t> gid_own;       // coarse levels
  DevBuf<int64_t> chunk_ptr;     // coarse levels
  DevBuf<int32_t> col;
  DevBuf<uint32_t> wgt;
  DevBuf<int32_t> seg;           // segment of a live row, -1 otherwise
  DevBuf<int32_t> rowlen;        // nonzero slots of the row
  DevBuf<double> dinv;           // 1 / L_ii (0 for an empty row)
  DevBuf<int32_t> agg;           // row of the next level (-1: none)
  DevBuf<int32_t> mem;           // coarse levels: the 1 or 2 rows collapsed into each row
  DevBuf<double> f;              // V-cycle right side (coarse levels)
  DevBuf<double> u, u2, r, r2;   // correction and residual, two buffers each
};

struct AmgDev {
  std::vector<AmgLevelDev> lv;
  double sigma = 2.0 / 3.0;      // damped-Jacobi weight
  int nsmooth = 1;               // Jacobi steps per smoothing phase
};

// Hierarchy of every segment with a component to cut (rows with
// root == that segment's strad); d_st: the solver's segment states.
void amg_setup(const LevelView &L, const int32_t *d_root, const SegState *d_st, AmgDev &A,
               Ctx &ctx);
// u = M f for the rows of running segments (d_st == nullptr: all live rows)
// into the level-0 buffer amg_result(A) (zero on rows that take no part),
// which it returns.  Launches only; graph-capturable.
const double *amg_vcycle(AmgDev &A, const double *d_f, const SegState *d_st, hipStream_t s);
const double *amg_result(const AmgDev &A);

// Inverse iteration with CG on every segment with a component to cut.
struct InverseParams {
  int max_outer;
  int cg_max_iter;
  double cg_tol;
  double tol;
  uint64_t seed;
  int precond;           // RSB_PRECOND_NONE or RSB_PRECOND_AMG
  double amg_sigma;
  int amg_smooth;
  int *amg_levels;       // out (may be null): levels of the largest hierarchy
  int full_projection;   // 0, or k: L-orthogonalise each new direction against the last k
};
// FP64 vectors of the inverse-iteration workspace: 8, plus 2 k for the
// directions kept by full projection
size_t inverse_workspace_bytes(int64_t rows, int full_projection = 0);
int64_t inverse_level(const LevelView &L, CompDev &C, SolveDev &S, const InverseParams &p,
                      void *work, double *y64_out, bool use_graph, Ctx &ctx);

// Sweep over the Fiedler pair (thick restart): for every segment whose
// second Ritz value lies within sweep_gap (relative) of the first, replace
// y64 by the combination cos(a) y1 + sin(a) y2 (y2 orthonormalised against
// u0 and y1, both with the canonical sign; a = k pi / nangles) whose split
// cuts the least weight.  Counts swept segments and those that moved.  A
// segment is swept only if the part of y2 off u0 and y1 has squared norm
// above min_perp2 (y2 of unit norm).  on_out (optional): 1 per swept segment.
void fiedler_sweep(Level &L, CompDev &C, SolveDev &S, double *y64, const double *y2, int nangles,
                   double sweep_gap, int *swept, int *moved, Ctx &ctx,
                   double min_perp2 = 1e-12, std::vector<int32_t> *on_out = nullptr);

// Warm start for the next level: warm[orig[row]] = the second Ritz vector y2
// at unit root-mean-square on each segment's cut component (segments whose
// last cycle formed a second Ritz vector; other entries keep their values).
void warm_update(Level &L, CompDev &C, SolveDev &S, const double *y2, double *warm, Ctx &ctx);

// Canonical sign of y on every segment being cut (in place).
void canonical_sign_level(Level &L, CompDev &C, SolveDev &S, double *y, Ctx &ctx);

// Sign rule, radix select and side assignment.  side[row]: 0 low, 1 high,
// 2 padding.
void split_level(Level &L, CompDev &C, SolveDev &S, const double *y64, uint8_t *side, Ctx &ctx);

// Split of a single vector with given gids (test entry point).
void split_vector(const double *d_y, const int64_t *d_gid, int64_t n, int64_t n_low,
                  uint8_t *d_side, Ctx &ctx);

// Next level from the sides; leaves write part ids into part_out (indexed
// by orig).  Returns the new level (possibly empty).
void compact_level(Level &L, const uint8_t *side, int32_t *d_part_out, Level &next, int rpt,
                   Ctx &ctx);

// y = L x on a plain CSR (FP64), through the sliced-ELL kernel.
void laplacian_apply_csr(const DevCsr &g, const double *d_x, double *d_y, Ctx &ctx);

// Edge cut and neighbour counts of a partition on the level-0 graph.
void partition_metrics(Level &L0, const int32_t *d_part, int32_t nparts_total,
                       const std::vector<int32_t> &part_offset, rsb_stats *st, Ctx &ctx);

}  // namespace rsb
