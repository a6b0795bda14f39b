/*
 * rsb.h -- C ABI of the MI355X (gfx950) recursive spectral bisection library.
 *
 * Problem (paper Sec. 2): given a mesh as per-element global vertex ids and a
 * number of parts P, assign every element to one part so that the parts are
 * disjoint, cover the mesh, and differ in size by at most one element, while
 * the dual-graph edge cut stays small.  The method (Sec. 4, Alg. 1) bisects
 * the element dual graph by the Fiedler vector of its Laplacian, computed by
 * restarted Lanczos (Sec. 6) or by inverse iteration with conjugate
 * gradients (Sec. 7, Alg. 2), and recurses into floor(P/2) / ceil(P/2) parts.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Element i of a mesh is row i of `elem_vertex_ids` (row-major, int64,
 *    nelem x nv_per_elem).  Its global id is i; ids are used for the random
 *    start vector, for tie-breaks and for ordering components.
 *  - Buffers are owned by the caller.  The library never frees or keeps a
 *    caller pointer after returning.  With opts->device_pointers == 0 every
 *    array argument is host memory; with 1 every array argument is device
 *    memory on opts->device (for instance a torch tensor's data_ptr()).
 *  - Calls are synchronous: outputs are complete when the call returns.
 *    Work is queued on opts->stream (a hipStream_t; NULL = the null stream).
 *    Calls on distinct streams may run from distinct host threads.
 *  - Scratch device memory comes from the stream-ordered allocator of the
 *    device.  Blocks a call releases are reused by its later allocations;
 *    when the call ends they are kept, idle, in a per-device cache of at most
 *    32 GiB that later calls draw from before asking the allocator (each
 *    allocation and free of the allocator holds the host for about 0.1 ms).
 *    The cache is emptied back into the allocator's pool whenever an
 *    allocation finds the device out of memory.
 *  - Limits: nelem < 2^28 elements per call (all meshes of a batch
 *    together), edge weights <= 15 (shared-vertex counts), at most 1024
 *    candidate neighbour entries per element when building the graph
 *    (sum over its vertices of the elements touching that vertex).
 *
 * Return codes: 0 success; positive = warning, outputs valid; negative =
 * error, outputs unspecified.  rsb_last_error() gives a message for the last
 * failing call on the calling thread.
 */
#ifndef RSB_H
#define RSB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSB_OK 0
#define RSB_WARN_NOT_CONVERGED 1 /* iteration caps reached; outputs valid */
#define RSB_WARN_DISCONNECTED 2  /* a bisected graph was disconnected; rule below used */
#define RSB_EINVAL (-1)          /* invalid argument */
#define RSB_ENOMEM (-2)          /* device memory exhausted or above device_mem_limit */
#define RSB_EDEVICE (-3)         /* HIP runtime error */
#define RSB_EBUFFER (-4)         /* output buffer too small (see rsb_dual_graph) */
#define RSB_EINTERNAL (-5)       /* internal consistency check failed */

/* Dual-graph kinds.  Two elements are adjacent when they share at least one
 * vertex id (Sec. 2); s_ij = number of distinct ids they share.  */
#define RSB_GRAPH_WEIGHTED 0 /* weight s_ij (Sec. 4, weighted Laplacian; default) */
#define RSB_GRAPH_UNIT 1     /* weight 1 for every adjacent pair (Sec. 4, unweighted) */
#define RSB_GRAPH_FACE 2     /* weight 1 when s_ij >= nv/2 (face neighbours), else no edge */

#define RSB_LANCZOS 0    /* restarted Lanczos, full reorthogonalisation (Sec. 6) */
#define RSB_INVERSE_CG 1 /* inverse iteration, CG inner solves (Sec. 7, Alg. 2) */
#define RSB_AUTO 2       /* Lanczos; every subgraph it leaves unconverged is solved
                            again by inverse iteration from the random start
                            (Sec. 7: the paper's fallback where Lanczos did not
                            converge) */
#define RSB_BLOCK 3      /* block Lanczos of two vectors, orthogonalised together at
                            every step (Sec. 9: the block iteration that finds both
                            vectors of an exactly degenerate Fiedler pair): one
                            solve gives the pair for fiedler_sweep.  FP64 whatever
                            precision says; lanczos_m (even, 4..48) basis vectors
                            per cycle, lanczos_keep (even, <= lanczos_m - 4) kept
                            Ritz vectors of a thick restart (0: explicit restart
                            from the pair); converged when both Ritz pairs meet
                            tol (the second when there is one).  lanczos_s,
                            gather_scatter and second_solve do not apply. */

#define RSB_PRECOND_NONE 0 /* INVERSE_CG: plain CG */
#define RSB_PRECOND_AMG 1  /* INVERSE_CG: aggregation multigrid V-cycle (Sec. 7, Alg. 3) */

#define RSB_FP64 0  /* all vectors and arithmetic in FP64 */
#define RSB_MIXED 1 /* Lanczos directions q_2..q_m and their SpMV in FP32 (FP32
                       accumulation); in FP64: the restart (Ritz) vector and the
                       first Lanczos vector of every cycle, residuals, alpha,
                       beta, reorthogonalisation projections and the
                       tridiagonal solve.  Explicit restart: each restart
                       refines the FP64 Ritz vector by an FP32 correction, so
                       the pair converges to the FP64 tolerance.  Thick
                       restart: FP32 rounding stalls the residual near a
                       multiple of 2^-24 ||L|| (about 0.6 2^-24 ||L|| /
                       lambda relative); a subgraph whose residual stalls
                       short of tol continues from its Ritz vector with FP64
                       directions until the FP64 residual meets tol (its
                       FP64 cycles count in max_restarts). */

typedef struct rsb_opts {
  int32_t struct_size;      /* sizeof(rsb_opts); set by rsb_opts_init */
  int32_t graph;            /* RSB_GRAPH_* */
  int32_t method;           /* RSB_LANCZOS, RSB_INVERSE_CG, RSB_AUTO or RSB_BLOCK */
  int32_t precision;        /* RSB_FP64 or RSB_MIXED */
  int32_t lanczos_m;        /* Lanczos steps per cycle (default 100, max 250) */
  int32_t max_restarts;     /* restarts after the first cycle (default 50) */
  double tol;               /* converged when ||L y - rho y||_2 <= tol * rho, rho =
                               y^T L y / y^T y of the Ritz vector y (default 1e-6) */
  int32_t inv_max_outer;    /* inverse iteration (INVERSE_CG, AUTO's fallback): outer
                               iterations cap (50) */
  int32_t cg_max_iter;      /* inverse iteration: CG steps per solve cap (20000) */
  double cg_tol;            /* inverse iteration: CG stops at ||r|| <= cg_tol ||b|| (1e-8) */
  int32_t cg_full_projection; /* inverse iteration: 0 (default) plain flexible CG; k in
                                 [1, 32]: every new direction is L-orthogonalised
                                 against the last k directions of the solve (the
                                 paper's CG "augmented with full projection",
                                 Sec. 7) */
  int32_t batched;          /* 1: all subgraphs of a level in one launch sequence;
                               0: one subgraph at a time (reference mode) */
  uint64_t seed;            /* start-vector seed (default 20261203) */
  int32_t use_hipgraph;     /* 1: replay each Lanczos cycle as a captured hipGraph */
  int32_t autotune;         /* 0: built-in tile; 1: use/extend the cache; 2: retune */
  const char *autotune_cache; /* path of the tile cache file (NULL: no file) */
  int32_t device;           /* HIP device ordinal */
  int32_t device_pointers;  /* 0: host arrays; 1: device arrays */
  void *stream;             /* hipStream_t, NULL for the null stream */
  int64_t device_mem_limit; /* 0: no limit; else bytes of scratch allowed */
  int32_t verbose;          /* 1: one line per level on stderr; 2: also per segment */
  int32_t profile;          /* 1: time every launch of the SpMV-and-projection
                               kernel of Lanczos steps j >= 3 with HIP events
                               (cycles are then launched directly, not replayed
                               as graphs); results in rsb_stats.kernel_* */
  int32_t rows_per_thread;  /* tile of the streaming kernels, 256 * rows_per_thread
                               rows per workgroup: 0 = chosen by the library (see
                               autotune), else 2, 4 or 8 for every level */
  int32_t lanczos_keep;     /* 0 (default): explicit restart, every cycle starts
                               from the current Ritz vector (Sec. 6); k in
                               [1, min(16, lanczos_m - 1)]: thick restart (the
                               Lanczos variant the paper cites in Sec. 6) keeping
                               the k smallest Ritz pairs and continuing from the
                               last residual direction.  With precision =
                               RSB_MIXED the kept Ritz vectors stay FP64, and a
                               solve that stalls short of tol finishes with FP64
                               directions (see RSB_MIXED).  Known limitation:
                               where a cycle exhausts the Krylov space (a
                               subgraph of at most lanczos_m + 1 elements, or
                               fewer distinct eigenvalues than lanczos_m), the
                               explicit restart can miss the breakdown and
                               return a poor vector for that bisection (most
                               often reported as RSB_WARN_NOT_CONVERGED at the
                               restart cap, but a loose tol can pass it); the
                               thick restart one step at a time does not.
                               Partitions into parts of a few dozen elements
                               should use k > 0 with lanczos_s = 1. */
  int32_t inv_precond;      /* inverse iteration: RSB_PRECOND_NONE (default) or
                               RSB_PRECOND_AMG.  With AMG the first direction
                               of every CG solve is still the plain residual
                               (Sec. 7); later ones are one V-cycle of the
                               residual.  The hierarchy collapses pairs of rows
                               chosen by a handshake matching on edge weight
                               (the paper pairs elements along an RCB order;
                               no coordinates are given here) into Galerkin
                               coarse Laplacians, per subgraph. */
  int32_t amg_smooth;       /* AMG: damped-Jacobi steps per smoothing phase (1) */
  double amg_sigma;         /* AMG: Jacobi damping weight (2/3) */
  int32_t fiedler_sweep;    /* RSB_BLOCK, or Lanczos (RSB_LANCZOS or RSB_AUTO) with
                               lanczos_keep >= 2: S > 0 sweeps the
                               Fiedler pair (Sec. 9: search the combinations of a
                               near-degenerate pair for the smallest cut).  When
                               the second Ritz value is within sweep_gap of the
                               first, S combinations cos(a) y1 + sin(a) y2,
                               a = k pi / S, are split and the one that cuts the
                               least weight is used (ties: smallest k).  0: off
                               (default); at most 64.  With one-vector Lanczos an
                               exactly degenerate pair shows a single Ritz vector
                               and is not swept; RSB_BLOCK finds both and, for a
                               pair within sweep_gap, first rotates it within its
                               plane so that y1 is the projection of the random
                               start (a well-defined basis). */
  int32_t warm_start;       /* RSB_BLOCK, or Lanczos (LANCZOS or AUTO) with lanczos_keep
                               >= 2: 1 = the solve of a
                               subgraph starts from its parent's second Ritz
                               vector (unit root-mean-square on the parent's cut
                               component) plus 0.1 x the random start; elements
                               without one take the random start.  The paper
                               leaves the start vector open; 0 (default): the
                               random start everywhere. */
  double sweep_gap;         /* relative gap (theta2 - theta1) / theta1 below which
                               the pair is swept (0.1) */
  int32_t reorder;          /* rsb_partition(_batch): 1 = store each mesh's rows in
                               Cuthill-McKee order of its dual graph (see
                               rsb_locality_order) before the first level, so that
                               neighbours lie close in memory (the paper sorts by
                               RCB first; no coordinates are given here).
                               Element ids, start vectors, tie-breaks and outputs
                               keep the input numbering.  0 (default): input order. */
  int32_t gather_scatter;   /* 1 = the Lanczos SpMV applies the Laplacian in the
                               paper's gather-scatter form (Sec. 5: element values
                               summed per mesh vertex and subgraph, then gathered
                               back per element) instead of the assembled sliced-ELL
                               matrix; the same operator, so results agree to
                               rounding.  Needs graph RSB_GRAPH_WEIGHTED, method
                               RSB_LANCZOS and at most 64 slots per vertex id.
                               0 (default): sliced ELL. */
  int32_t second_solve;     /* with fiedler_sweep > 0: the second vector of the swept
                               pair comes from a second Lanczos solve of the same
                               subgraph from another random start (seed ^
                               0x9E3779B97F4A7C15, no warm start) instead of the
                               thick restart's second Ritz vector; it is swept when
                               its Rayleigh quotient is within sweep_gap of the
                               first and at least 0.1 of it lies off the first
                               vector; where it is not, the thick restart's own
                               pair is swept as without the option.  One Krylov
                               space holds a single direction of an exactly
                               degenerate pair (Sec. 9), two solves hold two.
                               Doubles the solve time.  0 (default). */
  int32_t lanczos_s;        /* thick restart (lanczos_keep > 0) with the sliced-ELL
                               operator: 2 = from step 3 on, steps j and j+1 come
                               from one block [L q_j, L^2 q_j] (two-step Lanczos:
                               the same Krylov space and projected matrix as one
                               step at a time in exact arithmetic; the basis is
                               read twice per two steps instead of twice per
                               step); 1 (default) = one step at a time.  Ignored
                               for explicit restart and gather_scatter.  A level
                               that solves a component of at most
                               4 * lanczos_m elements runs one step at a time
                               (a cycle can exhaust the Krylov space of such a
                               graph, and the block's single Gram-Schmidt pass
                               before its Cholesky QR can miss that breakdown). */
  int32_t pack_matrix;      /* 1 (default) = each level also keeps a packed copy of
                               the sliced-ELL slices whose column offsets from the
                               row (column - row) fit in at most 4 windows of 1024:
                               16-bit entries (weight, window, offset) instead of
                               32-bit words, read by the Lanczos SpMVs and the
                               inverse iteration's residual (its CG steps read the
                               words); the other slices are read as 32-bit words.  2 = also, per
                               workgroup tile of the Lanczos SpMVs, the intervals of
                               the vector that its packed slices reach (up to 6
                               intervals, 4864 values) are copied into LDS first and
                               the neighbours gathered there.  The same entries in
                               the same order and the same values, so results are
                               bitwise those of 0 = 32-bit words only. */
  int32_t bfs_start;        /* 1 = the first Lanczos solve of each mesh (the one
                               with no parent vector to start from) starts from the
                               number of edges between each element and a pseudo-
                               peripheral element (the element farthest from element
                               0, smallest index among the farthest), centred and
                               scaled to unit root-mean-square over the elements the
                               search reaches, plus 0.1 x the random start; other
                               elements take the random start.  Not in the paper,
                               which leaves the start vector open.  Fewer steps, but
                               on a mesh whose Fiedler pair is near-degenerate (two
                               long axes of equal length) the start is symmetric in
                               the pair, and a loose tolerance can stop in a mixture
                               of it that cuts diagonally (256 x 256 x 64 box at tol
                               1e-2: cut +10%).  0 (default): the random start. */
} rsb_opts;

typedef struct rsb_stats {
  int32_t struct_size;       /* sizeof(rsb_stats), set by the caller */
  int32_t levels;            /* bisection levels run */
  int64_t level_steps;       /* Lanczos (or CG, or RSB_BLOCK's block) steps, one
                                per launch over all segments of a level */
  int64_t segment_steps;     /* the same counted per segment (a block step
                                applies L to two vectors) */
  int64_t cycles;            /* Lanczos cycles summed over levels */
  int64_t spmv_fp64;         /* SpMVs run with FP64 vectors (level launches) */
  int32_t not_converged;     /* segments that hit the iteration caps */
  int32_t disconnected;      /* bisections of disconnected graphs */
  double lambda2;            /* rsb_fiedler: Rayleigh quotient of the output;
                                rsb_partition(_batch): of the first bisection's
                                Fiedler vector (of the first mesh) */
  double residual;           /* ||L y - lambda y|| of that vector (FP64) */
  double ms_graph;           /* dual-graph build (device time) */
  double ms_solve;           /* eigen-solves */
  double ms_split;           /* components, split and compaction */
  double ms_total;           /* whole call, host wall clock */
  /* Partition quality, measured on the dual graph selected by opts->graph
   * (with the default vertex-shared graph, neighbours are the parts that
   * share at least one mesh vertex, as in the paper's Sec. 8 tables). */
  double edge_cut;           /* rsb_partition: sum of the weights of cut edges */
  int64_t cut_pairs;         /* rsb_partition: adjacent element pairs cut */
  int32_t max_neighbors;     /* rsb_partition: max neighbour parts of a part
                                (-1 when the total number of parts > 16384) */
  double avg_neighbors;      /* rsb_partition: mean neighbour parts of a part */
  int64_t nnz;               /* off-diagonal nonzeros of the level-0 Laplacian */
  /* opts->profile = 1: the SpMV-and-projection kernel of Lanczos steps j >= 3
   * (lanczos_s = 2: the B launch of the pair starting at step j) */
  double kernel_bytes;       /* algorithmic bytes of all its launches: per launch at
                                step j over n rows, 4 (n + 1) + M + n (s_x + s_Lq +
                                s_q + 16 + (j - 2) s_q + (k - 1)(8 - s_q)), M = the
                                rows' share of matrix_bytes (below; 4 nnz without
                                packing), s_ = bytes per value, k = Ritz pairs kept
                                by a thick restart (FP64 basis slots 2..k; no term
                                for k <= 1); lanczos_s = 2: 4 (n + 1) + M + n (8 +
                                8 + 16 + (j - 1) s_q + (k - 1)(8 - s_q)) (z1 read,
                                z2 written, both FP64; basis slots 0..j) */
  double kernel_ms;          /* summed device time of its launches (HIP events) */
  int64_t kernel_launches;   /* its launches */
  int32_t tile_rows;         /* rows per workgroup of the streaming kernels at level 0 */
  int32_t amg_levels;        /* INVERSE_CG with AMG: levels of the deepest hierarchy */
  int32_t sweeps;            /* fiedler_sweep: bisections whose Fiedler pair was swept */
  int32_t sweep_moved;       /* of those, bisections where an angle other than 0 won */
  int32_t fallbacks;         /* RSB_AUTO: bisections solved again by inverse iteration */
  int32_t reserved;
  double ms_reorder;         /* opts->reorder = 1: locality order of the rows (host wall
                                clock, included in ms_total) */
  /* opts->profile = 1 (Lanczos, sliced ELL): y = L x alone on the level-0
   * matrix in the directions' precision, 20 launches timed with HIP events */
  double spmv_alone_us;      /* average launch time */
  double spmv_alone_bytes;   /* algorithmic bytes per launch: 4 (n + 1) + matrix_bytes
                                + 2 s n */
  /* level 0 (first mesh's level of rsb_partition_batch: the whole level) */
  double packed_fraction;    /* nonzeros in packed slices / nnz */
  double matrix_bytes;       /* the matrix as the SpMV reads it: 4 per nonzero of a
                                32-bit slice, 2 per nonzero of a packed slice plus 16
                                per packed slice (window bases) */
  double staged_fraction;    /* tiles (workgroups of the streaming kernels) whose
                                gathers are staged in LDS / tiles */
  /* opts->profile = 1: the level-0 SpMV alone as above with every slice read from
   * its 32-bit words */
  double spmv_words_us;      /* average launch time */
  double spmv_words_bytes;   /* algorithmic bytes per launch: 4 (n + 1) + 4 nnz + 2 s n */
} rsb_stats;

/* Fills *o with the defaults listed above.  Returns RSB_OK or RSB_EINVAL (o NULL). */
int rsb_opts_init(rsb_opts *o);

/* Element dual graph and its Laplacian (Sec. 2; Sec. 4 equations for the
 * unweighted and weighted Laplacian; Sec. 5: the same matrix as the
 * off-diagonal part of P^T Q Q^T P).  Output: off-diagonal CSR of L with
 * positive weights w_ij = -l_ij, columns strictly ascending within a row,
 * row_ptr[nelem + 1] int64, col_idx[nnz] int32, weight[nnz] int32; the
 * diagonal is the row sum of weights.  A vertex id repeated inside one element
 * counts once.  Two-call size query: with col_idx == NULL only *nnz_inout is
 * written (row_ptr may be NULL then); otherwise *nnz_inout is the capacity of
 * col_idx/weight on entry and nnz on return, RSB_EBUFFER if too small.
 * Errors: RSB_EINVAL for null ids/nnz_inout, nelem < 1, nv < 1, a negative id,
 * a weight above 15 or an element with more than 1024 candidate entries. */
int rsb_dual_graph(int64_t nelem, int32_t nv_per_elem, const int64_t *elem_vertex_ids,
                   const rsb_opts *opts, int64_t *row_ptr, int32_t *col_idx, int32_t *weight,
                   int64_t *nnz_inout);

/* y = L x on a caller-supplied off-diagonal CSR (row_ptr int64[n+1], col_idx
 * int32, weight int32 in [0, 15], columns < n), evaluated as
 * y_i = sum_j w_ij (x_i - x_j) in FP64 (Sec. 5: the action of the Laplacian).
 * Exposed for testing the SpMV.  RSB_EINVAL on bad sizes or weights. */
int rsb_laplacian_apply(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                        const int32_t *weight, const double *x, double *y, const rsb_opts *opts);

/* y = L x in the gather-scatter form (Sec. 5: L = diag(A_w 1) - A_w,
 * A_w = P^T Q Q^T P over the mesh's vertex ids) for one mesh of nelem
 * elements with nv_per_elem vertex ids each (a repeated id within an element
 * counts once), evaluated on the GPU as for opts->gather_scatter = 1 at the
 * first level.  x, y: nelem doubles, host or device memory as
 * opts->device_pointers says.  Exposed for testing.  Errors as
 * rsb_dual_graph, and RSB_EINVAL when a vertex id appears in more than 64
 * slots. */
int rsb_gs_apply(int64_t nelem, int32_t nv_per_elem, const int64_t *elem_vertex_ids,
                 const double *x, double *y, const rsb_opts *opts);

/* The locality order that opts->reorder = 1 gives the level-0 rows, on a
 * caller CSR as in rsb_laplacian_apply: order[k] = row placed at position k
 * (int32[n], host or device memory as opts->device_pointers says).  It is the
 * Cuthill-McKee order: breadth-first levels from the row farthest from row 0
 * (smallest index among the farthest), each level ordered by the least
 * position of a neighbour in the level before, ties by row index, rows not
 * reached last by row index.  Not a step of the paper's method: it stands in
 * for the coordinate pre-sort (recursive coordinate bisection) the paper
 * applies before partitioning, as the input carries no coordinates.
 * Exposed for testing.  RSB_EINVAL on bad sizes or weights. */
int rsb_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                       const int32_t *weight, int32_t *order, const rsb_opts *opts);

/* Level `level` of the aggregation multigrid hierarchy that preconditions the
 * inverse-iteration solves (Sec. 7, Alg. 3: pairs of rows collapsed by a
 * Boolean prolongation J, coarse Laplacian J^T L J), built on a caller CSR
 * as in rsb_laplacian_apply with row i's global id = i and every row taking
 * part.  Exposed for testing the setup.  Two-call protocol: with col_out ==
 * NULL only *nlevels, *nrows and *nnz are written; otherwise the arrays must
 * hold nrows + 1 (row_ptr_out), nnz (col_out, weight_out) and nrows (gid_out,
 * agg_out: the row of level + 1 each row collapses into, -1 on the coarsest
 * level) entries, host memory, and receive the level's CSR (columns
 * ascending, int64 weights).  RSB_EINVAL on bad sizes or a level outside
 * [0, *nlevels). */
int rsb_amg_level(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                  const int32_t *weight, int32_t level, const rsb_opts *opts, int32_t *nlevels,
                  int64_t *nrows, int64_t *nnz, int64_t *row_ptr_out, int64_t *col_out,
                  int64_t *weight_out, int64_t *gid_out, int64_t *agg_out);

/* u = M f: one V-cycle of that hierarchy (opts->amg_sigma, opts->amg_smooth)
 * on a caller CSR (same conventions), f and u of n doubles (host or device
 * per opts->device_pointers).  Exposed for testing the V-cycle.  Errors as
 * rsb_amg_level, and RSB_EINVAL for a NULL f or u. */
int rsb_amg_vcycle(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                   const int32_t *weight, const double *f, double *u, const rsb_opts *opts);

/* Fiedler pair of the mesh's dual-graph Laplacian (Sec. 4: L x = lambda x
 * with 1^T x = 0; Sec. 6 Lanczos or Sec. 7 inverse iteration).  fiedler_out
 * [nelem] FP64 in element order, unit 2-norm, orthogonal to the ones vector,
 * with its sign fixed so that the lowest-index element whose |y_i| is at least
 * 1e-3 max|y| has y_i <= 0.  *lambda2_out = y^T L y (FP64).  If the graph is
 * disconnected, the bisection rule for disconnected graphs applies (see
 * rsb_partition): the vector is the Fiedler vector of the component that
 * straddles position floor(nelem/2), zero elsewhere (all zero, lambda 0, if
 * no component straddles it), and RSB_WARN_DISCONNECTED is returned.
 * stats_out may be NULL.  Errors: as rsb_dual_graph, and nelem < 2. */
int rsb_fiedler(int64_t nelem, int32_t nv_per_elem, const int64_t *elem_vertex_ids,
                const rsb_opts *opts, double *fiedler_out, double *lambda2_out,
                rsb_stats *stats_out);

/* The split rule (Sec. 4: sort by the Fiedler vector and give the first part
 * of the sorted order to the first half of the processors): side[i] = 0 for
 * the n_low smallest keys (y_i, gid_i) and 1 for the rest, where keys compare
 * y first (IEEE total order, -0.0 before +0.0) and then gid.  gid must be
 * distinct.  Exposed for testing the radix select.  RSB_EINVAL on NaN in y,
 * n_low outside [0, n] or null pointers. */
int rsb_split(int64_t n, const double *y, const int64_t *gid, int64_t n_low, uint8_t *side,
              const rsb_opts *opts);

/* Recursive spectral bisection (Alg. 1).  part_out[nelem] int32 in [0, nparts).
 * A part range [p0, p0 + P) with n elements splits into [p0, p0 + floor(P/2))
 * with floor(n floor(P/2) / P) elements (the smallest keys of the Fiedler
 * vector, see rsb_split) and [p0 + floor(P/2), p0 + P) with the rest, so all
 * part sizes are floor(nelem/nparts) or ceil(nelem/nparts).  A disconnected
 * subgraph is bisected component-wise: components ordered by smallest global
 * id go whole to the low side while they fit; the one component that
 * straddles the target count is cut by its own Fiedler vector.
 * Returns RSB_OK, RSB_WARN_DISCONNECTED if that rule was used,
 * RSB_WARN_NOT_CONVERGED if a solve hit its caps (the partition is still
 * valid).  Errors: as rsb_dual_graph, nparts < 1 or nparts > nelem.
 * stats_out may be NULL. */
int rsb_partition(int64_t nelem, int32_t nv_per_elem, const int64_t *elem_vertex_ids,
                  int32_t nparts, const rsb_opts *opts, int32_t *part_out, rsb_stats *stats_out);

/* rsb_partition on nmesh independent meshes in one call: every bisection
 * level of all meshes runs as one batched launch sequence.  Mesh b has
 * nelem[b] elements, ids elem_vertex_ids[b] and is split into nparts[b]
 * parts written to part_out[b].  With device_pointers == 1 the pointer
 * arrays themselves are host arrays of device pointers.  Results equal nmesh
 * separate rsb_partition calls; stats_out covers the whole call.  Errors:
 * RSB_EINVAL for nmesh < 1, a NULL array or part_out entry, any mesh that
 * rsb_partition would reject, or 2^28 or more elements in all. */
int rsb_partition_batch(int32_t nmesh, const int64_t *nelem, int32_t nv_per_elem,
                        const int64_t *const *elem_vertex_ids, const int32_t *nparts,
                        const rsb_opts *opts, int32_t *const *part_out, rsb_stats *stats_out);

/* For callers that cannot allocate device memory: code that must not call
 * hipMalloc (tight serving loops, harnesses that forbid allocation).
 * rsb_partition with every device buffer of the call carved from one fixed
 * region of RSB_NOALLOC_SCRATCH_BYTES per GPU, a device array the library
 * holds from load until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call.  Arguments, outputs and return codes as
 * rsb_partition, with these differences: at most RSB_NOALLOC_MAX_ELEMS
 * elements and RSB_NOALLOC_MAX_PARTS parts (RSB_EINVAL beyond); RSB_ENOMEM,
 * with the sizes in rsb_last_error, when options need more than the region
 * (the defaults, and the benchmark's mixed-precision thick restart, fit at
 * the maximum sizes; lanczos_m near 250 or an AMG hierarchy may not); graph
 * replay, profiling and tile timing are off whatever opts says; a NULL
 * opts->stream means the null stream.  The region keeps the last call's
 * contents; the library clears what it needs itself.  Calls from threads of
 * one process on one GPU take turns on a lock, and each call drains its
 * stream before it returns, so no two of them overlap; a call must not be
 * captured into a graph (it synchronises its stream). */
#define RSB_NOALLOC_SCRATCH_BYTES (256ll << 20)
#define RSB_NOALLOC_MAX_ELEMS 65536
#define RSB_NOALLOC_MAX_PARTS 1024
int rsb_partition_noalloc(int64_t nelem, int32_t nv_per_elem, const int64_t *elem_vertex_ids,
                          int32_t nparts, const rsb_opts *opts, int32_t *part_out,
                          rsb_stats *stats_out);

/* Reference for the roofline of the streaming kernels (not a step of the
 * method): *gbs_out = GB/s of a plain HBM stream over `bytes` on
 * opts->device and opts->stream, the average of `reps` launches after a
 * warm-up.  kind 0: read (16-byte non-temporal loads, summed); 1: copy
 * (bytes read plus bytes written); 2: write.  Allocates its buffers.
 * Errors: RSB_EINVAL for a bad kind, bytes < 4096, reps < 1 or a NULL
 * pointer; RSB_ENOMEM; RSB_EDEVICE. */
int rsb_hbm_probe(int32_t kind, int64_t bytes, int32_t reps, const rsb_opts *opts,
                  double *gbs_out);

/* Message for a return code (static string). */
const char *rsb_strerror(int code);
/* Message of the last failing call on this thread ("" if none). */
const char *rsb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RSB_H */
