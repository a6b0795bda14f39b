/*
 * oracle.h -- plain FP64 CPU reference for recursive spectral bisection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the partitioning library links,
 * includes or calls this code; only the test-suite, the smoke check and the
 * CPU baseline of the benchmark load it.  It shares no source with the GPU
 * library.
 *
 * What it computes (paper sections in brackets):
 *   - the element dual graph and its Laplacian [Sec. 2, Sec. 4 eqs. for the
 *     unweighted and weighted Laplacian, Sec. 5 A_w = P^T Q Q^T P];
 *   - the Fiedler pair by restarted Lanczos with full reorthogonalisation
 *     [Sec. 6] or by inverse iteration with conjugate gradients [Sec. 7,
 *     Alg. 2];
 *   - the median split and the recursion into floor(P/2) / ceil(P/2) parts
 *     [Sec. 4, Alg. 1];
 *   - the Laplacian in gather-scatter form [Sec. 5] and a Cuthill-McKee
 *     locality order of the elements (standing in for the coordinate
 *     pre-sort of Sec. 5 and Sec. 8).
 *
 * All arithmetic is IEEE double, round to nearest, without contraction into
 * fused multiply-adds.  Loops over vector elements may run on several
 * threads (OpenMP, see orc_set_threads); every sum over elements is taken in
 * a fixed order of fixed chunks, so the results do not depend on the number
 * of threads, bit for bit.
 */
#ifndef RSB_ORACLE_H
#define RSB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GRAPH_WEIGHTED = 0, ORC_GRAPH_UNIT = 1, ORC_GRAPH_FACE = 2 };
enum { ORC_LANCZOS = 0, ORC_INVERSE_CG = 1, ORC_AUTO = 2, ORC_BLOCK = 3 };
enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_AMG = 1 };

typedef struct orc_opts {
  int32_t graph;             /* ORC_GRAPH_* */
  int32_t method;            /* ORC_LANCZOS, ORC_INVERSE_CG, ORC_AUTO: Lanczos,
                                and inverse iteration from a fresh random start
                                where Lanczos does not converge (Sec. 7), or
                                ORC_BLOCK: block Lanczos of two vectors giving
                                the Fiedler pair (Sec. 9; lanczos_m even >= 4,
                                lanczos_keep even <= lanczos_m - 4) */
  int32_t lanczos_m;         /* Lanczos steps per cycle */
  int32_t max_restarts;      /* cycles after the first one */
  double tol;                /* stop when ||L y - rho y|| <= tol * rho, rho = y^T L y */
  int32_t inv_max_outer;     /* inverse iteration: outer cap */
  int32_t cg_max_iter;       /* CG iteration cap per solve */
  double cg_tol;             /* CG: ||r|| <= cg_tol * ||b|| */
  int32_t cg_full_projection;/* 0: plain CG; k>0: L-orthogonalise each new
                                direction against up to k kept directions */
  uint64_t seed;             /* start-vector seed */
  int32_t lanczos_keep;      /* 0: explicit restart from the Ritz vector; k > 0:
                                thick restart keeping the k smallest Ritz pairs */
  int32_t inv_precond;       /* inverse iteration: ORC_PRECOND_NONE or _AMG */
  int32_t amg_smooth;        /* AMG: damped-Jacobi steps per smoothing phase */
  double amg_sigma;          /* AMG: Jacobi damping weight */
  int32_t fiedler_sweep;     /* Lanczos with thick restart: S > 0 sweeps S angles of
                                the Fiedler pair when it is within sweep_gap */
  double sweep_gap;          /* relative gap (theta2 - theta1) / theta1 of the sweep */
  int32_t warm_start;        /* thick restart: a child's solve starts from its
                                parent's second Ritz vector (plus 0.1 x the
                                random start) */
  int32_t second_solve;      /* fiedler_sweep > 0: the second vector of the swept
                                pair comes from a second Lanczos solve from
                                another random start (seed ^ ORC_SECOND_SEED),
                                so that an exactly degenerate pair is swept;
                                where that pair is not swept, the thick
                                restart's own pair is (as without the option) */
  int32_t lanczos_s;         /* 1: one Lanczos step at a time; 2: from step 3 on,
                                steps j+1 and j+2 from one block [L q_j, L^2 q_j]
                                (two-step Lanczos; the same Krylov space and
                                projected matrix in exact arithmetic) */
  int32_t bfs_start;         /* 1: the first bisection's solve (no parent vector)
                                starts from the graph distance to a pseudo-
                                peripheral element, centred and scaled to unit
                                root-mean-square (plus 0.1 x the random start);
                                elements the search does not reach take the
                                random start.  0: the random start. */
} orc_opts;

#define ORC_SECOND_SEED 0x9E3779B97F4A7C15ull

typedef struct orc_info {
  int32_t cycles;      /* Lanczos cycles (or inverse-iteration outer steps) */
  int32_t converged;   /* 1 if the tolerance was met */
  int64_t matvecs;     /* Laplacian applications */
  double theta;        /* last Ritz value (Lanczos) */
  double residual;     /* ||L y - theta y|| of the returned vector */
  int32_t ncomp;       /* connected components of the graph solved on */
  int32_t cg_iters;    /* inverse iteration: CG steps summed over solves */
  int32_t amg_levels;  /* inverse iteration with AMG: levels of the hierarchy */
  int32_t sweeps;      /* bisections whose Fiedler pair was swept */
  int32_t sweep_moved; /* of those, bisections where an angle other than 0 won */
  int32_t fallbacks;   /* ORC_AUTO: bisections solved by inverse iteration */
} orc_info;

void orc_opts_default(orc_opts *o);

/* Start-vector entry for a global element id: uniform in [-1, 1) from the
 * splitmix64 output for counter gid+1 of the stream started at seed. */
double orc_start_value(uint64_t seed, int64_t gid);

/* Dual graph: off-diagonal CSR, columns ascending.  Two-call protocol: with
 * col == NULL only *nnz_inout is written.  Returns 0, or -1 on bad input,
 * -4 if *nnz_inout is too small. */
int orc_dual_graph(int64_t nelem, int32_t nv, const int64_t *ids, int32_t graph,
                   int64_t *row_ptr, int32_t *col, int32_t *weight, int64_t *nnz_inout);

/* y = L x with L = D - A from the CSR above. */
void orc_laplacian_apply(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *weight, const double *x, double *y);

/* Eigenvalues (ascending) and eigenvectors (columns of V, row-major k x k)
 * of a symmetric k x k matrix A (row-major), cyclic Jacobi. */
void orc_jacobi_eigen(int32_t k, const double *A, double *ev, double *V);

/* Smallest eigenpair of the symmetric tridiagonal matrix with diagonal
 * a[0..k-1] and off-diagonal b[1..k-1] (b[0] ignored), skipping eigenvalues
 * below spurious_thr.  Returns 0 on success. */
int orc_tridiag_smallest(int32_t k, const double *a, const double *b, double spurious_thr,
                         double *theta, double *t);

/* Fiedler pair of the mesh's dual-graph Laplacian.  Returns 0, 2 if the graph
 * is disconnected (then y is the Fiedler vector of the component straddling
 * the median, zero elsewhere), 1 if the iteration did not converge, <0 on
 * error.  y has unit norm and canonical sign. */
int orc_fiedler(int64_t nelem, int32_t nv, const int64_t *ids, const orc_opts *o,
                double *y, double *lambda, orc_info *info);

/* Same on an explicit CSR graph (columns ascending, no diagonal), with
 * global ids gid[i] used for the start vector and tie-breaks. */
int orc_fiedler_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                    const int64_t *gid, const orc_opts *o, double *y, double *lambda,
                    orc_info *info);

/* Block Lanczos of two vectors (method ORC_BLOCK's solver) on a connected
 * CSR graph: y1 (unit norm, canonical sign) and y2 (unit norm, orthogonal to
 * y1; zero when the graph has no second direction) span the pair's plane;
 * theta[0] <= theta[1] are the Ritz values of the pair (theta[1] = +inf
 * without a second direction).  A pair within sweep_gap (fiedler_sweep > 0)
 * is rotated so that y1 is the projection of the random start on its plane.
 * Returns 0 converged, 1 not converged, -1 bad input, -2 disconnected. */
int orc_block_pair(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                   const int64_t *gid, const orc_opts *o, double *y1, double *y2, double *theta,
                   orc_info *info);

/* One inner solve of inverse iteration (Sec. 7, Alg. 2): CG for L x = b on
 * the ones-complement, from x = 0, with the options' cg_tol, cg_max_iter,
 * cg_full_projection and preconditioner (gid[i]: global id of row i, used by
 * the multigrid setup).  Returns the number of CG steps (<0 on bad input).
 * With max_dirs > 0 the first max_dirs search directions p_0, p_1, ... are
 * written row-major to dirs ([max_dirs][n]) and their count to *ndirs. */
int orc_cg_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                 const int64_t *gid, const orc_opts *o, const double *b, double *x,
                 int32_t max_dirs, double *dirs, int32_t *ndirs);

/* Threads for the element loops (when built with OpenMP; otherwise one).
 * nthreads < 1 leaves the setting unchanged.  Returns the thread count in
 * effect. */
int orc_set_threads(int32_t nthreads);

/* The split rule on a given vector: side[i] = 0 for the n_low smallest keys
 * (y_i, gid_i), 1 otherwise. */
int orc_split(int64_t n, const double *y, const int64_t *gid, int64_t n_low, uint8_t *side);

/* Level `level` of the aggregation multigrid hierarchy of a CSR graph (the
 * preconditioner of the inverse-iteration solves, Sec. 7), with gid[i] the
 * global id of row i.  Writes *nlevels and the level's row count *nrows and
 * entry count *nnz; when the arrays are non-NULL also its CSR (row_ptr of
 * nrows + 1, col and weight of nnz entries, columns ascending), the global
 * id carried by every row, and agg[i] = row of level + 1 that row i of this
 * level collapses into (-1 on the coarsest level).  Returns 0, -1 on bad
 * input (level out of range). */
int orc_amg_level(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                  const int64_t *gid, int32_t level, int32_t *nlevels, int64_t *nrows,
                  int64_t *nnz, int64_t *row_ptr_out, int64_t *col_out, int64_t *weight_out,
                  int64_t *gid_out, int64_t *agg);

/* u = M f: one V-cycle of that hierarchy (Sec. 7, Alg. 3). */
int orc_amg_vcycle(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                   const int64_t *gid, double sigma, int32_t nsmooth, const double *f, double *u);

/* y = L x with the weighted Laplacian in gather-scatter form (Sec. 5):
 * A_w = P^T Q Q^T P over the distinct vertex ids of each element,
 * L = diag(A_w 1) - A_w.  Returns 0, -1 on bad input. */
int orc_gs_apply(int64_t nelem, int32_t nv, const int64_t *ids, const double *x, double *y);

/* Cuthill-McKee order of a CSR graph (queue form, from the row farthest
 * from row 0, neighbours appended in increasing index, unreached rows last):
 * order[k] = row placed at position k.  Not part of the paper's method (it
 * stands in for the coordinate pre-sort of the elements).  Returns 0, -1 on
 * bad input. */
/* The start values of bfs_start on a CSR graph (row i = global id i): out[i]
 * = (d_i - mean) / sd, NaN for rows the search does not reach. */
int orc_bfs_start(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                  double *out);

int orc_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col,
                       const int32_t *weight, int32_t *order);

/* Recursive spectral bisection into nparts parts; part[i] in [0, nparts). */
int orc_partition(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts,
                  const orc_opts *o, int32_t *part, orc_info *info);

/* Quality metrics of a partition on the weighted vertex-shared dual graph:
 * out[0] weighted cut (sum of shared-vertex counts across parts),
 * out[1] number of cut element pairs, out[2] max neighbour parts,
 * out[3] mean neighbour parts, out[4] min part size, out[5] max part size. */
int orc_metrics(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts,
                const int32_t *part, double *out);

#ifdef __cplusplus
}
#endif
#endif
