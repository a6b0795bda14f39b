// lanczos.hip -- batched restarted Lanczos with full reorthogonalisation
// (paper Sec. 6) for all segments of a bisection level.
//
// Every segment solves for the smallest eigenpair of its Laplacian restricted
// to the component being cut, orthogonal to the ones vector of that component
// (Sec. 4: L x = lambda x with 1^T x = 0).  Per Lanczos step j of a cycle:
//
//   project: q_j = (w - c u0) s is written to the basis, the Laplacian is
//            applied in difference form (L q)_i = s sum_j w_ij (w_i - w_j),
//            and the partial sums of h = [u0, q_1 .. q_j]^T (L q_j) are
//            written per block;
//   update:  w = L q_j - [u0, Q] h and the partial sums of ||w||^2; alpha_j =
//            h_j, beta_{j+1} = ||w||.  If the norm dropped below 1/sqrt(2) of
//            the three-term-recurrence norm a second Gram-Schmidt pass runs
//            (its launches return at once otherwise).
//
// Each of these streaming launches is followed by a small reduction launch
// (fixed summation order per segment) that finishes the step.  q_{j+1} =
// w / beta_{j+1} is never formed as a separate pass: the next project launch
// reads w and applies the scale.  After m steps (or breakdown) the
// tridiagonal eigenproblem is solved on the device, the Ritz vector y = Q t
// becomes the next start vector and its residual decides convergence.
//
// Precision.  The restart vector Y (the Ritz vector of the previous cycle),
// u0, q_1 and the first residual direction are FP64 in both modes; the
// directions q_2 .. q_m, their work vectors and their SpMVs have type T
// (double, or float with float accumulation).  With T = float the Ritz vector
// y = t_1 q_1 + sum_k t_k q_k is an FP64 vector plus an FP32 correction, so
// each restart gains about the FP32 precision factor and the pair reaches the
// FP64 tolerance; scalars, projections and the tridiagonal solve are FP64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

// Warm start of a child subgraph: weight of the random start added to the
// parent's second Ritz vector.
constexpr double kWarmNoise = 0.1;

// Mixed precision with thick restart: FP32 directions carry rounding errors
// of order u ||L|| (u = 2^-24) into the Lanczos relation, so the residual of
// the FP64 Ritz vector stalls near a multiple of u ||L|| (measured: 0.6 u ||T||
// to within a factor two, from 6.9e-7 lambda on a 60-element box to 4.2e-4
// lambda on a 1M-element mesh).  A segment whose residual has changed by at
// most kStallChange over kStallCycles consecutive cycles, within
// kStallScale u ||T|| (the early cycles of a solve can swing widely above
// that), and has not met the tolerance, switches to FP64 directions.
constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24
constexpr double kStallChange = 0.05;
constexpr int kStallCycles = 2;
constexpr double kStallScale = 64.0;
// Two-step Lanczos: the Cholesky QR's R11^2 = g11 - R01^2 at or below
// kCholRel g11 ends the cycle (R11 would carry a relative error of about
// u / kCholRel from the cancellation)
constexpr double kCholRel = 1e-8;

template <typename T>
struct LzArgs {
  const BlkDev *blk;
  const GrpDev *grp;
  const SegDev *seg;
  SegState *st;
  double *alpha, *beta, *h;         // [nseg][ps]
  double *tvec, *tvals;             // [nseg][nkcap][ps], [nseg][nkcap]
  double *arrow;                    // [nseg][ps]
  double *cdel;                     // [nseg][ps] delayed second-pass coefficients
  int nkcap;
  int keep;                         // 0: explicit restart; k > 0: thick restart
  double *part, *gpart;             // [nblk][ps], [ngrp][ps]
  unsigned *gcnt, *scnt;
  int ps;
  const int64_t *chunk_ptr;
  const uint32_t *cols;
  const uint32_t *pk;  // packed slices (see SellRef)
  const int4 *meta;
  const TileStage *stage;  // LDS staging of the current tiles (null: none)
  const int4 *lmeta;
  const int32_t *root;
  const int32_t *gid;
  double *U0;    // u0 (ones vector of the cut component, normalised)
  double *Q1;    // q_1 of the current cycle
  double *Y;     // restart vector (unnormalised Ritz vector)
  double *Wd;    // FP64 work vector of step 1
  T *V;          // q_k at V + k * vs for k >= 2
  double *K;     // kept Ritz vectors of a thick restart, slot k (2 <= k <= nk) at
                 // K + (k - 2) * vs, FP64 (the basis slots themselves when T = double)
  int64_t vs;
  T *Wt0, *Wt1;  // ping-pong work vectors of steps >= 2
  double *Z1, *Z2;  // two-step Lanczos: L q~_j and L^2 q~_j of the current pair (FP64)
  double2 *Pw;      // two-step Lanczos: the pair's block after projection, (W1, W2) per
                    // row (FP64, interleaved: the next launch gathers both at once)
  int pairs;     // 1: steps j >= 3 run two at a time (thick restart, sliced ELL)
  int m;
  double tol;
  int fp32_stall;     // T = float, thick restart: park a segment whose residual
                      // stalls (it continues with FP64 directions)
  int max_restarts;
  double brk;    // breakdown threshold (relative to ||T||) of the type-T steps
  int32_t *flags;          // [0] active segments after the cycle, [1] last step index
                           // reached in the cycle, [2] most steps run by a segment,
                           // [3] segments stopped at the FP32 switch point (whole level)
  unsigned long long *ctr; // [0] segment steps
  uint64_t seed;
  const int32_t *orig;     // row -> element index of the whole call (-1: padding)
  const double *warm;      // warm start by element (NaN: none), or null
  GsView gs;               // gather-scatter operator (gs.nv > 0) instead of the sliced ELL
  __device__ SellRef sell() const { return {chunk_ptr, cols, pk, meta, stage, lmeta}; }
};

// Vector types of step j: STEP 1 reads Y and works in FP64; STEP 2 reads the
// FP64 work vector and writes type T; STEP 3 (j >= 3) is all type T.
template <typename T, int STEP>
struct StepTypes;
template <typename T>
struct StepTypes<T, 1> {
  using Tin = double;
  using Tw = double;
};
template <typename T>
struct StepTypes<T, 2> {
  using Tin = double;
  using Tw = T;
};
template <typename T>
struct StepTypes<T, 3> {
  using Tin = T;
  using Tw = T;
};

template <typename T, int STEP>
__device__ inline const typename StepTypes<T, STEP>::Tin *step_in(const LzArgs<T> &a, int j) {
  if constexpr (STEP == 1) return a.Y;
  else if constexpr (STEP == 2) return a.Wd;
  else return ((j - 1) & 1) ? a.Wt1 : a.Wt0;
}

template <typename T, int STEP>
__device__ inline typename StepTypes<T, STEP>::Tw *step_out(const LzArgs<T> &a, int j) {
  if constexpr (STEP == 1) return a.Wd;
  else return (j & 1) ? a.Wt1 : a.Wt0;
}

// Does segment S run step j with the one-step launches?  With two-step
// Lanczos only steps 1 and 2, and a first step j0 >= 4 that is even, do
// (pairs start at odd steps j >= 3).
template <typename T>
__device__ inline bool single_step(const LzArgs<T> &a, const SegState &S, int j) {
  return !a.pairs || j < 3 || (j == S.j0 && (j & 1) == 0);
}

// Does segment S run the pair of steps j, j + 1 (j odd, j >= 3)?
__device__ inline bool pair_step(const SegState &S, int j) {
  return S.active && !S.cycle_done && j >= S.j0 && j >= 3 && (j & 1);
}

// v_k^T z over one tile for a wavefront: slices of 64 rows, NSL of them
// (compile-time for full tiles), lane-strided, all loads issued together.
template <int NSL, typename P>
__device__ inline double wave_dot_full(const P *__restrict__ v, const double *zs, int lane) {
  double x[NSL];
#pragma unroll
  for (int t = 0; t < NSL; ++t) x[t] = (double)ld_stream(v + t * kWave);
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < NSL; ++t) acc += x[t] * zs[t * kWave + lane];
  return acc;
}

template <typename P>
__device__ inline double wave_dot_part(const P *__restrict__ v, const double *zs, int lane,
                                       int nsl) {
  double acc = 0.0;
  for (int t = 0; t < nsl; ++t) acc += (double)ld_stream(v + t * kWave) * zs[t * kWave + lane];
  return acc;
}

// Two dot products of v_k with the staged vectors z and q from one read of
// v_k (thick restart: the projection of L q_j and, for the delayed second
// Gram-Schmidt pass, of q_j itself).
template <int NSL, typename P>
__device__ inline void wave_dot2_full(const P *__restrict__ v, const double *zs, const double *qs,
                                      int lane, double &az, double &aq) {
  // slices in batches of 8 loads (fewer live registers than one batch)
  constexpr int NB = NSL < 8 ? NSL : 8;
  az = 0.0;
  aq = 0.0;
#pragma unroll
  for (int t0 = 0; t0 < NSL; t0 += NB) {
    P x[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) x[t] = ld_stream(v + (t0 + t) * kWave);
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      az += (double)x[t] * zs[(t0 + t) * kWave + lane];
      aq += (double)x[t] * qs[(t0 + t) * kWave + lane];
    }
  }
}

template <typename P>
__device__ inline void wave_dot2_part(const P *__restrict__ v, const double *zs, const double *qs,
                                      int lane, int nsl, double &az, double &aq) {
  az = 0.0;
  aq = 0.0;
  for (int t = 0; t < nsl; ++t) {
    const double x = (double)ld_stream(v + t * kWave);
    az += x * zs[t * kWave + lane];
    aq += x * qs[t * kWave + lane];
  }
}

template <int NSL, typename P>
__device__ inline void proj_dot(bool dual, bool full, const P *__restrict__ v, const double *zs,
                                const double *qs, int lane, int nsl, double &az, double &aq) {
  if (dual) {
    if (full) wave_dot2_full<NSL>(v, zs, qs, lane, az, aq);
    else wave_dot2_part(v, zs, qs, lane, nsl, az, aq);
  } else {
    az = full ? wave_dot_full<NSL>(v, zs, lane) : wave_dot_part(v, zs, lane, nsl);
    aq = 0.0;
  }
}

// acc[r] += sum_{k = k0..k1} c_k B[k - kb][row_r] (vectors of stride vs), 4
// vectors per round so that 4 * RPT loads are in flight per thread.
template <typename P, int RPT>
__device__ inline void accumulate_slots(const P *__restrict__ B, int kb, int64_t vs,
                                        const TileRows<RPT> &tr, const double *coef, int k0,
                                        int k1, double (&acc)[RPT]) {
  int k = k0;
  for (; k + 4 <= k1 + 1; k += 4) {
    P v[4][RPT];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int r = 0; r < RPT; ++r) v[kk][r] = ld_stream(B + (int64_t)(k + kk - kb) * vs + tr.row[r]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double ck = coef[k + kk];
#pragma unroll
      for (int r = 0; r < RPT; ++r) acc[r] += (double)v[kk][r] * ck;
    }
  }
  for (; k <= k1; ++k) {
    const double ck = coef[k];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] += (double)B[(int64_t)(k - kb) * vs + tr.row[r]] * ck;
  }
}

// Two combinations from one read: acc[r] += sum a_k B.., acd[r] += sum d_k B..
template <typename P, int RPT>
__device__ inline void accumulate_slots2(const P *__restrict__ B, int kb, int64_t vs,
                                         const TileRows<RPT> &tr, const double *ca,
                                         const double *cd, int k0, int k1, double (&acc)[RPT],
                                         double (&acd)[RPT]) {
  int k = k0;
  for (; k + 4 <= k1 + 1; k += 4) {
    P v[4][RPT];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int r = 0; r < RPT; ++r) v[kk][r] = ld_stream(B + (int64_t)(k + kk - kb) * vs + tr.row[r]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double a = ca[k + kk], d = cd[k + kk];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        acc[r] += (double)v[kk][r] * a;
        acd[r] += (double)v[kk][r] * d;
      }
    }
  }
  for (; k <= k1; ++k) {
    const double a = ca[k], d = cd[k];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double x = (double)B[(int64_t)(k - kb) * vs + tr.row[r]];
      acc[r] += x * a;
      acd[r] += x * d;
    }
  }
}

// acc[r] += sum_{k = 2..k1} c_k b_k[row_r] over the basis slots >= 2: the
// FP64 kept Ritz vectors (2..nk) and the type-T Lanczos vectors after them.
template <typename T, int RPT>
__device__ inline void accumulate_basis(const LzArgs<T> &a, const TileRows<RPT> &tr,
                                        const double *coef, int nk, int k1, double (&acc)[RPT]) {
  const int kk = min(nk, k1);
  if (kk >= 2) accumulate_slots<double, RPT>(a.K, 2, a.vs, tr, coef, 2, kk, acc);
  accumulate_slots<T, RPT>(a.V, 0, a.vs, tr, coef, max(2, kk + 1), k1, acc);
}

template <typename T, int RPT>
__device__ inline void accumulate_basis2(const LzArgs<T> &a, const TileRows<RPT> &tr,
                                         const double *ca, const double *cd, int nk, int k1,
                                         double (&acc)[RPT], double (&acd)[RPT]) {
  const int kk = min(nk, k1);
  if (kk >= 2) accumulate_slots2<double, RPT>(a.K, 2, a.vs, tr, ca, cd, 2, kk, acc, acd);
  accumulate_slots2<T, RPT>(a.V, 0, a.vs, tr, ca, cd, max(2, kk + 1), k1, acc, acd);
}

// ----------------------------------------------------------------------------
// begin: u0 and the hashed random start vector (the Lanczos start; Sec. 7,
// Alg. 2 uses the same kind of start) of every segment with a component to cut.
// ----------------------------------------------------------------------------
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_begin(LzArgs<T> a) {
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.solve) return;
  const TileRows<RPT> tr(b);
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!tr.ok[r]) continue;
    const int64_t row = tr.row[r];
    const bool in = (a.root[row] == S.strad);
    const double u = in ? S.invsqrt_nc : 0.0;
    double x = in ? start_value(a.seed, a.gid[row]) : 0.0;
    if (in && a.warm) {
      // the parent's second Ritz vector, if it had one, plus 0.1 x the random start
      const double v = a.warm[a.orig[row]];
      if (!isnan(v)) x = v + kWarmNoise * x;
    }
    a.U0[row] = u;
    a.Y[row] = x;
    acc[0] += u * x;
    acc[1] += x * x;
  }
  block_reduce_into<2>(acc, red, vals, 2);
  write_partials(a, lb, vals, 2);
}

// ----------------------------------------------------------------------------
// project: MODE 0 = first pass of step j (SpMV of q_j, write q_j);
//          MODE 1 = second Gram-Schmidt pass (project the current w again).
// Phase 1 (RPT rows per thread): the vector z to project is formed and
// staged in LDS.  Phase 2: each wavefront takes every fourth basis vector k
// and reduces v_k^T z over the whole tile with coalesced loads, so no
// block-wide reduction is needed per coefficient.
// ----------------------------------------------------------------------------
// Threads per block of the projection launch: up to 512, so that a thread
// owns few rows (their gathers are not overlapped with each other) while
// the register budget still allows several blocks per compute unit.
template <int RPT>
constexpr int proj_threads() {
  return (kBlock * RPT <= 512) ? kBlock * RPT : 512;
}

template <typename T, int RPT, int MODE, int STEP>
__global__ __launch_bounds__(proj_threads<RPT>()) __attribute__((amdgpu_waves_per_eu(RPT <= 4 ? 6 : 4))) void k_lz_project(LzArgs<T> a, int j) {
  using Tin = typename StepTypes<T, STEP>::Tin;
  using Tw = typename StepTypes<T, STEP>::Tw;
  constexpr int NT = proj_threads<RPT>();
  constexpr int TILE = kBlock * RPT;
  constexpr int RT = TILE / NT;  // rows per thread
  constexpr int NW = NT / kWave;
  constexpr int NSL = TILE / kWave;
  // LDS: the step input staged for the SpMV (FP32 steps j >= 3 of a staged
  // tile), L q_j, q_j and the partial sums of the projection
  constexpr int kStageN = (STEP == 3 && MODE == 0 && sizeof(Tin) == 4) ? kStageCap : 1;
  __shared__ Tin xs[kStageN];
  __shared__ double zs[TILE];
  __shared__ double qs[MODE == 0 ? TILE : 1];
  __shared__ double vals[2 * kMaxM + 8];
  __shared__ double red[NW];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cycle_done || j < S.j0 || !single_step(a, S, j)) return;
  if (MODE == 1 && !S.need2) return;
  const Tin *Win = step_in<T, STEP>(a, j);
  Tw *Wout = step_out<T, STEP>(a, j);
  const double c = S.c, sc = S.s;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const SellRef m = a.sell();
  const bool staged = kStageN > 1 && a.gs.nv == 0 && tile_staged(m, b.row0);
  if (staged) {
    stage_copy(m, b.row0, Win, xs, (int)threadIdx.x, NT);
    __syncthreads();
  }
  int64_t rows[RT];
  bool oks[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int lr = r * NT + (int)threadIdx.x;
    oks[r] = lr < b.nrows;
    rows[r] = b.row0 + (oks[r] ? lr : 0);
  }
  double zz = 0.0;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int64_t row = rows[r];
    double z, q = 0.0;
    if (MODE == 0) {
      const Tin wi = Win[row];
      const double qd = ((double)wi - c * a.U0[row]) * sc;
      const Tin lw = a.gs.nv ? gs_row<Tin>(a.gs, row, wi)
                     : staged ? lap_row<Tin, true>(m, Win, xs, row, wi)
                              : lap_row<Tin, false>(m, Win, nullptr, row, wi);
      const Tw lq = (Tw)(sc * (double)lw);
      if (STEP == 1) {
        q = qd;
        if (oks[r]) a.Q1[row] = qd;
      } else {
        const T qt = (T)qd;
        q = (double)qt;
        if (oks[r]) a.V[(int64_t)j * a.vs + row] = qt;
      }
      if (oks[r]) Wout[row] = lq;
      z = (double)lq;
    } else {
      z = (double)Wout[row];
    }
    if (!oks[r]) z = q = 0.0;
    zs[r * NT + threadIdx.x] = z;
    if (MODE == 0) qs[r * NT + threadIdx.x] = q;
    zz += z * z;
  }
  zz = wave_sum(zz);
  if (lane == 0) red[wave] = zz;
  __syncthreads();
  const bool full = (b.nrows == TILE);
  const int nsl = b.nrows / kWave;
  const bool delayed = (MODE == 0) && a.keep > 0;
  for (int k = wave; k <= j; k += NW) {
    double acc, accq;
    const bool dual = delayed && k < j;
    if (MODE == 0 && k == j) {
      acc = full ? wave_dot_full<NSL>(qs + lane, zs, lane) : wave_dot_part(qs + lane, zs, lane, nsl);
      accq = 0.0;
    } else if (k <= 1) {
      const double *v = (k == 0 ? a.U0 : a.Q1) + b.row0 + lane;
      proj_dot<NSL>(dual, full, v, zs, qs, lane, nsl, acc, accq);
    } else if (k <= S.nk) {
      const double *v = a.K + (int64_t)(k - 2) * a.vs + b.row0 + lane;
      proj_dot<NSL>(dual, full, v, zs, qs, lane, nsl, acc, accq);
    } else {
      const T *v = a.V + (int64_t)k * a.vs + b.row0 + lane;
      proj_dot<NSL>(dual, full, v, zs, qs, lane, nsl, acc, accq);
    }
    acc = wave_sum(acc);
    if (dual) accq = wave_sum(accq);
    if (lane == 0) {
      vals[k] = acc;
      if (dual) vals[j + 2 + k] = accq;
    }
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w];
    vals[j + 1] = s;
  }
  __syncthreads();
  const int nval = delayed ? 2 * j + 2 : j + 2;
  for (int i = threadIdx.x; i < nval; i += NT) a.part[(int64_t)lb * a.ps + i] = vals[i];
}

// ----------------------------------------------------------------------------
// update: w -= [u0, Q] h and the partial sums of ||w||^2.
// ----------------------------------------------------------------------------
template <typename T, int RPT, int PASS, int STEP>
__global__ __launch_bounds__(kBlock) void k_lz_update(LzArgs<T> a, int j) {
  using Tw = typename StepTypes<T, STEP>::Tw;
  __shared__ double red[4];
  __shared__ double vals[2];
  __shared__ double hs[kMaxM + 2];
  __shared__ double cs[PASS == 1 ? kMaxM + 2 : 1];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cycle_done || j < S.j0 || !single_step(a, S, j)) return;
  if (PASS == 2 && !S.need2) return;
  const bool delayed = (PASS == 1) && a.keep > 0;
  const double *hg = a.h + (int64_t)b.seg * a.ps;
  const double *cg = a.cdel + (int64_t)b.seg * a.ps;
  for (int k = threadIdx.x; k <= j; k += kBlock) {
    hs[k] = hg[k];
    if (delayed) cs[k] = (k < j) ? cg[k] : 0.0;
  }
  __syncthreads();
  Tw *Wout = step_out<T, STEP>(a, j);
  const TileRows<RPT> tr(b);
  double acc[RPT];
  if (!delayed) {
    const double h0 = hs[0], h1 = hs[1];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = a.U0[tr.row[r]] * h0 + a.Q1[tr.row[r]] * h1;
    accumulate_basis<T, RPT>(a, tr, hs, S.nk, j, acc);
  } else {
    // w = L q_j - [u0, Q] h as usual, and in the same pass over the basis
    // the second Gram-Schmidt pass of q_j: q_j -= [u0, q_1..q_{j-1}] c
    double acd[RPT];
    const double h0 = hs[0], h1 = hs[1], c0 = cs[0], c1 = cs[1];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const double u = a.U0[tr.row[r]], q1 = a.Q1[tr.row[r]];
      acc[r] = u * h0 + q1 * h1;
      acd[r] = u * c0 + q1 * c1;
    }
    accumulate_basis2<T, RPT>(a, tr, hs, cs, S.nk, j, acc, acd);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (!tr.ok[r]) continue;
      const int64_t row = tr.row[r];
      // (steps run from j0 = nk + 1, so q_j is never a kept slot)
      if (j == 1) a.Q1[row] -= acd[r];
      else a.V[(int64_t)j * a.vs + row] = (T)((double)a.V[(int64_t)j * a.vs + row] - acd[r]);
    }
  }
  double nn[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const Tw zt = (Tw)((double)Wout[tr.row[r]] - acc[r]);
    if (tr.ok[r]) {
      Wout[tr.row[r]] = zt;
      nn[0] += (double)zt * (double)zt;
    }
  }
  block_reduce_into<1>(nn, red, vals, 1);
  write_partials(a, lb, vals, 1);
}

// ----------------------------------------------------------------------------
// Ritz vector y = Q t into Y (FP64; the next start vector) and the partial
// sums of u0^T y and y^T y.
// ----------------------------------------------------------------------------
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_ritz(LzArgs<T> a) {
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  __shared__ double ts[kMaxM + 2];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const int k = S.k;
  // ts[c] = coefficient of basis vector c (c = 1: q_1, ...)
  const double *tg = a.tvec + (int64_t)b.seg * a.ps;
  if (threadIdx.x == 0) ts[0] = 0.0;
  for (int i = threadIdx.x; i < k; i += kBlock) ts[i + 1] = tg[i];
  __syncthreads();
  const TileRows<RPT> tr(b);
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = a.Q1[tr.row[r]] * ts[1];
  accumulate_basis<T, RPT>(a, tr, ts, 0, k, acc);
  double p[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (tr.ok[r]) {
      a.Y[tr.row[r]] = acc[r];
      p[0] += a.U0[tr.row[r]] * acc[r];
      p[1] += acc[r] * acc[r];
    }
  }
  block_reduce_into<2>(p, red, vals, 2);
  write_partials(a, lb, vals, 2);
}

// ----------------------------------------------------------------------------
// residual of the (projected, normalised) Ritz vector in FP64: partial sums
// of ||L y - theta y||^2, y^T L y and y^T y.
// ----------------------------------------------------------------------------
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_residual(LzArgs<T> a) {
  __shared__ double red[4 * 3];
  __shared__ double vals[3];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const double c = S.c, sc = S.s, th = S.theta;
  const TileRows<RPT> tr(b);
  double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double wi = a.Y[row];
    const double y = (wi - c * a.U0[row]) * sc;
    const double ly =
        sc * (a.gs.nv ? gs_row<double>(a.gs, row, wi) : lap_row<double>(a.sell(), a.Y, row, wi));
    const double rr = ly - th * y;
    if (tr.ok[r]) {
      // the normalised Ritz vector is q_1 of a thick-restarted next cycle
      // (an explicitly restarted one forms the same values in its step 1)
      a.Q1[row] = y;
      p[0] += rr * rr;
      p[1] += y * ly;
      p[2] += y * y;
    }
  }
  block_reduce_into<3>(p, red, vals, 3);
  write_partials(a, lb, vals, 3);
}

// ----------------------------------------------------------------------------
// Thick restart: the nnext smallest Ritz vectors y_c = Q t_c.  y_1 goes to Y
// (it is tested for convergence and, normalised, heads the next basis);
// y_c for c >= 2 become the kept slots c of the next cycle, rewritten in
// place, which is safe because each thread reads every basis value of a
// row before it writes that row.  The last residual direction (output of
// step m) is copied to the input buffer of step nnext + 1, where the next
// cycle continues.  The kept vectors are FP64 whatever T is: rounded to
// FP32, their coupling to the next (high-frequency) direction would carry an
// error of order 1e-7 ||L||, large next to the small eigenvalues sought.
// ----------------------------------------------------------------------------
template <typename T, int RPT, int NKB>
__global__ __launch_bounds__(kBlock) void k_lz_ritz_thick(LzArgs<T> a) {
  constexpr int TS = kMaxM + 4;
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  __shared__ double ts[NKB][TS];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const int k = S.k, nv = S.nnext, nkc = S.nk;
  // ts[c][l]: coefficient of basis slot l (1..k) in y_{c+1}; zero elsewhere
  const double *tg = a.tvec + (int64_t)b.seg * a.nkcap * a.ps;
  for (int i = threadIdx.x; i < NKB * TS; i += kBlock) {
    const int c = i / TS, l = i % TS;
    ts[c][l] = (c < nv && l >= 1 && l <= k) ? tg[(int64_t)c * a.ps + l - 1] : 0.0;
  }
  __syncthreads();
  if (S.pair == 3) {
    // two-step Lanczos: the last basis vector is stored before its second
    // Gram-Schmidt pass, q_k = q~_k - sum_{l<k} d_l v_l (slot 0: u0); the
    // Ritz vectors take the pass in their coefficients instead:
    // t_l q_l summed = sum_{l<k} (t_l - t_k d_l) v_l + t_k q~_k
    const double *dg = a.cdel + (int64_t)b.seg * a.ps;
    for (int i = threadIdx.x; i < NKB * k; i += kBlock) {
      const int c = i / k, l = i % k;
      ts[c][l] -= ts[c][k] * dg[l];
    }
    __syncthreads();
  }
  const bool cont = (k == a.m && k >= 2 && nv >= 1);
  const T *csrc = (k & 1) ? a.Wt1 : a.Wt0;          // output of step k >= 2
  T *cdst = (nv & 1) ? a.Wt1 : a.Wt0;               // input of step nv + 1 >= 3
  const bool to_wd = (nv == 1);                     // step 2 reads the FP64 vector
  const TileRows<RPT> tr(b);
  double p[2] = {0.0, 0.0};
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    double acc[NKB];
    const double q1 = a.Q1[row], u0 = a.U0[row];
#pragma unroll
    for (int c = 0; c < NKB; ++c) acc[c] = q1 * ts[c][1] + u0 * ts[c][0];
    // kept FP64 slots 2..nk, then type-T slots (coefficients past k are 0)
    const int kk = min(nkc, k);
    for (int l = 2; l <= kk; l += 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = a.K[(int64_t)(min(l + u, kk) - 2) * a.vs + row];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double vu = (l + u <= kk) ? v[u] : 0.0;
#pragma unroll
        for (int c = 0; c < NKB; ++c) acc[c] += vu * ts[c][l + u];
      }
    }
    for (int l = max(2, kk + 1); l <= k; l += 4) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = a.V[(int64_t)min(l + u, k) * a.vs + row];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double vu = (double)v[u];
#pragma unroll
        for (int c = 0; c < NKB; ++c) acc[c] += vu * ts[c][l + u];
      }
    }
    if (tr.ok[r]) {
      a.Y[row] = acc[0];
      p[0] += a.U0[row] * acc[0];
      p[1] += acc[0] * acc[0];
#pragma unroll
      for (int c = 1; c < NKB; ++c)
        if (c < nv) a.K[(int64_t)(c - 1) * a.vs + row] = acc[c];
      if (cont) {
        if (to_wd) a.Wd[row] = (double)csrc[row];
        else if (cdst != csrc) cdst[row] = csrc[row];
      }
    }
  }
  block_reduce_into<2>(p, red, vals, 2);
  write_partials(a, lb, vals, 2);
}

// ----------------------------------------------------------------------------
// Two-step Lanczos (thick restart, steps j >= 3).  Steps j and j + 1 come
// from one block [L q~_j, L^2 q~_j] (the same Krylov space and projected
// matrix as one step at a time, in exact arithmetic).  Per pair:
//   A: the step input q~_j (after a pair also that pair's first vector
//      q~_{j-1}) is formed and stored; z1 = L q~_j;
//   B: z2 = L z1; per block, the dot products of every basis vector with
//      z1, z2 and with the vectors still waiting for their second
//      Gram-Schmidt pass (q~_j, and after a pair q~_{j-1});
//   reduce: the second-pass coefficients and the projections of z1 and z2
//      on the corrected basis, written on the stored vectors; alpha_j;
//   C: W = [z1, z2] - V H and the second pass of the waiting vectors from
//      one read of the basis; partial sums of the Gram matrix of W;
//   reduce: Cholesky QR W = [q~_{j+1}, q~_{j+2}] R: beta_{j+1} = R00,
//      alpha_{j+1} = R01 / R00 - alpha_j (only q_j of the old basis couples
//      to q_{j+1}), beta_{j+2} = R11 / R00.
// The next pair's A forms q~_{j+1} = W1 / R00 and q~_{j+2} = (W2 - R01
// q~_{j+1}) / R11; after the cycle's last pair the closing launches store
// q~_k, give it its second pass and write the continuation direction.  When
// j = m the pair has one column (step m alone).  The basis is read twice per
// two steps instead of twice per step.
// ----------------------------------------------------------------------------
template <typename T, int RPT>
__global__ __launch_bounds__(proj_threads<RPT>()) void k_lz_pa(LzArgs<T> a, int j) {
  constexpr int NT = proj_threads<RPT>();
  constexpr int TILE = kBlock * RPT;
  constexpr int RT = TILE / NT;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!pair_step(S, j)) return;
  const bool from_pair = S.pair == 1;
  const T *Win = ((j - 1) & 1) ? a.Wt1 : a.Wt0;
  const double s1 = from_pair ? 1.0 / S.r00 : 0.0;
  const double s2 = from_pair ? 1.0 / S.r11 : 0.0;
  const double s3 = from_pair ? -S.r01 / (S.r00 * S.r11) : 0.0;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int lr = r * NT + (int)threadIdx.x;
    const bool ok = lr < b.nrows;
    const int64_t row = b.row0 + (ok ? lr : 0);
    if (from_pair) {
      const double2 wp = a.Pw[row];
      const double w1 = wp.x, w2 = wp.y;
      double l1, l2;
      lap_row2i(a.sell(), a.Pw, row, w1, w2, l1, l2);
      const double qa = w1 * s1;
      const double qb = w2 * s2 + w1 * s3;
      if (ok) {
        a.V[(int64_t)(j - 1) * a.vs + row] = (T)qa;
        a.V[(int64_t)j * a.vs + row] = (T)qb;
        a.Z1[row] = l2 * s2 + l1 * s3;
      }
    } else {
      // (the one-step input: its SpMV in the directions' precision, as the
      // one-step launches take it)
      const T wi = Win[row];
      const double qd = ((double)wi - S.c * a.U0[row]) * S.s;
      const T lw = lap_row<T>(a.sell(), Win, row, wi);
      if (ok) {
        a.V[(int64_t)j * a.vs + row] = (T)qd;
        a.Z1[row] = S.s * (double)lw;
      }
    }
  }
}

// v_k^T q over one tile (wavefront) for a staged q of any type.
template <int NSL, typename P, typename SQ>
__device__ inline double wave_dot1(const P *__restrict__ v, const SQ *q, int lane, int nsl) {
  constexpr int NB = NSL < 8 ? NSL : 8;
  double acc = 0.0;
  for (int t0 = 0; t0 < nsl; t0 += NB) {
    P x[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) x[t] = (t0 + t < nsl) ? ld_stream(v + (t0 + t) * kWave) : (P)0;
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t0 + t < nsl) acc += (double)x[t] * (double)q[(t0 + t) * kWave + lane];
  }
  return acc;
}

// v_k^T of four staged vectors over one tile (wavefront), one read of v_k;
// the vectors staged as two interleaved pairs (one LDS read each).
template <int NSL, typename P, typename SQ2>
__device__ inline void wave_dot4i(const P *__restrict__ v, const double2 *zz, const SQ2 *qq,
                                  int lane, int nsl, double (&acc)[4]) {
  constexpr int NB = NSL < 8 ? NSL : 8;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = 0.0;
  for (int t0 = 0; t0 < nsl; t0 += NB) {
    P x[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) x[t] = (t0 + t < nsl) ? ld_stream(v + (t0 + t) * kWave) : (P)0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int o = (t0 + t) * kWave + lane;
      if (t0 + t < nsl) {
        const double xv = (double)x[t];
        const double2 z = zz[o];
        const SQ2 q = qq[o];
        acc[0] += xv * z.x;
        acc[1] += xv * z.y;
        acc[2] += xv * (double)q.x;
        acc[3] += xv * (double)q.y;
      }
    }
  }
}

// LDS of the B launch: z1 staged for the SpMV (a staged tile), then the four
// vectors of the projection and its partial sums.
template <typename T, int TILE>
constexpr size_t pb_lds_bytes() {
  constexpr size_t stage = (size_t)kStageCap * sizeof(double);
  constexpr size_t proj = (size_t)TILE * (2 * sizeof(double) + 2 * sizeof(T)) +
                          (4 * kMaxM + 8) * sizeof(double);
  return stage > proj ? stage : proj;
}

template <typename T, int RPT>
__global__ __launch_bounds__(proj_threads<RPT>()) __attribute__((amdgpu_waves_per_eu(RPT <= 4 ? 6 : 4))) void k_lz_pb(LzArgs<T> a, int j) {
  constexpr int NT = proj_threads<RPT>();
  constexpr int TILE = kBlock * RPT;
  constexpr int RT = TILE / NT;
  constexpr int NW = NT / kWave;
  constexpr int NSL = TILE / kWave;
  __shared__ __align__(16) char smem[pb_lds_bytes<T, TILE>()];
  using T2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  double *xs = reinterpret_cast<double *>(smem);
  double2 *zz = reinterpret_cast<double2 *>(smem);
  T2 *qq = reinterpret_cast<T2 *>(zz + TILE);
  double *vals = reinterpret_cast<double *>(qq + TILE);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!pair_step(S, j)) return;
  const bool two = j < a.m;
  const bool pend2 = S.pair == 1;
  const SellRef m = a.sell();
  const bool staged = two && tile_staged(m, b.row0);
  if (staged) {
    stage_copy(m, b.row0, a.Z1, xs, (int)threadIdx.x, NT);
    __syncthreads();
  }
  double z1v[RT], z2v[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int lr = r * NT + (int)threadIdx.x;
    const bool ok = lr < b.nrows;
    const int64_t row = b.row0 + (ok ? lr : 0);
    const double z1 = a.Z1[row];
    double z2 = 0.0;
    if (two) {
      z2 = staged ? lap_row<double, true>(m, a.Z1, xs, row, z1)
                  : lap_row<double, false>(m, a.Z1, nullptr, row, z1);
      if (ok) a.Z2[row] = z2;
    }
    z1v[r] = ok ? z1 : 0.0;
    z2v[r] = ok ? z2 : 0.0;
  }
  if (staged) __syncthreads();  // the staged z1 is overwritten below
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int lr = r * NT + (int)threadIdx.x;
    const bool ok = lr < b.nrows;
    const int64_t row = b.row0 + (ok ? lr : 0);
    zz[lr] = make_double2(z1v[r], z2v[r]);
    T2 q;
    q.x = ok ? a.V[(int64_t)j * a.vs + row] : (T)0;
    q.y = (ok && pend2) ? a.V[(int64_t)(j - 1) * a.vs + row] : (T)0;
    qq[lr] = q;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nsl = b.nrows / kWave;
  // vals: [0, j] v_k^T z1 | [j+1, 2j+1] v_k^T z2 | [2j+2, 3j+1] v_k^T q~_j (k < j) |
  //       [3j+2, 4j] v_k^T q~_{j-1} (k < j - 1)
  for (int k = wave; k <= j; k += NW) {
    double acc[4];
    if (k <= 1) {
      const double *v = (k == 0 ? a.U0 : a.Q1) + b.row0 + lane;
      wave_dot4i<NSL>(v, zz, qq, lane, nsl, acc);
    } else if (k <= S.nk) {
      const double *v = a.K + (int64_t)(k - 2) * a.vs + b.row0 + lane;
      wave_dot4i<NSL>(v, zz, qq, lane, nsl, acc);
    } else {
      const T *v = a.V + (int64_t)k * a.vs + b.row0 + lane;
      wave_dot4i<NSL>(v, zz, qq, lane, nsl, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0) {
      vals[k] = acc[0];
      vals[j + 1 + k] = acc[1];
      if (k < j) vals[2 * j + 2 + k] = acc[2];
      if (k < j - 1) vals[3 * j + 2 + k] = acc[3];
    }
  }
  __syncthreads();
  const int nval = 4 * j + 1;
  for (int i = threadIdx.x; i < nval; i += NT) a.part[(int64_t)lb * a.ps + i] = vals[i];
}

// acc_c[r] += sum_k coef_c[k] B[k - kb][row_r] for four coefficient vectors.
template <typename P, int RPT>
__device__ inline void accumulate_slots4(const P *__restrict__ B, int kb, int64_t vs,
                                         const TileRows<RPT> &tr, const double *const *coef,
                                         int k0, int k1, double (&acc)[4][RPT]) {
  for (int k = k0; k <= k1; k += 4) {
    P v[4][RPT];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        v[kk][r] = ld_stream(B + (int64_t)(min(k + kk, k1) - kb) * vs + tr.row[r]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (k + kk > k1) break;
      double cf[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) cf[c] = coef[c][k + kk];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const double x = (double)v[kk][r];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c][r] += x * cf[c];
      }
    }
  }
}

template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_pc(LzArgs<T> a, int j) {
  __shared__ double cs[4][kMaxM + 4];
  __shared__ double red[4 * 3];
  __shared__ double vals[3];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!pair_step(S, j)) return;
  const bool two = j < a.m;
  const bool pend2 = S.pair == 1;
  // coefficient vectors over slots 0..j: g1, g2 (W = z - V g), e (second
  // pass of q~_j), ei (second pass of q~_{j-1}); zero past their ranges
  const double *hg = a.h + (int64_t)b.seg * a.ps;
  const double *cg = a.cdel + (int64_t)b.seg * a.ps;
  for (int k = threadIdx.x; k <= j + 3; k += kBlock) {
    cs[0][k] = (k <= j) ? hg[k] : 0.0;
    cs[1][k] = (two && k <= j) ? hg[j + 1 + k] : 0.0;
    cs[2][k] = (k < j) ? cg[k] : 0.0;
    cs[3][k] = (pend2 && k < j - 1) ? cg[j + k] : 0.0;
  }
  __syncthreads();
  const TileRows<RPT> tr(b);
  double acc[4][RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const double u = a.U0[tr.row[r]], q1 = a.Q1[tr.row[r]];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c][r] = u * cs[c][0] + q1 * cs[c][1];
  }
  const double *coef[4] = {cs[0], cs[1], cs[2], cs[3]};
  const int kk = min(S.nk, j);
  if (kk >= 2) accumulate_slots4<double, RPT>(a.K, 2, a.vs, tr, coef, 2, kk, acc);
  if (j >= max(2, kk + 1)) accumulate_slots4<T, RPT>(a.V, 0, a.vs, tr, coef, max(2, kk + 1), j, acc);
  double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double w1 = a.Z1[row] - acc[0][r];
    const double w2 = two ? a.Z2[row] - acc[1][r] : 0.0;
    if (!tr.ok[r]) continue;
    T *qj = a.V + (int64_t)j * a.vs + row;
    *qj = (T)((double)*qj - acc[2][r]);
    if (pend2) {
      T *qi = a.V + (int64_t)(j - 1) * a.vs + row;
      *qi = (T)((double)*qi - acc[3][r]);
    }
    a.Pw[row] = make_double2(w1, w2);
    p[0] += w1 * w1;
    p[1] += w1 * w2;
    p[2] += w2 * w2;
  }
  block_reduce_into<3>(p, red, vals, 3);
  write_partials(a, lb, vals, 3);
}

// Closing launch of a cycle that ended in a pair (S.pair 1) or in a
// one-column pair (S.pair 2).  With S.pair 1 the last basis vector
// q~_k = W1 / R00 is stored and its dot products with the basis before it
// are summed (its second pass, applied by the Ritz launch through its
// coefficients); the continuation direction (unnormalised, norm
// beta_{k+1}) is written where the Ritz launch expects the output of step k.
template <typename T, int RPT>
__global__ __launch_bounds__(proj_threads<RPT>()) void k_lz_px1(LzArgs<T> a) {
  constexpr int NT = proj_threads<RPT>();
  constexpr int TILE = kBlock * RPT;
  constexpr int RT = TILE / NT;
  constexpr int NW = NT / kWave;
  constexpr int NSL = TILE / kWave;
  __shared__ T qs[TILE];
  __shared__ double vals[kMaxM + 4];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || (S.pair != 1 && S.pair != 2)) return;
  const int k = S.k;
  T *cont = (k & 1) ? a.Wt1 : a.Wt0;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int lr = r * NT + (int)threadIdx.x;
    const bool ok = lr < b.nrows;
    const int64_t row = b.row0 + (ok ? lr : 0);
    T q = (T)0;
    if (S.pair == 1) {
      const double2 wp = a.Pw[row];
      const double w1 = wp.x, w2 = wp.y;
      const double qk = w1 / S.r00;
      q = (T)qk;
      if (ok) {
        a.V[(int64_t)k * a.vs + row] = q;
        cont[row] = (T)((w2 - S.r01 * qk) / S.r00);
      }
    } else if (ok) {
      cont[row] = (T)a.Pw[row].x;
    }
    qs[lr] = ok ? q : (T)0;
  }
  if (S.pair != 1) return;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nsl = b.nrows / kWave;
  for (int kb = wave; kb < k; kb += NW) {
    double acc;
    if (kb <= 1) {
      acc = wave_dot1<NSL>((kb == 0 ? a.U0 : a.Q1) + b.row0 + lane, qs, lane, nsl);
    } else if (kb <= S.nk) {
      acc = wave_dot1<NSL>(a.K + (int64_t)(kb - 2) * a.vs + b.row0 + lane, qs, lane, nsl);
    } else {
      acc = wave_dot1<NSL>(a.V + (int64_t)kb * a.vs + b.row0 + lane, qs, lane, nsl);
    }
    acc = wave_sum(acc);
    if (lane == 0) vals[kb] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += NT) a.part[(int64_t)lb * a.ps + i] = vals[i];
}

// ----------------------------------------------------------------------------
// Gather-scatter operator: the group sums of the vector that the next launch
// multiplies (the step's input, or the Ritz vector for the residual), for
// the groups of the segments that launch works on.
// ----------------------------------------------------------------------------
template <typename T>
__device__ inline bool gs_group_live(const LzArgs<T> &a, int64_t g, int j, bool resid) {
  int sg = a.gs.gseg[g];
  if (a.gs.only_seg >= 0) {
    if (sg != a.gs.only_seg) return false;
    sg = 0;
  }
  const SegState S = a.st[sg];
  return resid ? S.active != 0 : (S.active && !S.cycle_done && j >= S.j0);
}

template <typename T, int STEP>
__global__ __launch_bounds__(kBlock) void k_lz_gsum(LzArgs<T> a, int j) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.gs.ngroups) return;
  const uint32_t p0 = a.gs.gptr[g], p1 = a.gs.gptr[g + 1];
  if (!gs_group_live(a, g, j, false)) return;
  gs_group_sum(a.gs, g, p0, p1, step_in<T, STEP>(a, j));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_gsum_y(LzArgs<T> a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.gs.ngroups) return;
  const uint32_t p0 = a.gs.gptr[g], p1 = a.gs.gptr[g + 1];
  if (!gs_group_live(a, g, 0, true)) return;
  gs_group_sum(a.gs, g, p0, p1, a.Y);
}

inline unsigned gs_grid(const GsView &g) { return (unsigned)((g.ngroups + kBlock - 1) / kBlock); }

// ----------------------------------------------------------------------------
// Reductions and the per-segment logic that finishes each launch above.
// ----------------------------------------------------------------------------
enum LzOp { OP_BEGIN, OP_PROJ0, OP_PROJ1, OP_UPD1, OP_UPD2, OP_RITZ, OP_RESID, OP_PB, OP_PC,
            OP_PX };

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_lz_reduce(LzArgs<T> a, int j) {
  __shared__ double vals[4 * kMaxM + 8];
  const int g = blockIdx.x;
  const GrpDev G = a.grp[g];
  const int s = G.seg;
  // the segment's state and table entry are loaded together with the
  // group's partial sums (a short chain of dependent loads is most of this
  // launch's time); whether the segment takes part is decided after
  const SegState S = a.st[s];
  const SegDev sg = a.seg[s];
  const int nval = (OP == OP_BEGIN || OP == OP_RITZ) ? 2
                   : (OP == OP_PROJ0) ? (a.keep > 0 ? 2 * j + 2 : j + 2)
                   : (OP == OP_PROJ1) ? j + 2
                   : (OP == OP_UPD1 || OP == OP_UPD2) ? 1
                   : (OP == OP_PB) ? 4 * j + 1
                   : (OP == OP_PX) ? max(S.k, 1)
                   : 3;
  group_sums(a, G, vals, nval);
  bool take;
  switch (OP) {
    case OP_BEGIN:
      take = S.solve != 0;
      break;
    case OP_PROJ0:
    case OP_UPD1:
      take = S.active && !S.cycle_done && j >= S.j0 && single_step(a, S, j);
      break;
    case OP_PROJ1:
    case OP_UPD2:
      take = S.active && !S.cycle_done && j >= S.j0 && S.need2 && single_step(a, S, j);
      break;
    case OP_PB:
    case OP_PC:
      take = pair_step(S, j);
      break;
    case OP_PX:
      take = S.active && S.pair == 1;
      break;
    default:
      take = S.active != 0;
      break;
  }
  if (!take) return;
  if (!group_finish(a, g, G, sg, vals, nval)) return;
  double *hs = a.h + (int64_t)s * a.ps;
  if (OP == OP_PB) {
    // Two-step Lanczos, after B.  q~_{j-1} (waiting when the input came from
    // a pair) and q~_j get their second Gram-Schmidt pass:
    //   q_{j-1} = q~_{j-1} - sum_{k<j-1} ci_k v_k,   ci_k = v_k^T q~_{j-1},
    //   q_j = q~_j - sum_{k<j-1} c_k v_k - c_{j-1} q_{j-1},
    // with c_k = v_k^T q~_j and c_{j-1} = q_{j-1}^T q~_j.  z1, z2 are
    // projected on the corrected basis (h) and the combinations are
    // written on the stored vectors (g; e and ei for the corrections).
    __shared__ double sc[5];
    const double *a1 = vals, *a2 = vals + j + 1, *d = vals + 2 * j + 2, *dd = vals + 3 * j + 2;
    const bool pend2 = S.pair == 1;
    if (threadIdx.x == 0) {
      double cjm1 = d[j - 1], h1m = a1[j - 1], h2m = a2[j - 1];
      if (pend2)
        for (int k = 0; k < j - 1; ++k) {
          cjm1 -= dd[k] * d[k];
          h1m -= dd[k] * a1[k];
          h2m -= dd[k] * a2[k];
        }
      double h1j = a1[j], h2j = a2[j];
      for (int k = 0; k < j - 1; ++k) {
        h1j -= d[k] * a1[k];
        h2j -= d[k] * a2[k];
      }
      h1j -= cjm1 * h1m;
      h2j -= cjm1 * h2m;
      sc[0] = cjm1;
      sc[1] = h1m;
      sc[2] = h2m;
      sc[3] = h1j;
      sc[4] = h2j;
    }
    __syncthreads();
    const double cjm1 = sc[0], h1j = sc[3], h2j = sc[4];
    const double g1m = sc[1] - h1j * cjm1, g2m = sc[2] - h2j * cjm1;
    double *cd = a.cdel + (int64_t)s * a.ps;
    for (int k = threadIdx.x; k <= j; k += kBlock) {
      double g1, g2;
      if (k == j) {
        g1 = h1j;
        g2 = h2j;
      } else if (k == j - 1) {
        g1 = g1m;
        g2 = g2m;
        cd[k] = cjm1;
      } else {
        const double ci = pend2 ? dd[k] : 0.0;
        g1 = a1[k] - h1j * d[k] - g1m * ci;
        g2 = a2[k] - h2j * d[k] - g2m * ci;
        cd[k] = d[k] - cjm1 * ci;
        cd[j + k] = ci;
      }
      hs[k] = g1;
      hs[j + 1 + k] = g2;
    }
    if (threadIdx.x == 0) a.alpha[(int64_t)s * a.ps + j - 1] = h1j;
    return;
  }
  if (OP == OP_PX) {
    // closing second pass of the cycle's last vector q~_k
    double *cd = a.cdel + (int64_t)s * a.ps;
    for (int i = threadIdx.x; i < S.k; i += kBlock) cd[i] = vals[i];
    if (threadIdx.x == 0) a.st[s].pair = 3;
    return;
  }
  if (OP == OP_PROJ0 || OP == OP_PROJ1) {
    if (OP == OP_PROJ0 && a.keep > 0) {
      // delayed second pass: q_j = q~_j - sum_{k<j} c_k b_k.  The step must
      // project L q~_j against the corrected q_j, whose coefficient is
      // q_j^T L q~_j = h~_j - sum c_k h_k; expressed on the stored q~_j the
      // other coefficients become h_k - h_j c_k (k < j)
      __shared__ double s_hj;
      if (threadIdx.x == 0) {
        double t = vals[j];
        for (int k = 0; k < j; ++k) t -= vals[j + 2 + k] * vals[k];
        s_hj = t;
      }
      __syncthreads();
      const double hj = s_hj;
      double *cd = a.cdel + (int64_t)s * a.ps;
      for (int k = threadIdx.x; k < j; k += kBlock) {
        const double ck = vals[j + 2 + k];
        cd[k] = ck;
        hs[k] = vals[k] - hj * ck;
      }
      if (threadIdx.x == 0) hs[j] = hj;
    } else {
      for (int k = threadIdx.x; k <= j; k += kBlock) hs[k] = vals[k];
    }
    if (threadIdx.x == 0 && OP == OP_PROJ0) {
      // what one projection pass is expected to leave: ||L q_j||^2 minus the
      // squares of all projections (three-term part, and the couplings to
      // the kept Ritz vectors after a thick restart)
      double h2 = 0.0;
      for (int k = 0; k <= j; ++k) h2 += vals[k] * vals[k];
      a.st[s].lq2 = vals[j + 1] - h2;
    }
    return;
  }
  if (threadIdx.x != 0) return;
  SegState &W = a.st[s];
  if (OP == OP_PC) {
    // Two-step Lanczos, after C: Cholesky QR of W = [W1, W2]
    const double g00 = vals[0], g01 = vals[1], g11 = vals[2];
    double *al = a.alpha + (int64_t)s * a.ps;
    double *be = a.beta + (int64_t)s * a.ps;
    const double alj = al[j - 1];
    const double r00 = sqrt(fmax(g00, 0.0));
    W.tnorm = fmax(W.tnorm, fabs(alj) + r00 + be[j - 1]);
    be[j] = r00;
    W.k = j;
    W.r00 = r00;
    if (j >= a.m) {  // one column (step m alone): W1 continues the next cycle
      W.cycle_done = 1;
      W.pair = 2;
      return;
    }
    if (r00 <= a.brk * W.tnorm) {
      W.cycle_done = 1;
      W.pair = 0;
      return;
    }
    const double r01 = g01 / r00;
    const double r11 = sqrt(fmax(g11 - r01 * r01, 0.0));
    const double al1 = r01 / r00 - alj, b2 = r11 / r00;
    al[j] = al1;
    be[j + 1] = b2;
    W.tnorm = fmax(W.tnorm, fabs(al1) + b2 + r00);
    W.k = j + 1;
    W.r01 = r01;
    W.r11 = r11;
    W.pair = 1;
    // R11^2 = g11 - R01^2 is the difference of two numbers of size g11:
    // below kCholRel g11 (the second column nearly in the span of the first
    // and the basis, the Krylov space exhausted or nearly so) beta_{j+2} is
    // not known to working accuracy, and the cycle ends after step j + 1 as
    // at a breakdown
    if (j + 1 >= a.m || b2 <= a.brk * W.tnorm || g11 - r01 * r01 <= kCholRel * g11)
      W.cycle_done = 1;
    return;
  }
  if (OP == OP_BEGIN || OP == OP_RITZ) {
    const double c = vals[0];
    W.c = c;
    W.s = 1.0 / sqrt(fmax(vals[1] - c * c, 1e-300));
    if (OP == OP_BEGIN) {
      W.active = 1;
      W.k = 0;
      W.j0 = 1;
      W.nk = 0;
      W.nnext = 0;
      W.cycle_done = 0;
      W.need2 = 0;
      W.converged = 0;
      W.refine = 0;
      W.stall = 0;
      W.pair = 0;
      W.restarts = 0;
      W.tnorm = 0.0;
      W.res = 0.0;
      W.cycles = 0;
      W.steps = 0;
    } else {
      const int ran = W.k - W.j0 + 1;  // steps of this cycle
      W.steps += ran;
      atomicAdd(&a.ctr[0], (unsigned long long)ran);
      atomicMax(&a.flags[1], W.k);
      atomicMax(&a.flags[2], ran);
    }
    return;
  }
  if (OP == OP_RESID) {
    const double th = W.theta;
    const double rho = vals[1] / vals[2];
    const double dth = th - rho;
    const double res = sqrt(fmax(vals[0] - dth * dth * vals[2], 0.0));
    const double res_prev = W.res;
    W.res = res;
    W.rho = rho;
    W.cycles += 1;
    bool stop = false;
    if (res <= a.tol * rho) {
      W.converged = 1;
      stop = true;
    } else if (W.restarts >= a.max_restarts) {
      stop = true;
    }
    if (stop) {
      W.active = 0;
      return;
    }
    // FP32 directions stall the residual near a multiple of u ||L||: such a
    // segment is parked, and the level continues it with FP64 directions by
    // an explicit restart from the Ritz vector.  (A thick restart would carry
    // on the relation L y_i = theta_i y_i + s_i q of the kept vectors, which
    // FP32 rounding has broken at about the stall level: the FP64 cycles
    // would not see the error and the residual would not move.)
    bool to_fp64 = false;
    if (a.fp32_stall) {
      const bool flat = res_prev > 0.0 && fabs(res - res_prev) <= kStallChange * res_prev &&
                        res <= kStallScale * kU32 * W.tnorm;
      W.stall = flat ? W.stall + 1 : 0;
      to_fp64 = W.stall >= kStallCycles;
    }
    W.restarts += 1;
    W.cycle_done = 0;
    W.need2 = 0;
    W.pair = 0;
    const double *be = a.beta + (int64_t)s * a.ps;
    const int kc = W.k;
    if (a.keep > 0 && kc == a.m && W.nnext >= 1 && be[kc] > 0.0 && !to_fp64) {
      // thick restart: the kept Ritz pairs head the next basis and the last
      // residual direction w / beta continues it (step nk + 1)
      const int nk = W.nnext;
      double *al = a.alpha + (int64_t)s * a.ps;
      double *bw = a.beta + (int64_t)s * a.ps;
      double *ar = a.arrow + (int64_t)s * a.ps;
      const double *tv = a.tvec + (int64_t)s * a.nkcap * a.ps;
      const double *tl = a.tvals + (int64_t)s * a.nkcap;
      const double bl = be[kc];
      double tn = 0.0;
      for (int i = 0; i < nk; ++i) {
        al[i] = tl[i];
        ar[i] = bl * tv[(int64_t)i * a.ps + kc - 1];
        bw[i + 1] = 0.0;
        tn = fmax(tn, fabs(al[i]) + fabs(ar[i]));
      }
      W.nk = nk;
      W.j0 = nk + 1;
      W.k = nk;
      W.tnorm = tn;
      W.c = 0.0;
      W.s = 1.0 / bl;
      // two-step Lanczos: a cycle starting at an even step >= 4 needs the
      // one-step launches of even steps
      if (a.pairs && !to_fp64 && W.j0 >= 4 && !(W.j0 & 1)) atomicAdd(&a.flags[4], 1);
    } else {
      // explicit restart from the Ritz vector (c, s stay the transform of Y)
      W.nk = 0;
      W.j0 = 1;
      W.k = 0;
      W.tnorm = 0.0;
    }
    if (to_fp64) {
      W.refine = 1;
      W.active = 0;
      atomicAdd(&a.flags[3], 1);
      return;
    }
    atomicAdd(&a.flags[0], 1);
    return;
  }
  // OP_UPD1 / OP_UPD2: finish step j
  const double w2 = vals[0];
  double alpha_j;
  if (OP == OP_UPD1) {
    const double hj = hs[j];
    // immediate second Gram-Schmidt pass when ||w||^2 fell below half of
    // what one pass is expected to leave (cancellation); with thick restart
    // every vector gets its second pass, delayed into the next step
    if (a.keep == 0 && w2 < 0.5 * W.lq2) {
      W.need2 = 1;
      W.alpha_tmp = hj;
      return;
    }
    alpha_j = hj;
  } else {
    alpha_j = W.alpha_tmp + hs[j];
    W.need2 = 0;
  }
  const double beta = sqrt(w2);
  double *al = a.alpha + (int64_t)s * a.ps;
  double *be = a.beta + (int64_t)s * a.ps;
  al[j - 1] = alpha_j;
  const double bprev = (j >= 2) ? be[j - 1] : 0.0;
  W.tnorm = fmax(W.tnorm, fabs(alpha_j) + beta + bprev);
  W.k = j;
  // the FP64 first step breaks down only at FP64 rounding level
  const double brk = (j == 1) ? 1e-12 : a.brk;
  be[j] = beta;  // (beta_{m+1} couples the kept Ritz vectors of a thick restart)
  if (j >= a.m || beta <= brk * W.tnorm) {
    W.cycle_done = 1;
  } else {
    W.c = 0.0;
    W.s = 1.0 / beta;
  }
}

// ----------------------------------------------------------------------------
// Smallest eigenpair of T (Sturm multisection by one wavefront, then inverse
// iteration with partial pivoting by lane 0).  Ritz values below 1e-10 ||T||
// are taken as spurious null modes and skipped.
// ----------------------------------------------------------------------------
__device__ inline int sturm_count(const double *a, const double *b2, int k, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = (i == 0) ? 0.0 : b2[i] / q;
    q = (a[i] - x) - off;
    if (q == 0.0) q = -1e-300;
    cnt += (q < 0.0);
  }
  return cnt;
}

__global__ __launch_bounds__(kWave) void k_trieig(SegState *__restrict__ st,
                                                  const double *__restrict__ alpha,
                                                  const double *__restrict__ beta,
                                                  double *__restrict__ tvec, int ps, int nseg) {
  __shared__ double ad[kMaxM], bd[kMaxM], b2[kMaxM];
  __shared__ double d[kMaxM], u[kMaxM], u2[kMaxM], l[kMaxM], rhs[kMaxM];
  const int s = blockIdx.x;
  if (s >= nseg) return;
  const SegState S = st[s];
  if (!S.active) return;
  const int k = S.k;
  const int lane = threadIdx.x;
  for (int i = lane; i < k; i += kWave) {
    ad[i] = alpha[(int64_t)s * ps + i];
    bd[i] = (i == 0) ? 0.0 : beta[(int64_t)s * ps + i];
    b2[i] = bd[i] * bd[i];
  }
  __syncthreads();
  // Gershgorin bounds
  double lo = 1e300, hi = -1e300;
  for (int i = lane; i < k; i += kWave) {
    double r = (i > 0 ? fabs(bd[i]) : 0.0) + (i + 1 < k ? fabs(bd[i + 1]) : 0.0);
    lo = fmin(lo, ad[i] - r);
    hi = fmax(hi, ad[i] + r);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
  }
  const double thr = 1e-10 * S.tnorm;
  const int c0 = sturm_count(ad, b2, k, thr);
  const int target = std::min(c0 + 1, k);
  lo = fmax(lo, thr);
  hi = hi + 1e-12 * fabs(hi) + 1e-300;
  for (int it = 0; it < 40; ++it) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(kWave + 1);
    const bool ge = sturm_count(ad, b2, k, x) >= target;
    const unsigned long long mask = __ballot(ge);
    const int f = mask ? (__ffsll((unsigned long long)mask) - 1) : kWave;
    const double xf = __shfl(x, f < kWave ? f : 0, kWave);
    const double xp = __shfl(x, f > 0 ? f - 1 : 0, kWave);
    double nlo = (f == 0) ? lo : xp;
    double nhi = (f == kWave) ? hi : xf;
    if (!(nlo < nhi) || (nlo == lo && nhi == hi)) break;
    lo = nlo;
    hi = nhi;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi))) break;
  }
  const double th = 0.5 * (lo + hi);
  if (lane == 0) {
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = fmax(scale, fabs(ad[i]) + (i ? fabs(bd[i]) : 0.0));
    const double tiny = fmax(scale, 1e-300) * 2.220446049250313e-16;
    double *t = tvec + (int64_t)s * ps;
    for (int i = 0; i < k; ++i) rhs[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i < k; ++i) {
        d[i] = ad[i] - th;
        u[i] = (i + 1 < k) ? bd[i + 1] : 0.0;
        u2[i] = 0.0;
        l[i] = (i > 0) ? bd[i] : 0.0;
      }
      for (int i = 0; i + 1 < k; ++i) {
        if (fabs(l[i + 1]) > fabs(d[i])) {
          double tmp;
          tmp = d[i]; d[i] = l[i + 1]; l[i + 1] = tmp;
          tmp = u[i]; u[i] = d[i + 1]; d[i + 1] = tmp;
          tmp = u2[i]; u2[i] = u[i + 1]; u[i + 1] = tmp;
          tmp = rhs[i]; rhs[i] = rhs[i + 1]; rhs[i + 1] = tmp;
        }
        if (d[i] == 0.0) d[i] = tiny;
        const double f = l[i + 1] / d[i];
        d[i + 1] -= f * u[i];
        u[i + 1] -= f * u2[i];
        rhs[i + 1] -= f * rhs[i];
      }
      if (d[k - 1] == 0.0) d[k - 1] = tiny;
      for (int i = k - 1; i >= 0; --i) {
        double v = rhs[i];
        if (i + 1 < k) v -= u[i] * rhs[i + 1];
        if (i + 2 < k) v -= u2[i] * rhs[i + 2];
        rhs[i] = v / d[i];
      }
      double big = 0.0;
      for (int i = 0; i < k; ++i) big = fmax(big, fabs(rhs[i]));
      double nrm = 0.0;
      for (int i = 0; i < k; ++i) {
        rhs[i] /= big;
        nrm += rhs[i] * rhs[i];
      }
      nrm = sqrt(nrm);
      for (int i = 0; i < k; ++i) rhs[i] /= nrm;
    }
    for (int i = 0; i < k; ++i) t[i] = rhs[i];
    st[s].theta = th;
  }
}

// ----------------------------------------------------------------------------
// Thick restart: the nnext smallest eigenpairs, above the spurious-mode
// threshold, of the cycle's projected matrix
//   [ diag(theta_1 .. theta_nk)  s                       ]
//   [ s^T                        alpha_{nk+1}  beta ...   ]
//   [                            beta          tridiagonal]
// (nk = 0: plain tridiagonal).  Eigenvalues: lane c bisects the c-th one
// with Sturm counts from the LDL^T pivots taken in the order kept rows
// first (their pivots are theta_i - x; the next row collects
// -sum s_i^2 / (theta_i - x)).  Eigenvectors: inverse iteration per lane
// with the same elimination order and partial pivoting in the tridiagonal
// part, then modified Gram-Schmidt across the lanes' vectors, which keeps
// the vectors of close Ritz values orthonormal.
// ----------------------------------------------------------------------------
__device__ inline int sturm_arrow(const double *a, const double *b2, const double *s2, int nk,
                                  int k, double x) {
  int cnt = 0;
  double sum = 0.0;
  for (int i = 0; i < nk; ++i) {
    double d = a[i] - x;
    if (d == 0.0) d = -1e-300;
    cnt += (d < 0.0);
    sum += s2[i] / d;
  }
  double q = (a[nk] - x) - sum;
  if (q == 0.0) q = -1e-300;
  cnt += (q < 0.0);
  for (int i = nk + 1; i < k; ++i) {
    q = (a[i] - x) - b2[i] / q;
    if (q == 0.0) q = -1e-300;
    cnt += (q < 0.0);
  }
  return cnt;
}

// MB >= rows of the projected matrix (lanczos_m), KB >= pairs kept: the
// per-lane work arrays take 4 MB KB doubles of LDS, so the bucket decides
// how many segments a compute unit works on at once.
template <int MB, int KB>
__global__ __launch_bounds__(kWave) void k_trieig_arrow(SegState *__restrict__ st,
                                                        const double *__restrict__ alpha,
                                                        const double *__restrict__ beta,
                                                        const double *__restrict__ arrow,
                                                        double *__restrict__ tvec,
                                                        double *__restrict__ tvals, int ps,
                                                        int nkcap, int keep, int nseg) {
  __shared__ double ad[MB], bd[MB], b2[MB], sv[KB], s2[KB];
  // per-lane work of the inverse iteration, [row][lane]
  __shared__ double wd[MB][KB], wu[MB][KB], wu2[MB][KB], wr[MB][KB];
  __shared__ double red[kWave];
  const int seg = blockIdx.x;
  if (seg >= nseg) return;
  const SegState S = st[seg];
  if (!S.active) return;
  const int k = S.k, nk = S.nk;
  const int lane = threadIdx.x;
  for (int i = lane; i < k; i += kWave) {
    ad[i] = alpha[(int64_t)seg * ps + i];
    bd[i] = (i <= nk) ? 0.0 : beta[(int64_t)seg * ps + i];  // bd[i] couples rows i-1, i
    b2[i] = bd[i] * bd[i];
  }
  for (int i = lane; i < nk; i += kWave) {
    sv[i] = arrow[(int64_t)seg * ps + i];
    s2[i] = sv[i] * sv[i];
  }
  __syncthreads();
  // Gershgorin bounds and scale
  double lo = 1e300, hi = -1e300, scale = 0.0;
  double ssum = 0.0;
  for (int i = 0; i < nk; ++i) ssum += fabs(sv[i]);
  for (int i = lane; i < k; i += kWave) {
    double r;
    if (i < nk) r = fabs(sv[i]);
    else if (i == nk) r = ssum + (i + 1 < k ? fabs(bd[i + 1]) : 0.0);
    else r = fabs(bd[i]) + (i + 1 < k ? fabs(bd[i + 1]) : 0.0);
    lo = fmin(lo, ad[i] - r);
    hi = fmax(hi, ad[i] + r);
    scale = fmax(scale, fabs(ad[i]) + r);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
    scale = fmax(scale, __shfl_xor(scale, off, kWave));
  }
  const double thr = 1e-10 * S.tnorm;
  const int c0 = sturm_arrow(ad, b2, s2, nk, k, thr);
  int nv = (keep > 0) ? min(min(keep, k - 1), k - c0) : 1;
  nv = max(1, min(nv, KB));
  const double tiny = fmax(scale, 1e-300) * 2.220446049250313e-16;
  // Multisection: GS lanes per eigenvalue (group c = lane / GS finds the
  // c-th one) each count at one of GS interior points of the group's
  // bracket; the bracket shrinks to the two points around the first count
  // that reaches the target, until no interior point is left.
  constexpr int GS = kWave / KB;
  const int grp = lane / GS, sub = lane % GS;
  double l0 = fmax(lo, thr), h0 = hi + 1e-12 * fabs(hi) + 1e-300;
  {
    const int target = min(c0 + 1 + grp, k);
    bool done = grp >= nv;
    const unsigned long long gm = (((1ull << (GS - 1)) << 1) - 1ull) << (grp * GS);
    for (int it = 0; it < 200; ++it) {
      const double x = l0 + (h0 - l0) * (double)(sub + 1) / (double)(GS + 1);
      // a point rounded onto an end of the bracket takes that end's side
      const bool inside = x > l0 && x < h0;
      const bool ge = inside ? sturm_arrow(ad, b2, s2, nk, k, x) >= target : x >= h0;
      const unsigned long long any_inside = __ballot(inside) & gm;
      const unsigned long long hit = __ballot(ge) & gm;
      // first point of the group whose count reaches the target (all lanes
      // take part in the shuffles)
      const int f = hit ? (__ffsll((unsigned long long)hit) - 1 - grp * GS) : GS;
      const double xf = __shfl(x, grp * GS + (f < GS ? f : 0), kWave);
      const double xp = __shfl(x, grp * GS + (f > 0 ? f - 1 : 0), kWave);
      if (!done) {
        const double nl = (f == 0) ? l0 : xp, nh = (f == GS) ? h0 : xf;
        if (!any_inside || !(nl < nh) || (nl == l0 && nh == h0)) {
          done = true;
        } else {
          l0 = nl;
          h0 = nh;
        }
      }
      if (__ballot(!done) == 0ull) break;
    }
  }
  double th = __shfl(0.5 * (l0 + h0), min(lane, KB - 1) * GS, kWave);
  if (lane < nv) {
    // distinct start vectors per lane (a fixed hash of row and lane), so
    // that close eigenvalues do not start from the same vector
    for (int i = 0; i < k; ++i) {
      uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull + (uint64_t)(lane + 1) * 0xD1B54A32D192ED03ull;
      z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
      z ^= z >> 29;
      wr[i][lane] = 1.0 + 0.5 * ((double)(z >> 11) * 0x1.0p-53);
    }
  }
  __syncthreads();
  // inverse subspace iteration: every lane one shifted solve per sweep,
  // then modified Gram-Schmidt across the lanes' vectors
  for (int it = 0; it < 4; ++it) {
    if (lane < nv) {
      // kept rows eliminated into row nk
      double dn = ad[nk] - th, rn = wr[nk][lane];
      for (int i = 0; i < nk; ++i) {
        double dk = ad[i] - th;
        if (fabs(dk) < tiny) dk = (dk < 0.0) ? -tiny : tiny;
        dn -= s2[i] / dk;
        rn -= sv[i] * wr[i][lane] / dk;
      }
      // tridiagonal rows nk..k-1 with partial pivoting (bands d, u, u2)
      for (int i = nk; i < k; ++i) {
        wd[i][lane] = (i == nk) ? dn : ad[i] - th;
        wu[i][lane] = (i + 1 < k) ? bd[i + 1] : 0.0;
        wu2[i][lane] = 0.0;
      }
      wr[nk][lane] = rn;
      for (int i = nk; i + 1 < k; ++i) {
        double li = bd[i + 1];  // sub-diagonal entry of row i + 1
        if (fabs(li) > fabs(wd[i][lane])) {
          double t;
          t = wd[i][lane]; wd[i][lane] = li; li = t;
          t = wu[i][lane]; wu[i][lane] = wd[i + 1][lane]; wd[i + 1][lane] = t;
          t = wu2[i][lane]; wu2[i][lane] = wu[i + 1][lane]; wu[i + 1][lane] = t;
          t = wr[i][lane]; wr[i][lane] = wr[i + 1][lane]; wr[i + 1][lane] = t;
        }
        if (wd[i][lane] == 0.0) wd[i][lane] = tiny;
        const double f = li / wd[i][lane];
        wd[i + 1][lane] -= f * wu[i][lane];
        wu[i + 1][lane] -= f * wu2[i][lane];
        wr[i + 1][lane] -= f * wr[i][lane];
      }
      if (wd[k - 1][lane] == 0.0) wd[k - 1][lane] = tiny;
      for (int i = k - 1; i >= nk; --i) {
        double v = wr[i][lane];
        if (i + 1 < k) v -= wu[i][lane] * wr[i + 1][lane];
        if (i + 2 < k) v -= wu2[i][lane] * wr[i + 2][lane];
        wr[i][lane] = v / wd[i][lane];
      }
      const double xn = wr[nk][lane];
      for (int i = 0; i < nk; ++i) {
        double dk = ad[i] - th;
        if (fabs(dk) < tiny) dk = (dk < 0.0) ? -tiny : tiny;
        wr[i][lane] = (wr[i][lane] - sv[i] * xn) / dk;
      }
      double big = 0.0;
      for (int i = 0; i < k; ++i) big = fmax(big, fabs(wr[i][lane]));
      for (int i = 0; i < k; ++i) wr[i][lane] /= big;
    }
    __syncthreads();
    for (int c = 0; c < nv; ++c) {
      for (int c2 = 0; c2 < c; ++c2) {
        double d = 0.0;
        for (int i = lane; i < k; i += kWave) d += wr[i][c] * wr[i][c2];
        d = wave_sum(d);
        for (int i = lane; i < k; i += kWave) wr[i][c] -= d * wr[i][c2];
        __syncthreads();
      }
      double nn = 0.0;
      for (int i = lane; i < k; i += kWave) nn += wr[i][c] * wr[i][c];
      nn = wave_sum(nn);
      const double inv = 1.0 / sqrt(fmax(nn, 1e-300));
      for (int i = lane; i < k; i += kWave) wr[i][c] *= inv;
      __syncthreads();
    }
  }
  // Rayleigh-Ritz in the span of the vectors: G = X^T H X (H applied in
  // its arrow form), diagonalised by cyclic Jacobi; the rotated vectors
  // and G's eigenvalues are the Ritz pairs handed on, consistent with each
  // other whatever the spacing of the eigenvalues
  if (lane < nv) {
    double xs = 0.0;  // sum_i s_i x_i over the kept rows
    for (int i = 0; i < nk; ++i) xs += sv[i] * wr[i][lane];
    const double xn = wr[nk][lane];
    for (int i = 0; i < k; ++i) {
      double hx;
      if (i < nk) hx = ad[i] * wr[i][lane] + sv[i] * xn;
      else {
        hx = ad[i] * wr[i][lane];
        if (i == nk) hx += xs;
        else hx += bd[i] * wr[i - 1][lane];
        if (i + 1 < k) hx += bd[i + 1] * wr[i + 1][lane];
      }
      wd[i][lane] = hx;
    }
  }
  __syncthreads();
  __shared__ double G[KB][KB], U[KB][KB], gev[KB];
  if (lane < nv)
    for (int c2 = 0; c2 < nv; ++c2) {
      double g = 0.0;
      for (int i = 0; i < k; ++i) g += wr[i][lane] * wd[i][c2];
      G[lane][c2] = g;
    }
  __syncthreads();
  // cyclic Jacobi on G: every rotation's rows and columns are updated by
  // lane r for entry r (the same arithmetic as one lane taking r in order:
  // the column pass reads the entries before it, the row pass after it)
  if (lane < KB)
    for (int b1 = 0; b1 < KB; ++b1) U[lane][b1] = (lane == b1) ? 1.0 : 0.0;
  __syncthreads();
  if (lane == 0)
    for (int a1 = 0; a1 < nv; ++a1)
      for (int b1 = a1 + 1; b1 < nv; ++b1) G[a1][b1] = G[b1][a1] = 0.5 * (G[a1][b1] + G[b1][a1]);
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int a1 = 0; a1 < nv; ++a1) {
      dia += G[a1][a1] * G[a1][a1];
      for (int b1 = a1 + 1; b1 < nv; ++b1) off += G[a1][b1] * G[a1][b1];
    }
    if (off <= 1e-32 * dia) break;  // the same decision in every lane
    for (int p1 = 0; p1 < nv; ++p1)
      for (int q1 = p1 + 1; q1 < nv; ++q1) {
        const double gpq = G[p1][q1];
        if (gpq == 0.0) continue;
        const double tau = (G[q1][q1] - G[p1][p1]) / (2.0 * gpq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        __syncthreads();  // every lane has read G[p][q], G[p][p], G[q][q]
        if (lane < nv) {
          const double grp = G[lane][p1], grq = G[lane][q1];
          G[lane][p1] = cs * grp - sn * grq;
          G[lane][q1] = sn * grp + cs * grq;
          const double urp = U[lane][p1], urq = U[lane][q1];
          U[lane][p1] = cs * urp - sn * urq;
          U[lane][q1] = sn * urp + cs * urq;
        }
        __syncthreads();
        if (lane < nv) {
          const double gpr = G[p1][lane], gqr = G[q1][lane];
          G[p1][lane] = cs * gpr - sn * gqr;
          G[q1][lane] = sn * gpr + cs * gqr;
        }
        __syncthreads();
      }
  }
  if (lane == 0) {
    // ascending order of the Ritz values (selection sort of the columns)
    for (int a1 = 0; a1 < nv; ++a1) gev[a1] = G[a1][a1];
    for (int a1 = 0; a1 < nv; ++a1) {
      int mn = a1;
      for (int b1 = a1 + 1; b1 < nv; ++b1)
        if (gev[b1] < gev[mn]) mn = b1;
      if (mn != a1) {
        double t = gev[a1]; gev[a1] = gev[mn]; gev[mn] = t;
        for (int r = 0; r < nv; ++r) {
          t = U[r][a1]; U[r][a1] = U[r][mn]; U[r][mn] = t;
        }
      }
    }
  }
  __syncthreads();
  double *tv = tvec + (int64_t)seg * nkcap * ps;
  for (int i = lane; i < k; i += kWave)
    for (int c = 0; c < nv; ++c) {
      double v = 0.0;
      for (int c2 = 0; c2 < nv; ++c2) v += wr[i][c2] * U[c2][c];
      tv[(int64_t)c * ps + i] = v;
    }
  if (lane < nv) tvals[(int64_t)seg * nkcap + lane] = gev[lane];
  if (lane == 0) {
    st[seg].theta = gev[0];
    st[seg].nnext = nv;
  }
  (void)red;
}

// final vector: y = (Y - c u0) s on the component, 0 elsewhere
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_output(LzArgs<T> a, double *__restrict__ y64) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    double y = 0.0;
    if (S.solve) y = (a.Y[row] - S.c * a.U0[row]) * S.s;
    y64[row] = y;
  }
}

// Second Ritz vector of the last thick-restart cycle (kept basis slot 2,
// FP64) on the rows of the component being cut; zero elsewhere and where the
// cycle formed a single Ritz vector.  refined = 0: segments whose last cycle
// ran with these arguments' directions (not continued in FP64); 1: only the
// segments continued with FP64 directions.
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_output2(LzArgs<T> a, double *__restrict__ y2,
                                                       int refined) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if ((S.refine == 2) != (refined != 0)) return;
  const bool have = S.solve && S.nnext >= 2 && a.keep >= 2;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    y2[row] = (have && a.U0[row] != 0.0) ? a.K[row] : 0.0;
  }
}

// Mixed precision: the segments parked at the switch point take part again
// (the FP64 cycles start with an explicit restart from their Ritz vector).
__global__ void k_lz_refine_on(SegState *st, int nseg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg || st[s].refine != 1) return;
  st[s].refine = 2;
  st[s].active = 1;
}

__global__ void k_flags_reset(int32_t *flags) {
  flags[0] = 0;
  flags[1] = 0;
  flags[2] = 0;
  flags[4] = 0;
}

template <int MB, int KB, typename T>
void trieig_arrow_bucket(const LzArgs<T> &a, int nseg, hipStream_t s) {
  k_trieig_arrow<MB, KB><<<nseg, kWave, 0, s>>>(a.st, a.alpha, a.beta, a.arrow, a.tvec, a.tvals,
                                               a.ps, a.nkcap, a.keep, nseg);
}

template <typename T>
void trieig_arrow_launch(const LzArgs<T> &a, int nseg, hipStream_t s) {
  static_assert(kMaxM <= 256 && kMaxKeep <= 16, "tri-eig buckets");
  if (a.m <= 64) {
    if (a.keep <= 8) trieig_arrow_bucket<64, 8>(a, nseg, s);
    else trieig_arrow_bucket<64, 16>(a, nseg, s);
  } else {
    if (a.keep <= 8) trieig_arrow_bucket<256, 8>(a, nseg, s);
    else trieig_arrow_bucket<256, 16>(a, nseg, s);
  }
}

template <typename T, int RPT>
struct LzLaunch {
  static constexpr int kRpt = RPT;
  static void begin(const LzArgs<T> &a, int nblk, int ngrp, hipStream_t s) {
    k_lz_begin<T, RPT><<<nblk, kBlock, 0, s>>>(a);
    k_lz_reduce<T, OP_BEGIN><<<ngrp, kBlock, 0, s>>>(a, 0);
  }
  template <int STEP>
  static void step(const LzArgs<T> &a, int nblk, int ngrp, int j, hipStream_t s,
                   hipEvent_t *ev) {
    if (a.gs.nv) k_lz_gsum<T, STEP><<<gs_grid(a.gs), kBlock, 0, s>>>(a, j);
    if (ev) (void)hipEventRecord(ev[0], s);
    k_lz_project<T, RPT, 0, STEP><<<nblk, proj_threads<RPT>(), 0, s>>>(a, j);
    if (ev) (void)hipEventRecord(ev[1], s);
    k_lz_reduce<T, OP_PROJ0><<<ngrp, kBlock, 0, s>>>(a, j);
    k_lz_update<T, RPT, 1, STEP><<<nblk, kBlock, 0, s>>>(a, j);
    k_lz_reduce<T, OP_UPD1><<<ngrp, kBlock, 0, s>>>(a, j);
    if (a.keep > 0) return;  // thick restart: the second pass is folded into the next step
    k_lz_project<T, RPT, 1, STEP><<<nblk, proj_threads<RPT>(), 0, s>>>(a, j);
    k_lz_reduce<T, OP_PROJ1><<<ngrp, kBlock, 0, s>>>(a, j);
    k_lz_update<T, RPT, 2, STEP><<<nblk, kBlock, 0, s>>>(a, j);
    k_lz_reduce<T, OP_UPD2><<<ngrp, kBlock, 0, s>>>(a, j);
  }
  // two-step Lanczos: steps j and j + 1 (j odd, j >= 3)
  static void pair(const LzArgs<T> &a, int nblk, int ngrp, int j, hipStream_t s,
                   hipEvent_t *ev) {
    k_lz_pa<T, RPT><<<nblk, proj_threads<RPT>(), 0, s>>>(a, j);
    if (ev) (void)hipEventRecord(ev[0], s);
    k_lz_pb<T, RPT><<<nblk, proj_threads<RPT>(), 0, s>>>(a, j);
    if (ev) (void)hipEventRecord(ev[1], s);
    k_lz_reduce<T, OP_PB><<<ngrp, kBlock, 0, s>>>(a, j);
    k_lz_pc<T, RPT><<<nblk, kBlock, 0, s>>>(a, j);
    k_lz_reduce<T, OP_PC><<<ngrp, kBlock, 0, s>>>(a, j);
  }
  // ev: null, or 2*(m+1) events; ev[2j], ev[2j+1] bracket the first-pass
  // project launch of every step j >= 3 (two-step Lanczos: the B launch of
  // the pair starting at odd j).
  // even_singles (two-step Lanczos): also the one-step launches of even
  // steps >= 4, for segments whose cycle starts at such a step
  static void cycle(const LzArgs<T> &a, int nblk, int ngrp, int nseg, hipStream_t s,
                    hipEvent_t *ev = nullptr, bool even_singles = true) {
    k_flags_reset<<<1, 1, 0, s>>>(a.flags);
    for (int j = 1; j <= a.m; ++j) {
      if (a.pairs && j >= 3 && (j & 1)) {
        pair(a, nblk, ngrp, j, s, ev ? ev + 2 * j : nullptr);
        continue;
      }
      if (a.pairs && j >= 4 && !even_singles) continue;
      if (j == 1) step<1>(a, nblk, ngrp, j, s, nullptr);
      else if (j == 2) step<2>(a, nblk, ngrp, j, s, nullptr);
      else step<3>(a, nblk, ngrp, j, s, (ev && !a.pairs) ? ev + 2 * j : nullptr);
    }
    if (a.pairs) {
      // (the second pass of the last vector is applied by the Ritz launch)
      k_lz_px1<T, RPT><<<nblk, proj_threads<RPT>(), 0, s>>>(a);
      k_lz_reduce<T, OP_PX><<<ngrp, kBlock, 0, s>>>(a, 0);
    }
    if (a.keep > 0) {
      trieig_arrow_launch(a, nseg, s);
      if (a.keep <= 4) k_lz_ritz_thick<T, RPT, 4><<<nblk, kBlock, 0, s>>>(a);
      else if (a.keep <= 8) k_lz_ritz_thick<T, RPT, 8><<<nblk, kBlock, 0, s>>>(a);
      else k_lz_ritz_thick<T, RPT, 16><<<nblk, kBlock, 0, s>>>(a);
    } else {
      k_trieig<<<nseg, kWave, 0, s>>>(a.st, a.alpha, a.beta, a.tvec, a.ps, nseg);
      k_lz_ritz<T, RPT><<<nblk, kBlock, 0, s>>>(a);
    }
    k_lz_reduce<T, OP_RITZ><<<ngrp, kBlock, 0, s>>>(a, 0);
    if (a.gs.nv) k_lz_gsum_y<T><<<gs_grid(a.gs), kBlock, 0, s>>>(a);
    k_lz_residual<T, RPT><<<nblk, kBlock, 0, s>>>(a);
    k_lz_reduce<T, OP_RESID><<<ngrp, kBlock, 0, s>>>(a, 0);
  }
  static void output(const LzArgs<T> &a, int nblk, double *y64, hipStream_t s) {
    k_lz_output<T, RPT><<<nblk, kBlock, 0, s>>>(a, y64);
  }
  static void output2(const LzArgs<T> &a, int nblk, double *y2, hipStream_t s, int refined) {
    k_lz_output2<T, RPT><<<nblk, kBlock, 0, s>>>(a, y2, refined);
  }
};

template <typename T, typename F>
void dispatch_rpt(int rpt, F &&f) {
  switch (rpt) {
    case 2: f(LzLaunch<T, 2>()); break;
    case 4: f(LzLaunch<T, 4>()); break;
    case 8: f(LzLaunch<T, 8>()); break;
    default: fail(RSB_EINTERNAL, "unsupported rows-per-thread " + std::to_string(rpt));
  }
}

}  // namespace

void solve_alloc(SolveDev &S, int nseg, int nblk, int ngrp, int m, int keep, Ctx &ctx) {
  S.m = m;
  // partial sums of 2 j + 2 values (delayed second pass), 4 j + 1 (two-step
  // Lanczos), or of the kept directions' coefficients of CG with full
  // projection
  S.pstride = std::max(4 * m + 8, kMaxFullProj);
  S.nkcap = std::max(1, keep);
  const size_t ns = std::max(nseg, 1), nb = std::max(nblk, 1), ng = std::max(ngrp, 1);
  if (!S.st.p || S.st.n < ns) S.st.alloc(ctx, ns);
  S.alpha.alloc(ctx, ns * S.pstride);
  S.beta.alloc(ctx, ns * S.pstride);
  S.h.alloc(ctx, ns * S.pstride);
  S.tvec.alloc(ctx, ns * S.nkcap * S.pstride);
  S.tvals.alloc(ctx, ns * S.nkcap);
  S.arrow.alloc(ctx, ns * S.pstride);
  S.cdel.alloc(ctx, ns * S.pstride);
  S.part.alloc(ctx, nb * S.pstride);
  S.gpart.alloc(ctx, ng * S.pstride);
  S.gcnt.alloc(ctx, ng);
  S.scnt.alloc(ctx, ns);
  S.n_active.alloc(ctx, 8);
  S.counters.alloc(ctx, 4);
  RSB_HIP(hipMemsetAsync(S.gcnt.get(), 0, S.gcnt.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.scnt.get(), 0, S.scnt.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.counters.get(), 0, S.counters.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.beta.get(), 0, S.beta.bytes(), ctx.stream));
}

size_t lanczos_workspace_bytes(int64_t rows, int m, bool fp32, int keep) {
  const size_t t = fp32 ? 4 : 8;
  const size_t kept = (fp32 && keep > 1) ? (size_t)(keep - 1) * 8 : 0;
  // FP64 u0, q1, Y, Wd (+1 spare); type-T basis (m + 1) and work vectors (2);
  // FP64 kept Ritz vectors; the four vectors of a two-step pair
  return (size_t)rows * (5 * 8 + (size_t)(m + 3) * t + kept + 4 * 8);
}

namespace {

// Per-cycle loop of a level (graph per cycle unless profiled); returns the
// level steps run.  Lz is the launcher of the argument type.
template <typename Lz, typename T>
int64_t run_cycles(const LzArgs<T> &a, const LevelView &L, const LanczosParams &p,
                   KernelProfile *profp, Ctx &ctx) {
  const int nblk = L.nblk, nseg = L.nseg, ngrp = L.ngrp;
  int64_t level_steps = 0;
  struct Res {
    hipGraphExec_t exec = nullptr, exec_lean = nullptr;
    hipGraph_t graph = nullptr, graph_lean = nullptr;
    std::vector<hipEvent_t> ev;
    ~Res() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      if (exec_lean) (void)hipGraphExecDestroy(exec_lean);
      if (graph_lean) (void)hipGraphDestroy(graph_lean);
      for (auto e : ev) (void)hipEventDestroy(e);
    }
  } res;
  const bool prof = profp != nullptr;
  if (prof) {
    res.ev.resize(2 * (a.m + 1));
    for (auto &e : res.ev) RSB_HIP(hipEventCreate(&e));
  }
  if (p.use_graph && !prof) {
    // (HIP events recorded by graph nodes cannot be timed: profiled cycles
    // are launched directly)
    RSB_HIP(hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal));
    Lz::cycle(a, nblk, ngrp, nseg, ctx.stream);
    hipError_t e = hipStreamEndCapture(ctx.stream, &res.graph);
    if (e != hipSuccess) fail(RSB_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
    RSB_HIP(hipGraphInstantiate(&res.exec, res.graph, nullptr, nullptr, 0));
    if (a.pairs) {
      RSB_HIP(hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal));
      Lz::cycle(a, nblk, ngrp, nseg, ctx.stream, nullptr, false);
      e = hipStreamEndCapture(ctx.stream, &res.graph_lean);
      if (e != hipSuccess) fail(RSB_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
      RSB_HIP(hipGraphInstantiate(&res.exec_lean, res.graph_lean, nullptr, nullptr, 0));
    }
  }
  // profiled byte count: per segment active in the cycle, its rows for
  // every step it ran (its nonzeros taken in proportion to its rows)
  std::vector<SegState> hst;
  std::vector<SegDev> hseg;
  std::vector<char> was_active;
  std::vector<int64_t> steps0;
  std::vector<int32_t> j00;
  auto read_state = [&]() {
    hst.resize(nseg);
    RSB_HIP(hipMemcpyAsync(hst.data(), a.st, nseg * sizeof(SegState), hipMemcpyDeviceToHost,
                           ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
  };
  if (prof) {
    hseg.resize(nseg);
    RSB_HIP(hipMemcpyAsync(hseg.data(), a.seg, nseg * sizeof(SegDev), hipMemcpyDeviceToHost,
                           ctx.stream));
    was_active.resize(nseg);
    steps0.resize(nseg);
    j00.resize(nseg);
  }
  int32_t flags[5] = {0, 0, 0, 0, 0};
  for (int cyc = 0; cyc <= p.max_restarts; ++cyc) {
    // (the first cycle of a solve starts at step 1 everywhere)
    const bool even_singles = flags[4] > 0;
    if (prof) {
      read_state();
      for (int i = 0; i < nseg; ++i) {
        was_active[i] = hst[i].active != 0;
        steps0[i] = hst[i].steps;
        j00[i] = hst[i].j0;
      }
    }
    if (res.exec) {
      RSB_HIP(hipGraphLaunch((res.exec_lean && !even_singles) ? res.exec_lean : res.exec,
                             ctx.stream));
    } else {
      Lz::cycle(a, nblk, ngrp, nseg, ctx.stream, prof ? res.ev.data() : nullptr, even_singles);
      RSB_LAUNCHED();
    }
    RSB_HIP(hipMemcpyAsync(flags, a.flags, sizeof(flags), hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    level_steps += flags[2];
    if (ctx.verbose >= 3) {
      std::vector<SegState> hv(nseg);
      RSB_HIP(hipMemcpy(hv.data(), a.st, nseg * sizeof(SegState), hipMemcpyDeviceToHost));
      for (int i = 0; i < std::min(nseg, 4); ++i)
        fprintf(stderr, "[rsb]     cycle %d seg %d (%s): k %d res/rho %.3e rho %.12g theta %.12g\n",
                cyc, i, sizeof(T) == 4 ? "fp32" : "fp64", hv[i].k,
                hv[i].res / std::max(hv[i].rho, 1e-300), hv[i].rho, hv[i].theta);
    }
    if (prof) {
      // launches of steps 3..flags[1] were timed; segment i took part in
      // those of steps j0_i..k_i (k_i - j0_i + 1: the steps it added in
      // this cycle); launches that no segment took part in count 0 bytes.
      // A thick-restart cycle starts at j0 = nk + 1 with the kept Ritz
      // vectors in basis slots 2..nk, stored in FP64 whatever T is.
      read_state();
      const double st = (double)sizeof(T);
      // operator bytes per row: the sliced-ELL matrix as read (32-bit
      // words or packed entries), or the gather-scatter slot words, degree
      // and group sums (each group read once)
      const double op_row = L.gs.nv ? 4.0 * L.gs.nv + 4.0 +
                                          8.0 * (double)L.gs.ngroups / (double)std::max<int64_t>(L.nrows, 1)
                                    : matrix_bytes(L) / (double)std::max<int64_t>(L.nrows, 1);
      for (int j = 3; j <= flags[1]; j += a.pairs ? 2 : 1) {
        if (a.pairs && !(j & 1)) continue;
        float ms = 0.f;
        RSB_HIP(hipEventElapsedTime(&ms, res.ev[2 * j], res.ev[2 * j + 1]));
        double rows = 0.0, kept_rows = 0.0;
        for (int i = 0; i < nseg; ++i)
          if (was_active[i] && j >= j00[i] && hst[i].steps - steps0[i] + j00[i] - 1 >= j) {
            rows += (double)hseg[i].npad;
            kept_rows += (double)hseg[i].npad * std::max(0, j00[i] - 2);
          }
        profp->ms += ms;
        profp->launches += 1;
        // one-step: x, q_j and L q_j, u0 and q_1 (FP64), slots 2..j-1;
        // two-step B: z1 read and z2 written (FP64), u0 and q_1, slots 2..j
        profp->bytes += (L.gs.nv ? 0.0 : 4.0 * (rows + 1)) + op_row * rows +
                        (a.pairs ? rows * (8.0 + 8.0 + 16.0 + (j - 1) * st)
                                 : rows * (st + st + st + 16.0 + (j - 2) * st)) +
                        kept_rows * (8.0 - st);
      }
    }
    if (flags[0] == 0) break;
  }
  return level_steps;
}

template <typename T>
LzArgs<T> level_args(const LevelView &L, CompDev &C, SolveDev &S, const LanczosParams &p,
                     void *work) {
  LzArgs<T> a{};
  a.blk = L.blk;
  a.grp = L.grp;
  a.seg = L.seg;
  a.st = S.st.get();
  a.alpha = S.alpha.get();
  a.beta = S.beta.get();
  a.h = S.h.get();
  a.tvec = S.tvec.get();
  a.tvals = S.tvals.get();
  a.arrow = S.arrow.get();
  a.nkcap = S.nkcap;
  a.cdel = S.cdel.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.gcnt = S.gcnt.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.chunk_ptr = L.chunk_ptr;
  a.cols = L.cols;
  a.pk = L.pk;
  a.meta = L.pmeta;
  a.stage = L.stage;
  a.lmeta = L.lmeta;
  a.root = C.root.get();
  a.gid = L.gid;
  a.orig = L.orig;
  a.warm = p.warm;
  a.gs = L.gs;
  // workspace layout: U0, Q1, Y, Wd (FP64), then V (m+1 slots), Wt0, Wt1 (T)
  double *wd = (double *)work;
  a.U0 = wd;
  a.Q1 = wd + L.nrows;
  a.Y = wd + 2 * L.nrows;
  a.Wd = wd + 3 * L.nrows;
  T *wt = (T *)(wd + 4 * L.nrows);
  a.V = wt;
  a.vs = L.nrows;
  a.Wt0 = wt + (int64_t)(p.m + 1) * L.nrows;
  a.Wt1 = a.Wt0 + L.nrows;
  // kept Ritz vectors (FP64): after the work vectors when the directions are
  // FP32, else the basis slots themselves; then the four vectors of a pair
  a.K = sizeof(T) == 8 ? (double *)(a.V + 2 * L.nrows) : (double *)(a.Wt1 + L.nrows);
  // (FP64 whatever T is: the second vector of a pair is formed from the
  // block with a cancellation, W2 - R01 q_{j+1}, that magnifies rounding)
  double *pb = sizeof(T) == 8 ? (double *)(a.Wt1 + L.nrows)
                              : a.K + (int64_t)std::max(p.keep - 1, 0) * L.nrows;
  a.Z1 = pb;
  a.Z2 = pb + L.nrows;
  a.Pw = reinterpret_cast<double2 *>(pb + 2 * L.nrows);
  a.pairs = (p.pairs && p.keep > 0 && L.gs.nv == 0) ? 1 : 0;
  a.m = p.m;
  a.tol = p.tol;
  a.fp32_stall = 0;
  a.max_restarts = p.max_restarts;
  a.brk = sizeof(T) == 4 ? 1e-5 : 1e-12;
  a.keep = p.keep;
  a.flags = S.n_active.get();
  a.ctr = (unsigned long long *)S.counters.get();
  a.seed = p.seed;
  return a;
}

}  // namespace

template <typename T>
int64_t lanczos_level(const LevelView &L, CompDev &C, SolveDev &S, const LanczosParams &p,
                      void *work, double *y64_out, Ctx &ctx) {
  if (L.nseg == 0) return 0;
  if (p.m < 1 || p.m > kMaxM) fail(RSB_EINVAL, "lanczos_m must be in [1, 250]");
  if (p.keep < 0 || p.keep > kMaxKeep || (p.keep > 0 && p.keep >= p.m))
    fail(RSB_EINVAL, "lanczos_keep must be 0 or in [1, min(16, lanczos_m - 1)]");
  if (S.nkcap < std::max(1, p.keep)) fail(RSB_EINTERNAL, "Ritz buffers smaller than lanczos_keep");
  LzArgs<T> a = level_args<T>(L, C, S, p, work);
  // FP32 directions with thick restart: a segment whose residual stalls
  // short of the tolerance continues with FP64 directions until the FP64
  // residual meets it.  Explicit restart needs no switch: its every restart
  // starts from the FP64 Ritz vector and gains the FP32 factor.
  const bool refine = sizeof(T) == 4 && p.keep > 0;
  a.fp32_stall = refine ? 1 : 0;
  const int nblk = L.nblk, ngrp = L.ngrp;
  int64_t level_steps = 0;
  int32_t nref = 0;
  dispatch_rpt<T>(L.rpt, [&](auto launcher) {
    using Lz = decltype(launcher);
    Lz::begin(a, nblk, ngrp, ctx.stream);
    RSB_LAUNCHED();
    if (refine) RSB_HIP(hipMemsetAsync(a.flags + 3, 0, sizeof(int32_t), ctx.stream));
    level_steps += run_cycles<Lz>(a, L, p, p.prof, ctx);
    if (refine) {
      RSB_HIP(hipMemcpyAsync(&nref, a.flags + 3, sizeof(nref), hipMemcpyDeviceToHost, ctx.stream));
      RSB_HIP(hipStreamSynchronize(ctx.stream));
    }
    if (p.y2_out) {
      Lz::output2(a, nblk, p.y2_out, ctx.stream, 0);
      RSB_LAUNCHED();
    }
  });
  if (nref > 0) {
    if constexpr (sizeof(T) == 4) {
      // FP64 directions for the parked segments: u0, q_1, the Ritz vector
      // and the step-1 work vector stay where they are; the basis, the kept
      // Ritz vectors and the work vectors get an FP64 layout of their own
      DevBuf<double> ws2(ctx, (size_t)(p.m + 3 + 4) * (size_t)L.nrows);
      LzArgs<double> d = level_args<double>(L, C, S, p, work);
      d.U0 = a.U0;
      d.Q1 = a.Q1;
      d.Y = a.Y;
      d.Wd = a.Wd;
      d.V = ws2.get();
      d.Wt0 = d.V + (int64_t)(p.m + 1) * L.nrows;
      d.Wt1 = d.Wt0 + L.nrows;
      d.K = d.V + 2 * L.nrows;
      d.Z1 = d.Wt1 + L.nrows;  // (T = double)
      d.Z2 = d.Z1 + L.nrows;
      d.Pw = reinterpret_cast<double2 *>(d.Z2 + L.nrows);
      dispatch_rpt<double>(L.rpt, [&](auto launcher) {
        using Lz = decltype(launcher);
        k_lz_refine_on<<<(L.nseg + kBlock - 1) / kBlock, kBlock, 0, ctx.stream>>>(d.st, L.nseg);
        RSB_LAUNCHED();
        // (the FP64 cycles are not part of the profiled FP32 kernel's count)
        const int64_t s64 = run_cycles<Lz>(d, L, p, nullptr, ctx);
        level_steps += s64;
        ctx.fp64_level_steps += s64;
        if (p.y2_out) {
          Lz::output2(d, nblk, p.y2_out, ctx.stream, 1);
          RSB_LAUNCHED();
        }
      });
      RSB_HIP(hipStreamSynchronize(ctx.stream));  // ws2 is freed on this stream
    }
  }
  if (y64_out) {
    dispatch_rpt<T>(L.rpt, [&](auto launcher) {
      using Lz = decltype(launcher);
      Lz::output(a, nblk, y64_out, ctx.stream);
      RSB_LAUNCHED();
    });
  }
  return level_steps;
}

// Device time of one Lanczos step (the two streaming launches and their
// reductions) at step j = max(3, m / 2) on the level's own matrix, for tile
// selection.  The vectors hold whatever the workspace holds; every segment
// is marked active and the state is restored before each timed repetition.
template <typename T>
double lanczos_trial_ms(const LevelView &L, int m, bool pairs, void *work, Ctx &ctx) {
  if (L.nseg == 0 || L.nblk == 0 || m < 4 || m > kMaxM) return 0.0;
  // a step in the middle of a cycle; the two-step form times the pair that
  // starts there (odd j)
  const int j = pairs ? ((m / 2) | 1) : (m / 2 >= 3 ? m / 2 : 3);
  SolveDev S;
  solve_alloc(S, L.nseg, L.nblk, L.ngrp, m, 0, ctx);
  std::vector<SegState> hs(L.nseg);
  for (auto &x : hs) {
    std::memset(&x, 0, sizeof(x));
    x.active = 1;
    x.solve = 1;
    x.s = 1.0;
    x.tnorm = 1.0;
  }
  DevBuf<SegState> pristine(ctx, L.nseg);
  RSB_HIP(hipMemcpyAsync(pristine.get(), hs.data(), L.nseg * sizeof(SegState),
                         hipMemcpyHostToDevice, ctx.stream));
  RSB_HIP(hipMemsetAsync(S.h.get(), 0, S.h.bytes(), ctx.stream));
  LzArgs<T> a{};
  a.blk = L.blk;
  a.grp = L.grp;
  a.seg = L.seg;
  a.st = S.st.get();
  a.alpha = S.alpha.get();
  a.beta = S.beta.get();
  a.h = S.h.get();
  a.tvec = S.tvec.get();
  a.tvals = S.tvals.get();
  a.arrow = S.arrow.get();
  a.nkcap = S.nkcap;
  a.cdel = S.cdel.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.gcnt = S.gcnt.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.chunk_ptr = L.chunk_ptr;
  a.cols = L.cols;
  a.pk = L.pk;
  a.meta = L.pmeta;
  a.stage = L.stage;
  a.lmeta = L.lmeta;
  a.gs = L.gs;
  double *wd = (double *)work;
  a.U0 = wd;
  a.Q1 = wd + L.nrows;
  a.Y = wd + 2 * L.nrows;
  a.Wd = wd + 3 * L.nrows;
  T *wt = (T *)(wd + 4 * L.nrows);
  a.V = wt;
  a.vs = L.nrows;
  a.Wt0 = wt + (int64_t)(m + 1) * L.nrows;
  a.Wt1 = a.Wt0 + L.nrows;
  // the pair's FP64 vectors where the kept Ritz vectors would start (no
  // kept vectors here; the workspace of the solve holds both)
  double *pv = (double *)(a.Wt1 + L.nrows);
  a.K = pv;
  a.Z1 = pv;
  a.Z2 = pv + L.nrows;
  a.Pw = reinterpret_cast<double2 *>(pv + 2 * L.nrows);
  a.pairs = pairs ? 1 : 0;
  a.m = m;
  a.tol = 1.0;
  a.brk = 0.0;
  a.flags = S.n_active.get();
  a.ctr = (unsigned long long *)S.counters.get();
  const int nblk = L.nblk, ngrp = L.ngrp;
  double total = 0.0;
  dispatch_rpt<T>(L.rpt, [&](auto launcher) {
    (void)launcher;
    constexpr int RPT = decltype(launcher)::kRpt;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RSB_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
      (void)hipEventDestroy(e0);
      fail(RSB_EDEVICE, "hipEventCreate");
    }
    constexpr int kReps = 4;  // the first one is a warm-up
    for (int r = 0; r < kReps && err == hipSuccess; ++r) {
      err = hipMemcpyAsync(a.st, pristine.get(), L.nseg * sizeof(SegState),
                           hipMemcpyDeviceToDevice, ctx.stream);
      if (err != hipSuccess) break;
      (void)hipEventRecord(e0, ctx.stream);
      if (pairs) {
        LzLaunch<T, RPT>::pair(a, nblk, ngrp, j, ctx.stream, nullptr);
      } else {
        if (a.gs.nv) k_lz_gsum<T, 3><<<gs_grid(a.gs), kBlock, 0, ctx.stream>>>(a, j);
        k_lz_project<T, RPT, 0, 3><<<nblk, proj_threads<RPT>(), 0, ctx.stream>>>(a, j);
        k_lz_reduce<T, OP_PROJ0><<<ngrp, kBlock, 0, ctx.stream>>>(a, j);
        k_lz_update<T, RPT, 1, 3><<<nblk, kBlock, 0, ctx.stream>>>(a, j);
        k_lz_reduce<T, OP_UPD1><<<ngrp, kBlock, 0, ctx.stream>>>(a, j);
      }
      (void)hipEventRecord(e1, ctx.stream);
      err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) fail(RSB_EDEVICE, std::string("tile trial: ") + hipGetErrorString(err));
    RSB_LAUNCHED();
    total /= (kReps - 1);
  });
  return total;
}

template double lanczos_trial_ms<float>(const LevelView &, int, bool, void *, Ctx &);
template double lanczos_trial_ms<double>(const LevelView &, int, bool, void *, Ctx &);

template int64_t lanczos_level<float>(const LevelView &, CompDev &, SolveDev &,
                                      const LanczosParams &, void *, double *, Ctx &);
template int64_t lanczos_level<double>(const LevelView &, CompDev &, SolveDev &,
                                       const LanczosParams &, void *, double *, Ctx &);

}  // namespace rsb
