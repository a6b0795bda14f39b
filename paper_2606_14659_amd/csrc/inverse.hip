// inverse.hip -- inverse iteration with conjugate gradients (paper Sec. 7,
// Alg. 2) for all segments of a bisection level, in FP64.
//
// Outer iteration: b <- b - (u0^T b) u0, b <- b / ||b||, solve L x = b, b <- x.
// Inner solver: CG from x0 = 0 whose first search direction is the
// unpreconditioned residual; later directions use the preconditioned
// residual z = M r (the identity, or one aggregation-multigrid V-cycle with
// the u0 component removed) and the flexible (Polak-Ribiere) beta
// z_new^T (r_new - r_old) / z_old^T r_old.  The outer loop stops when a solve
// needed a single CG step (b was an eigenvector, the stopping rule of
// Sec. 7) or when the Rayleigh-quotient residual of b meets the tolerance,
// or after max_outer iterations.  Every launch covers all segments of the
// level; reductions are fixed-order per segment as in the Lanczos solver.
//
// Full projection (the paper's flexible CG "augmented with full
// projection"): each new direction q = z + beta p_old is L-orthogonalised
// against the last k directions P_i, p = q - sum_i c_i P_i with
// c_i = (L P_i)^T q / P_i^T L P_i (classical Gram-Schmidt in the L inner
// product, all c_i from q).  The kept P_i and L P_i sit in a ring of k
// slots per row; L p = L q - sum_i c_i L P_i, so the SpMV of the fused
// direction launch is unchanged and the projection only adds row-local
// reads.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

struct InvArgs {
  const BlkDev *blk;
  const GrpDev *grp;
  const SegDev *seg;
  SegState *st;
  double *part, *gpart;
  unsigned *gcnt, *scnt;
  int ps;
  const int64_t *chunk_ptr;
  const uint32_t *cols;
  const uint32_t *pk;  // packed slices (see SellRef)
  const int4 *meta;
  const int32_t *root;
  const int32_t *gid;
  double *U0, *B, *X, *R, *P0, *P1, *LP;
  double *ROLD;             // previous residual (preconditioned CG)
  const double *Z;          // V-cycle output M r (preconditioned CG)
  int pre;                  // 1: AMG preconditioner
  double cg_tol, tol;
  int max_outer, cg_max_iter;
  int32_t *flags;           // [0] segments still running (CG or outer)
  unsigned long long *ctr;  // [0] segment CG steps
  uint64_t seed;
  int fpk;                  // full projection: ring slots (0: off)
  double *FP, *FLP;         // [fpk][vs] kept directions and their Laplacian
  int64_t vs;               // row stride of the ring
  double *fp_plp, *fp_c;    // [nseg][fpk] P_i^T L P_i, coefficients c_i
  int32_t *fp_tot;          // [nseg] directions pushed in the current solve
};

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_inv_begin(InvArgs a) {
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
    const double x = in ? start_value(a.seed, a.gid[row]) : 0.0;
    a.U0[row] = u;
    a.B[row] = x;
    acc[0] += u * x;
    acc[1] += x * x;
  }
  block_reduce_into<2>(acc, red, vals, 2);
  write_partials(a, lb, vals, 2);
}

// x = 0, r = b_hat = (b - c u0) s, p_old = 0; partial sums of r^T r.
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_cg_init(InvArgs a) {
  __shared__ double red[4];
  __shared__ double vals[1];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const TileRows<RPT> tr(b);
  double acc[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double rv = (a.B[row] - S.c * a.U0[row]) * S.s;
    if (tr.ok[r]) {
      a.R[row] = rv;
      a.X[row] = 0.0;
      a.P1[row] = 0.0;
      acc[0] += rv * rv;
    }
  }
  block_reduce_into<1>(acc, red, vals, 1);
  write_partials(a, lb, vals, 1);
}

// p_new = r + beta p_old (rows) and L p_new (gathers r and p_old); partial
// sums of p^T L p.
// z = r (identity, or the first direction of a solve) or z = Z - c u0.
template <int RPT, bool PRE>
__global__ __launch_bounds__(kBlock) void k_cg_a(InvArgs a, int it) {
  __shared__ double red[4];
  __shared__ double vals[1];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cg_done) return;
  const double *Pold = (it & 1) ? a.P0 : a.P1;
  double *Pnew = (it & 1) ? a.P1 : a.P0;
  const double beta = S.cg_beta;
  const bool use_z = PRE && S.cg_it > 0;
  const double cz = S.cg_c;
  const TileRows<RPT> tr(b);
  double acc[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double zi = use_z ? a.Z[row] - cz * a.U0[row] : a.R[row];
    const double pi = zi + beta * Pold[row];
    const int64_t c = row >> 6;
    const int lane = (int)(row & 63);
    const int64_t p = a.chunk_ptr[c];
    const int width = (int)((a.chunk_ptr[c + 1] - p) >> 6);
    const uint32_t *cp = a.cols + p + lane;
    double lp = 0.0;
    // unconditional loads of a whole slot group, masked as in lap_row
    for (int k0 = 0; k0 < width; k0 += kSlotGroup) {
      uint32_t w[kSlotGroup];
#pragma unroll
      for (int u = 0; u < kSlotGroup; ++u) w[u] = cp[(int64_t)(k0 + u) * 64];
#pragma unroll
      for (int u = 0; u < kSlotGroup; ++u) w[u] = (k0 + u < width) ? w[u] : 0u;
      double rj[kSlotGroup], pj[kSlotGroup];
#pragma unroll
      for (int u = 0; u < kSlotGroup; ++u) {
        const uint32_t j = colw_col(w[u]);
        rj[u] = use_z ? a.Z[j] - cz * a.U0[j] : a.R[j];
        pj[u] = Pold[j];
      }
#pragma unroll
      for (int u = 0; u < kSlotGroup; ++u)
        lp += colw_wt(w[u]) ? (double)colw_wt(w[u]) * (pi - (rj[u] + beta * pj[u])) : 0.0;
    }
    double pf = pi, lf = lp;
    if (a.fpk) {
      const int nk = min(a.fp_tot[b.seg], a.fpk);
      const double *cf = a.fp_c + (int64_t)b.seg * a.fpk;
      for (int k = 0; k < nk; ++k) {
        pf -= cf[k] * a.FP[(int64_t)k * a.vs + row];
        lf -= cf[k] * a.FLP[(int64_t)k * a.vs + row];
      }
    }
    if (tr.ok[r]) {
      Pnew[row] = pf;
      a.LP[row] = lf;
      acc[0] += pf * lf;
    }
  }
  block_reduce_into<1>(acc, red, vals, 1);
  write_partials(a, lb, vals, 1);
}

// Full projection, before the direction launch: partial sums of
// (L P_i)^T q over the kept slots i, q = z + beta p_old.  The tile's q is
// staged in LDS and each wave reduces every fourth slot over the tile.
template <int RPT, bool PRE>
__global__ __launch_bounds__(kBlock) void k_cg_fpdots(InvArgs a, int it) {
  constexpr int TILE = kBlock * RPT;
  __shared__ double qs[TILE];
  __shared__ double vals[kMaxFullProj];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cg_done) return;
  const int nk = min(a.fp_tot[b.seg], a.fpk);
  if (nk == 0) return;
  const double *Pold = (it & 1) ? a.P0 : a.P1;
  const double beta = S.cg_beta;
  const bool use_z = PRE && S.cg_it > 0;
  const double cz = S.cg_c;
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + (int)threadIdx.x;
    double q = 0.0;
    if (lr < b.nrows) {
      const int64_t row = b.row0 + lr;
      const double zi = use_z ? a.Z[row] - cz * a.U0[row] : a.R[row];
      q = zi + beta * Pold[row];
    }
    qs[lr] = q;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int k = wave; k < nk; k += kBlock / kWave) {
    const double *v = a.FLP + (int64_t)k * a.vs + b.row0;
    double acc = 0.0;
    for (int i = lane; i < b.nrows; i += kWave) acc += v[i] * qs[i];
    acc = wave_sum(acc);
    if (lane == 0) vals[k] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nk; i += kBlock) a.part[(int64_t)lb * a.ps + i] = vals[i];
}

// x += alpha p; r -= alpha L p; partial sums of r_new^T r_new, r_new^T r_old.
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_cg_b(InvArgs a, int it) {
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cg_done) return;
  const double *Pnew = (it & 1) ? a.P1 : a.P0;
  const double alpha = S.cg_alpha;
  const TileRows<RPT> tr(b);
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double xn = a.X[row] + alpha * Pnew[row];
    const double rold = a.R[row];
    const double rnew = rold - alpha * a.LP[row];
    if (tr.ok[r]) {
      a.X[row] = xn;
      a.R[row] = rnew;
      if (a.pre) a.ROLD[row] = rold;
      if (a.fpk) {
        // this step's direction joins the kept ones (oldest slot reused)
        const int64_t slot = a.fp_tot[b.seg] % a.fpk;
        a.FP[slot * a.vs + row] = Pnew[row];
        a.FLP[slot * a.vs + row] = a.LP[row];
      }
      acc[0] += rnew * rnew;
      acc[1] += rnew * rold;
    }
  }
  block_reduce_into<2>(acc, red, vals, 2);
  write_partials(a, lb, vals, 2);
}

// Preconditioned CG, after the V-cycle Z = M r: partial sums of u0^T Z,
// Z^T r, Z^T r_old, u0^T r and u0^T r_old (the u0 component of Z is removed
// in the finisher's formulas and in the next direction).
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_cg_z(InvArgs a) {
  __shared__ double red[4 * 5];
  __shared__ double vals[5];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cg_done) return;
  const TileRows<RPT> tr(b);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!tr.ok[r]) continue;
    const int64_t row = tr.row[r];
    const double z = a.Z[row], u = a.U0[row], rn = a.R[row], ro = a.ROLD[row];
    acc[0] += u * z;
    acc[1] += z * rn;
    acc[2] += z * ro;
    acc[3] += u * rn;
    acc[4] += u * ro;
  }
  block_reduce_into<5>(acc, red, vals, 5);
  write_partials(a, lb, vals, 5);
}

// After a solve: partial sums for the transform of the new b = x (c, s) and
// the shift estimate theta = x_hat^T b_hat / x_hat^T x_hat (L x ~ b_hat).
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_inv_eval(InvArgs a) {
  __shared__ double red[4 * 3];
  __shared__ double vals[3];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const TileRows<RPT> tr(b);
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!tr.ok[r]) continue;
    const int64_t row = tr.row[r];
    const double x = a.X[row];
    const double bh = (a.B[row] - S.c * a.U0[row]) * S.s;
    a.B[row] = x;  // the next b (row-local: read before write)
    acc[0] += a.U0[row] * x;
    acc[1] += x * x;
    acc[2] += x * bh;
  }
  block_reduce_into<3>(acc, red, vals, 3);
  write_partials(a, lb, vals, 3);
}

// Partial sums of the Rayleigh-quotient residual of the normalised new b.
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_inv_res(InvArgs a) {
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
    const double xi = a.X[row];
    const double y = (xi - c * a.U0[row]) * sc;
    const double ly = sc * lap_row<double>(SellRef{a.chunk_ptr, a.cols, a.pk, a.meta, nullptr, nullptr}, a.X, row, xi);
    const double rr = ly - th * y;
    if (tr.ok[r]) {
      p[0] += rr * rr;
      p[1] += y * ly;
      p[2] += y * y;
    }
  }
  block_reduce_into<3>(p, red, vals, 3);
  write_partials(a, lb, vals, 3);
}

// Reductions and the per-segment logic that finishes each launch above.
enum InvOp { OP_BEGIN, OP_CG_INIT, OP_CG_A, OP_CG_B, OP_CG_Z, OP_EVAL, OP_RES, OP_CG_FP };

template <int OP>
__global__ __launch_bounds__(kBlock) void k_inv_reduce(InvArgs a) {
  __shared__ double vals[OP == OP_CG_FP ? kMaxFullProj : 5];
  const int g = blockIdx.x;
  const int s = a.grp[g].seg;
  const SegState S = a.st[s];
  int nval;
  switch (OP) {
    case OP_BEGIN:
      if (!S.solve) return;
      nval = 2;
      break;
    case OP_CG_INIT:
      if (!S.active) return;
      nval = 1;
      break;
    case OP_CG_A:
      if (!S.active || S.cg_done) return;
      nval = 1;
      break;
    case OP_CG_B:
      if (!S.active || S.cg_done) return;
      nval = 2;
      break;
    case OP_CG_Z:
      if (!S.active || S.cg_done) return;
      nval = 5;
      break;
    case OP_CG_FP:
      if (!S.active || S.cg_done) return;
      nval = min(a.fp_tot[s], a.fpk);
      if (nval == 0) return;
      break;
    default:
      if (!S.active) return;
      nval = 3;
      break;
  }
  if (!group_reduce(a, g, vals, nval)) return;
  if (OP == OP_CG_FP) {
    const double *pl = a.fp_plp + (int64_t)s * a.fpk;
    double *cf = a.fp_c + (int64_t)s * a.fpk;
    for (int k = threadIdx.x; k < nval; k += kBlock) cf[k] = vals[k] / pl[k];
    return;
  }
  if (threadIdx.x != 0) return;
  SegState &W = a.st[s];
  switch (OP) {
    case OP_BEGIN:
      W.c = vals[0];
      W.s = 1.0 / sqrt(fmax(vals[1] - vals[0] * vals[0], 1e-300));
      W.active = 1;
      W.converged = 0;
      W.cycles = 0;
      W.steps = 0;
      W.theta = 0.0;
      break;
    case OP_CG_INIT:
      if (a.fpk) a.fp_tot[s] = 0;
      W.rr = vals[0];
      W.cg_it = 0;
      W.cg_c = 0.0;
      W.cg_done = (sqrt(vals[0]) <= a.cg_tol) ? 1 : 0;
      W.cg_beta = 0.0;
      break;
    case OP_CG_A:
      W.cg_alpha = W.rr / vals[0];
      if (a.fpk) a.fp_plp[(int64_t)s * a.fpk + a.fp_tot[s] % a.fpk] = vals[0];
      break;
    case OP_CG_B: {
      if (a.fpk) a.fp_tot[s] += 1;
      W.cg_it += 1;
      W.steps += 1;
      atomicAdd(&a.ctr[0], 1ull);
      const double rr = vals[0];
      if (sqrt(rr) <= a.cg_tol || W.cg_it >= a.cg_max_iter) {
        W.cg_done = 1;
      } else {
        if (!a.pre) {
          W.cg_beta = (rr - vals[1]) / W.rr;
          W.rr = rr;
        }
        atomicAdd(&a.flags[0], 1);
      }
      break;
    }
    case OP_CG_Z: {
      // z = Z - c u0; z^T r and z^T r_old with the u0 part taken out
      const double c = vals[0];
      const double zr = vals[1] - c * vals[3];
      const double zro = vals[2] - c * vals[4];
      W.cg_c = c;
      W.cg_beta = (zr - zro) / W.rr;
      W.rr = zr;
      break;
    }
    case OP_EVAL: {
      const double c = vals[0];
      const double xx = fmax(vals[1] - c * c, 1e-300);
      W.c = c;
      W.s = 1.0 / sqrt(xx);
      W.theta = vals[2] / xx;  // (u0^T b_hat = 0)
      break;
    }
    default: {
      const double th = W.theta;
      const double rho = vals[1] / vals[2];
      const double dth = th - rho;
      const double res = sqrt(fmax(vals[0] - dth * dth * vals[2], 0.0));
      W.res = res;
      W.rho = rho;
      W.cycles += 1;
      if (W.cg_it <= 1 || res <= a.tol * rho) {
        W.converged = 1;
        W.active = 0;
      } else if (W.cycles >= a.max_outer) {
        W.active = 0;
      } else {
        atomicAdd(&a.flags[0], 1);
      }
      break;
    }
  }
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_inv_output(InvArgs a, double *__restrict__ y64) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    y64[row] = S.solve ? (a.B[row] - S.c * a.U0[row]) * S.s : 0.0;
  }
}

__global__ void k_flag_reset(int32_t *flags) { flags[0] = 0; }

constexpr int kCgChunk = 16;  // CG steps per captured graph (even: keeps p parity)

template <int RPT>
int64_t inverse_impl(const LevelView &L, CompDev &C, SolveDev &S, const InverseParams &p,
                     void *work, double *y64_out, bool use_graph, Ctx &ctx) {
  InvArgs a{};
  a.blk = L.blk;
  a.grp = L.grp;
  a.seg = L.seg;
  a.st = S.st.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.gcnt = S.gcnt.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.chunk_ptr = L.chunk_ptr;
  a.cols = L.cols;
  a.pk = L.pk;
  a.meta = L.pmeta;
  a.root = C.root.get();
  a.gid = L.gid;
  double *w = (double *)work;
  a.U0 = w;
  a.B = w + L.nrows;
  a.X = w + 2 * L.nrows;
  a.R = w + 3 * L.nrows;
  a.P0 = w + 4 * L.nrows;
  a.P1 = w + 5 * L.nrows;
  a.LP = w + 6 * L.nrows;
  a.ROLD = w + 7 * L.nrows;
  a.pre = (p.precond == RSB_PRECOND_AMG) ? 1 : 0;
  a.cg_tol = p.cg_tol;
  a.tol = p.tol;
  a.max_outer = p.max_outer;
  a.cg_max_iter = p.cg_max_iter;
  a.flags = S.n_active.get();
  a.ctr = (unsigned long long *)S.counters.get();
  a.seed = p.seed;
  a.fpk = p.full_projection;
  a.vs = L.nrows;
  DevBuf<double> fp_plp, fp_c;
  DevBuf<int32_t> fp_tot;
  if (a.fpk) {
    a.FP = w + 8 * L.nrows;
    a.FLP = a.FP + (int64_t)a.fpk * L.nrows;
    fp_plp.alloc(ctx, (size_t)L.nseg * a.fpk);
    fp_c.alloc(ctx, (size_t)L.nseg * a.fpk);
    fp_tot.alloc(ctx, L.nseg);
    fill_i32(fp_tot.get(), L.nseg, 0, ctx);
    a.fp_plp = fp_plp.get();
    a.fp_c = fp_c.get();
    a.fp_tot = fp_tot.get();
  }
  const int nblk = L.nblk, ngrp = L.ngrp;
  hipStream_t s = ctx.stream;
  AmgDev amg;
  if (a.pre) {
    amg.sigma = p.amg_sigma;
    amg.nsmooth = p.amg_smooth;
    amg_setup(L, C.root.get(), a.st, amg, ctx);
    a.Z = amg_result(amg);
    if (p.amg_levels) *p.amg_levels = std::max(*p.amg_levels, (int)amg.lv.size());
  }
  k_inv_begin<RPT><<<nblk, kBlock, 0, s>>>(a);
  k_inv_reduce<OP_BEGIN><<<ngrp, kBlock, 0, s>>>(a);
  RSB_LAUNCHED();
  int64_t steps = 0;
  int32_t flags = 0;
  auto read_flags = [&]() {
    RSB_HIP(hipMemcpyAsync(&flags, a.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RSB_HIP(hipStreamSynchronize(s));
  };
  for (int outer = 0; outer < p.max_outer; ++outer) {
    k_cg_init<RPT><<<nblk, kBlock, 0, s>>>(a);
    k_inv_reduce<OP_CG_INIT><<<ngrp, kBlock, 0, s>>>(a);
    RSB_LAUNCHED();
    // CG chunks, each as one graph launch (or direct launches)
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    auto chunk = [&]() {
      k_flag_reset<<<1, 1, 0, s>>>(a.flags);
      for (int it = 0; it < kCgChunk; ++it) {
        if (a.fpk) {
          if (a.pre) k_cg_fpdots<RPT, true><<<nblk, kBlock, 0, s>>>(a, it);
          else k_cg_fpdots<RPT, false><<<nblk, kBlock, 0, s>>>(a, it);
          k_inv_reduce<OP_CG_FP><<<ngrp, kBlock, 0, s>>>(a);
        }
        if (a.pre) k_cg_a<RPT, true><<<nblk, kBlock, 0, s>>>(a, it);
        else k_cg_a<RPT, false><<<nblk, kBlock, 0, s>>>(a, it);
        k_inv_reduce<OP_CG_A><<<ngrp, kBlock, 0, s>>>(a);
        k_cg_b<RPT><<<nblk, kBlock, 0, s>>>(a, it);
        k_inv_reduce<OP_CG_B><<<ngrp, kBlock, 0, s>>>(a);
        if (a.pre) {
          amg_vcycle(amg, a.R, a.st, s);
          k_cg_z<RPT><<<nblk, kBlock, 0, s>>>(a);
          k_inv_reduce<OP_CG_Z><<<ngrp, kBlock, 0, s>>>(a);
        }
      }
    };
    if (use_graph) {
      RSB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      chunk();
      hipError_t e = hipStreamEndCapture(s, &graph);
      if (e != hipSuccess) fail(RSB_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(RSB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
    }
    struct GraphGuard {
      hipGraphExec_t &e;
      hipGraph_t &g;
      ~GraphGuard() {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
      }
    } guard{exec, graph};
    for (int done = 0; done < p.cg_max_iter; done += kCgChunk) {
      if (exec) RSB_HIP(hipGraphLaunch(exec, s));
      else {
        chunk();
        RSB_LAUNCHED();
      }
      steps += kCgChunk;
      read_flags();
      if (flags == 0) break;
    }
    k_flag_reset<<<1, 1, 0, s>>>(a.flags);
    k_inv_eval<RPT><<<nblk, kBlock, 0, s>>>(a);
    k_inv_reduce<OP_EVAL><<<ngrp, kBlock, 0, s>>>(a);
    k_inv_res<RPT><<<nblk, kBlock, 0, s>>>(a);
    k_inv_reduce<OP_RES><<<ngrp, kBlock, 0, s>>>(a);
    RSB_LAUNCHED();
    read_flags();
    if (flags == 0) break;
  }
  if (y64_out) {
    k_inv_output<RPT><<<nblk, kBlock, 0, s>>>(a, y64_out);
    RSB_LAUNCHED();
  }
  return steps;
}

}  // namespace

size_t inverse_workspace_bytes(int64_t rows, int full_projection) {
  return (size_t)rows * (8 + 2 * (size_t)full_projection) * sizeof(double);
}

int64_t inverse_level(const LevelView &L, CompDev &C, SolveDev &S, const InverseParams &p,
                      void *work, double *y64_out, bool use_graph, Ctx &ctx) {
  if (L.nseg == 0) return 0;
  switch (L.rpt) {
    case 2: return inverse_impl<2>(L, C, S, p, work, y64_out, use_graph, ctx);
    case 4: return inverse_impl<4>(L, C, S, p, work, y64_out, use_graph, ctx);
    case 8: return inverse_impl<8>(L, C, S, p, work, y64_out, use_graph, ctx);
    default: fail(RSB_EINTERNAL, "unsupported rows-per-thread");
  }
}

}  // namespace rsb
