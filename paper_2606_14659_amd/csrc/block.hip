// block.hip -- block Lanczos of two vectors for the Fiedler pair of every
// segment of a level (Sec. 9: a block iteration of two vectors orthogonalised
// together at every step finds both vectors of an exactly degenerate pair,
// where a one-vector iteration finds only the combination its start holds).
// FP64 throughout.
//
// Per block step j (all segments of the level in each launch):
//   step    X_j = (X~ - u0 c) R^-1 from the raw block X~ (first Cholesky QR
//           factor R), W = L X_j read through one 16-byte gather per
//           neighbour; partial dots of W with [u0, Q, X_j], ||W||, X_j^T X_j;
//   reduce  second Cholesky QR factor of X_j (from its Gram matrix), applied
//           to the dots: the first Gram-Schmidt coefficients H1;
//   orth 1  X_j and W take the second factor; W -= [u0 Q] H1; dots again;
//   reduce  H2; the projected matrix's columns of X_j: T = H1 + H2;
//   orth 2  W -= [u0 Q] H2; Gram matrix of W;
//   reduce  first Cholesky QR factor of W, the next raw block.
// After m/2 blocks (or a block with both columns dropped): the eigenpairs of
// T by Jacobi rotations (one wave per segment), the Ritz vectors, their
// residuals, and an explicit or thick restart.
//
// Deflation: a column whose part orthogonal to the column before it is at
// most kDeflRel of its norm, or below kDeflAbs times the largest ||L x||
// seen, is dropped (a zero column: later blocks keep it zero, so the block
// continues as a one-vector Lanczos); in T its diagonal entry is set above
// every eigenvalue, so that it never enters the pair.
#include "solver_dev.h"

namespace rsb {
namespace {

constexpr double kDeflRel = 1e-7;
constexpr double kDeflAbs = 1e-10;
constexpr uint64_t kSecondSeed = 0x9E3779B97F4A7C15ull;  // second column's start stream
constexpr double kBkWarmNoise = 0.1;  // warm start: parent vector + 0.1 x random start
constexpr double kNoSecond = 1e300;   // Ritz value reported when there is no second vector

struct BkState {
  double c0, c1;         // ones components of the raw block
  double r00, r01, r11;  // first Cholesky factor (of the raw block)
  double q00, q01, q11;  // second Cholesky factor (of X_j after the first)
  double tnorm;          // largest ||L x|| seen
  double big;            // diagonal of dropped columns in the last eigen-solve
  double th1, th2;       // the pair's Ritz values
  double cs, sn;         // rotation of the returned pair within its plane
  int32_t z0, z1;        // dropped columns of the current block
  int32_t cur;           // work buffer holding the raw block
  int32_t jb0;           // first block of the cycle
  int32_t nv;            // basis vectors of the cycle so far
  int32_t active, cycle_done, breakdown, converged, cycles, has2, fresh;
  int64_t steps;
};

struct BkArgs {
  const BlkDev *blk;
  const GrpDev *grp;
  const SegDev *seg;
  SegState *st;
  BkState *bs;
  double *part, *gpart;
  unsigned *scnt;
  int ps;
  double *h;  // [nseg][ps]: H1 at 0, H2 at hoff
  int hoff;
  double *Tm;     // [nseg][m][m]
  int32_t *Zq;    // [nseg][m] dropped basis columns
  double *tvec;   // [nseg][nkcap][ps]
  double *tvals;  // [nseg][nkcap]
  int nkcap;
  const int64_t *chunk_ptr;
  const uint32_t *cols;
  const uint32_t *pk;
  const int4 *meta;
  const int32_t *root, *gid, *orig;
  const double *warm;
  double *U0;
  double2 *W0, *W1;  // raw block / remainder, ping-pong
  double2 *Y;        // the pair's Ritz vectors
  double2 *Bq;       // basis blocks [m/2][vs]
  int64_t vs;
  int m, nb, keep, max_restarts, sweep;
  double tol, sweep_gap;
  uint64_t seed;
  int32_t *flags;  // [0] segments still active after a cycle
  __device__ SellRef sell() const { return {chunk_ptr, cols, pk, meta, nullptr, nullptr}; }
  __device__ double2 *W(int i) const { return i ? W1 : W0; }
};

// Cholesky factor of a 2 x 2 Gram matrix with the deflation rule.
__device__ inline void bk_factor(double g00, double g01, double g11, double thr, double &r00,
                                 double &r01, double &r11, int32_t &z0, int32_t &z1) {
  r00 = sqrt(fmax(g00, 0.0));
  z0 = !(r00 > thr);
  if (z0) {
    r00 = 0.0;
    r01 = 0.0;
  } else {
    r01 = g01 / r00;
  }
  r11 = sqrt(fmax(g11 - r01 * r01, 0.0));
  z1 = !(r11 > fmax(thr, kDeflRel * sqrt(fmax(g11, 0.0))));
  if (z1) r11 = 0.0;
}

// [v0, v1] -> [v0, v1] R^-1 (zero for dropped columns).
__device__ inline void bk_apply(double r00, double r01, double r11, int32_t z0, int32_t z1,
                                double v0, double v1, double &o0, double &o1) {
  o0 = z0 ? 0.0 : v0 / r00;
  o1 = z1 ? 0.0 : (v1 - r01 * o0) / r11;
}

__device__ inline bool bk_stepping(const BkState &B, int jb) {
  return B.active && !B.cycle_done && jb >= B.jb0;
}

// Dots of the pair w with basis block i over the tile (index 4 i + 2 c + r =
// b_r^T w_c), summed into vals[4i .. 4i+3].
template <int RPT>
__device__ inline void bk_block_dots(const double2 (&w)[RPT], const double2 (&b)[RPT],
                                     double *red, double *vals) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    v[0] += b[r].x * w[r].x;
    v[1] += b[r].y * w[r].x;
    v[2] += b[r].x * w[r].y;
    v[3] += b[r].y * w[r].y;
  }
  block_reduce_into<4>(v, red, vals, 4);
}

// ----------------------------------------------------------------------------
// begin: u0 and the raw start block of every segment with a component to cut:
// column 0 the usual start (random, or warm), column 1 the random start of
// the second stream; partial sums u^T x_c and x_a^T x_b.
// ----------------------------------------------------------------------------
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_begin(BkArgs a) {
  __shared__ double red[4 * 5];
  __shared__ double vals[5];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.solve) return;
  const TileRows<RPT> tr(b);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!tr.ok[r]) continue;
    const int64_t row = tr.row[r];
    const bool in = (a.root[row] == S.strad);
    const double u = in ? S.invsqrt_nc : 0.0;
    double x0 = in ? start_value(a.seed, a.gid[row]) : 0.0;
    const double x1 = in ? start_value(a.seed ^ kSecondSeed, a.gid[row]) : 0.0;
    if (in && a.warm) {
      const double v = a.warm[a.orig[row]];
      if (!isnan(v)) x0 = v + kBkWarmNoise * x0;
    }
    a.U0[row] = u;
    a.W0[row] = make_double2(x0, x1);
    acc[0] += u * x0;
    acc[1] += u * x1;
    acc[2] += x0 * x0;
    acc[3] += x0 * x1;
    acc[4] += x1 * x1;
  }
  block_reduce_into<5>(acc, red, vals, 5);
  write_partials(a, lb, vals, 5);
}

// ----------------------------------------------------------------------------
// step j: X_j from the raw block, W = L X_j, and the partial sums
//   [4 i + 2 c + r] b_r^T w_c for blocks i < j and X_j itself (i = j),
//   [2 nq + c] u^T w_c, [2 nq + 2 + c] ||w_c||^2, [2 nq + 4..6] X_j^T X_j,
// nq = 2 j + 2 basis vectors.
// ----------------------------------------------------------------------------
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_step(BkArgs a, int jb) {
  __shared__ double red[4 * 7];
  __shared__ double vals[4 * (kBkMaxM / 2) + 8];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const BkState B = a.bs[b.seg];
  if (!bk_stepping(B, jb)) return;
  const double2 *src = a.W(B.cur);
  double2 *dst = a.W(B.cur ^ 1);
  const TileRows<RPT> tr(b);
  double2 x[RPT], w[RPT];
  double tail[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double2 xr = src[row];
    const double u = a.U0[row];
    double x0, x1, w0, w1, l0, l1;
    bk_apply(B.r00, B.r01, B.r11, B.z0, B.z1, xr.x - u * B.c0, xr.y - u * B.c1, x0, x1);
    // L u0 = 0 on the component, so L X_j = (L X~) R^-1
    lap_row2i(a.sell(), src, row, xr.x, xr.y, l0, l1);
    bk_apply(B.r00, B.r01, B.r11, B.z0, B.z1, l0, l1, w0, w1);
    if (!tr.ok[r]) {
      x0 = x1 = w0 = w1 = 0.0;
    } else {
      a.Bq[(int64_t)jb * a.vs + row] = make_double2(x0, x1);
      dst[row] = make_double2(w0, w1);
    }
    x[r] = make_double2(x0, x1);
    w[r] = make_double2(w0, w1);
    tail[0] += u * w0;
    tail[1] += u * w1;
    tail[2] += w0 * w0;
    tail[3] += w1 * w1;
    tail[4] += x0 * x0;
    tail[5] += x0 * x1;
    tail[6] += x1 * x1;
  }
  for (int i = 0; i < jb; ++i) {
    double2 bb[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      bb[r] = tr.ok[r] ? a.Bq[(int64_t)i * a.vs + tr.row[r]] : make_double2(0.0, 0.0);
    bk_block_dots<RPT>(w, bb, red, vals + 4 * i);
  }
  bk_block_dots<RPT>(w, x, red, vals + 4 * jb);
  const int nq = 2 * jb + 2;
  block_reduce_into<7>(tail, red, vals + 2 * nq, 7);
  write_partials(a, lb, vals, 2 * nq + 7);
}

// ----------------------------------------------------------------------------
// orthogonalisation passes of step j on the remainder W (buffer cur ^ 1).
// PASS 1: X_j and W take the second Cholesky factor, W -= [u0 Q] H1, partial
// dots of the result with [Q, X_j] and u0 (layout of the step's first
// 2 nq + 2 sums).  PASS 2: W -= [u0 Q] H2, partial Gram matrix of W.
// ----------------------------------------------------------------------------
template <int RPT, int PASS>
__global__ __launch_bounds__(kBlock) void k_bk_orth(BkArgs a, int jb) {
  __shared__ double red[4 * 4];
  __shared__ double vals[4 * (kBkMaxM / 2) + 8];
  __shared__ double hc[4 * (kBkMaxM / 2) + 4];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const BkState B = a.bs[b.seg];
  if (!bk_stepping(B, jb)) return;
  const int nq = 2 * jb + 2;
  const double *hs = a.h + (int64_t)b.seg * a.ps + (PASS == 2 ? a.hoff : 0);
  for (int i = threadIdx.x; i < 2 * nq + 2; i += kBlock) hc[i] = hs[i];
  __syncthreads();
  double2 *wb = a.W(B.cur ^ 1);
  const TileRows<RPT> tr(b);
  double2 w[RPT], xj[RPT];
  double du[2] = {0.0, 0.0};
  double gm[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    double2 v = wb[row];
    double2 xq = a.Bq[(int64_t)jb * a.vs + row];
    if (PASS == 1) {
      double o0, o1;
      bk_apply(B.q00, B.q01, B.q11, B.z0, B.z1, v.x, v.y, o0, o1);
      v = make_double2(o0, o1);
      bk_apply(B.q00, B.q01, B.q11, B.z0, B.z1, xq.x, xq.y, o0, o1);
      xq = make_double2(o0, o1);
    }
    const double u = a.U0[row];
    double w0 = v.x - u * hc[2 * nq], w1 = v.y - u * hc[2 * nq + 1];
    for (int i = 0; i < jb; ++i) {
      const double2 q = a.Bq[(int64_t)i * a.vs + row];
      w0 -= q.x * hc[4 * i] + q.y * hc[4 * i + 1];
      w1 -= q.x * hc[4 * i + 2] + q.y * hc[4 * i + 3];
    }
    w0 -= xq.x * hc[4 * jb] + xq.y * hc[4 * jb + 1];
    w1 -= xq.x * hc[4 * jb + 2] + xq.y * hc[4 * jb + 3];
    if (!tr.ok[r]) {
      w0 = w1 = 0.0;
      xq = make_double2(0.0, 0.0);
    } else {
      wb[row] = make_double2(w0, w1);
      if (PASS == 1) a.Bq[(int64_t)jb * a.vs + row] = xq;
    }
    w[r] = make_double2(w0, w1);
    xj[r] = xq;
    du[0] += u * w0;
    du[1] += u * w1;
    gm[0] += w0 * w0;
    gm[1] += w0 * w1;
    gm[2] += w1 * w1;
  }
  if (PASS == 1) {
    for (int i = 0; i < jb; ++i) {
      double2 bb[RPT];
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        bb[r] = tr.ok[r] ? a.Bq[(int64_t)i * a.vs + tr.row[r]]
                         : make_double2(0.0, 0.0);
      bk_block_dots<RPT>(w, bb, red, vals + 4 * i);
    }
    bk_block_dots<RPT>(w, xj, red, vals + 4 * jb);
    block_reduce_into<2>(du, red, vals + 2 * nq, 2);
    write_partials(a, lb, vals, 2 * nq + 2);
  } else {
    block_reduce_into<3>(gm, red, vals, 3);
    write_partials(a, lb, vals, 3);
  }
}

// ----------------------------------------------------------------------------
// Ritz vectors of the pair (and, before a thick restart, of the kept set):
// y_c = sum_k s_{k,c} q_k over the cycle's nv basis vectors.  Each thread
// reads all basis values of its row before it rewrites that row's kept
// slots.
// ----------------------------------------------------------------------------
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_ritz(BkArgs a) {
  __shared__ double co[kMaxKeep * kBkMaxM];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const BkState B = a.bs[b.seg];
  if (!B.active) return;
  const int k = B.nv;
  const bool thick = a.keep > 0 && !B.breakdown;
  const int nn = thick ? a.keep : 2;
  const double *tv = a.tvec + (int64_t)b.seg * a.nkcap * a.ps;
  for (int i = threadIdx.x; i < nn * k; i += kBlock) co[i] = tv[(int64_t)(i / k) * a.ps + i % k];
  __syncthreads();
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + (int)threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    double y[kMaxKeep];
#pragma unroll
    for (int c = 0; c < kMaxKeep; ++c) y[c] = 0.0;
    for (int i = 0; 2 * i < k; ++i) {
      const double2 q = a.Bq[(int64_t)i * a.vs + row];
#pragma unroll
      for (int c = 0; c < kMaxKeep; ++c)
        if (c < nn) y[c] += co[c * k + 2 * i] * q.x + co[c * k + 2 * i + 1] * q.y;
    }
    a.Y[row] = make_double2(y[0], y[1]);
    if (thick) {
#pragma unroll
      for (int c = 0; c < kMaxKeep; c += 2)
        if (c < nn) a.Bq[(int64_t)(c / 2) * a.vs + row] = make_double2(y[c], y[c + 1]);
    }
  }
}

// ----------------------------------------------------------------------------
// residuals of the pair: partial sums of ||L y1 - th1 y1||^2, ||L y2 - th2 y2||^2,
// y1^T L y1, y2^T L y2, y1^T L y2, y1^T y1, y1^T y2, y2^T y2, u^T y1, u^T y2
// and s^T y1, s^T y2 with s the random start of seed on the component.
// ----------------------------------------------------------------------------
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_resid(BkArgs a) {
  __shared__ double red[4 * 12];
  __shared__ double vals[12];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const BkState B = a.bs[b.seg];
  if (!B.active) return;
  const SegState S = a.st[b.seg];
  const TileRows<RPT> tr(b);
  double p[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) p[i] = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t row = tr.row[r];
    const double2 y = a.Y[row];
    double l0, l1;
    lap_row2i(a.sell(), a.Y, row, y.x, y.y, l0, l1);
    if (!tr.ok[r]) continue;
    const double u = a.U0[row];
    const double s = (a.root[row] == S.strad) ? start_value(a.seed, a.gid[row]) : 0.0;
    const double r0 = l0 - B.th1 * y.x;
    const double r1 = B.has2 ? l1 - B.th2 * y.y : 0.0;
    p[0] += r0 * r0;
    p[1] += r1 * r1;
    p[2] += y.x * l0;
    p[3] += y.y * l1;
    p[4] += y.x * l1;
    p[5] += y.x * y.x;
    p[6] += y.x * y.y;
    p[7] += y.y * y.y;
    p[8] += u * y.x;
    p[9] += u * y.y;
    p[10] += s * y.x;
    p[11] += s * y.y;
  }
  block_reduce_into<12>(p, red, vals, 12);
  write_partials(a, lb, vals, 12);
}

// Explicit restart: the pair becomes the raw block of the next cycle.
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_restart(BkArgs a) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const BkState B = a.bs[b.seg];
  if (!(B.active && B.fresh)) return;
  double2 *dst = a.W(B.cur);
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + (int)threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    dst[row] = a.Y[row];
  }
}

// The returned pair (rotated within its plane when it is to be swept).
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bk_output(BkArgs a, double *__restrict__ y64,
                                                      double *__restrict__ y2) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  const BkState B = a.bs[b.seg];
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + (int)threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    double v1 = 0.0, v2 = 0.0;
    if (S.solve) {
      const double2 y = a.Y[row];
      v1 = B.cs * y.x + B.sn * y.y;
      v2 = B.cs * y.y - B.sn * y.x;
    }
    y64[row] = v1;
    if (y2) y2[row] = v2;
  }
}

// ----------------------------------------------------------------------------
// Eigenpairs of the cycle's projected matrix, one wave per segment: Jacobi
// rotations (Golub & Van Loan, Sec. 8.5) in round-robin order -- in each of
// the k - 1 rounds of a sweep the k / 2 pairs (p, q) of the circle method are
// disjoint, so their rotations commute and are applied together: angles from
// the current matrix, then the columns of A and V (one row per lane), then
// the rows of A (one column per lane).  Sweeps until the off-diagonal part
// is at rounding level; eigenvalues sorted ascending (stable).  Output: the
// first max(2, keep) Ritz values and coefficient vectors.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void k_bk_eig(BkArgs a) {
  // rows padded to an odd number of doubles: the lanes' row accesses of a
  // column spread over the LDS banks
  __shared__ double A[kBkMaxM * (kBkMaxM + 1)];
  __shared__ double V[kBkMaxM * (kBkMaxM + 1)];
  __shared__ double rot_c[kBkMaxM / 2], rot_s[kBkMaxM / 2];  // this round's rotations
  __shared__ int32_t rot_p[kBkMaxM / 2], rot_q[kBkMaxM / 2];
  __shared__ int32_t ord[kBkMaxM];
  const int s = blockIdx.x;
  const BkState B = a.bs[s];
  if (!B.active) return;
  const int k = B.nv;  // even
  const int h = k / 2;
  const int ld = k + 1;
  const int lane = threadIdx.x;
  const double *T = a.Tm + (int64_t)s * a.m * a.m;
  const int32_t *zq = a.Zq + (int64_t)s * a.m;
  for (int i = lane; i < k * k; i += kWave) {
    const int r = i / k, c = i % k;
    A[r * ld + c] = T[(int64_t)r * a.m + c];
    V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  // diagonal of the dropped columns: above every eigenvalue (row-sum bound)
  double rs = 0.0;
  if (lane < k && !zq[lane])
    for (int c = 0; c < k; ++c) rs += fabs(A[lane * ld + c]);
  for (int off = kWave / 2; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off, kWave));
  const double big = 1.0 + 2.0 * rs;
  __syncthreads();
  if (lane < k && zq[lane]) A[lane * ld + lane] = big;
  __syncthreads();
  double f = 0.0;
  for (int i = lane; i < k * k; i += kWave) {
    const double v = A[(i / k) * ld + i % k];
    f += v * v;
  }
  const double fro = sqrt(wave_sum(f));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = lane; i < k * k; i += kWave) {
      const int p = i / k, q = i % k;
      if (p < q) off += 2.0 * A[p * ld + q] * A[p * ld + q];
    }
    off = wave_sum(off);
    if (sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
    for (int rnd = 0; rnd < k - 1; ++rnd) {
      if (lane < h) {
        // circle method: player 0 fixed, players 1..k-1 rotate by one each round
        const int pa = lane == 0 ? 0 : 1 + (lane - 1 + rnd) % (k - 1);
        const int pb = 1 + (k - 2 - lane + rnd) % (k - 1);
        const int p = min(pa, pb), q = max(pa, pb);
        const double apq = A[p * ld + q];
        double c = 1.0, sn = 0.0;
        if (apq != 0.0) {
          const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
        rot_c[lane] = c;
        rot_s[lane] = sn;
        rot_p[lane] = p;
        rot_q[lane] = q;
      }
      __syncthreads();
      if (lane < k) {
        for (int i = 0; i < h; ++i) {
          const int p = rot_p[i], q = rot_q[i];
          const double c = rot_c[i], sn = rot_s[i];
          const double arp = A[lane * ld + p], arq = A[lane * ld + q];
          A[lane * ld + p] = c * arp - sn * arq;
          A[lane * ld + q] = sn * arp + c * arq;
          const double vrp = V[lane * ld + p], vrq = V[lane * ld + q];
          V[lane * ld + p] = c * vrp - sn * vrq;
          V[lane * ld + q] = sn * vrp + c * vrq;
        }
      }
      __syncthreads();
      if (lane < k) {
        for (int i = 0; i < h; ++i) {
          const int p = rot_p[i], q = rot_q[i];
          const double c = rot_c[i], sn = rot_s[i];
          const double apr = A[p * ld + lane], aqr = A[q * ld + lane];
          A[p * ld + lane] = c * apr - sn * aqr;
          A[q * ld + lane] = sn * apr + c * aqr;
        }
      }
      __syncthreads();
    }
  }
  if (lane < k) {
    const double d = A[lane * ld + lane];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double e = A[j * ld + j];
      rank += (e < d || (e == d && j < lane)) ? 1 : 0;
    }
    ord[rank] = lane;
  }
  __syncthreads();
  const int nn = min(max(2, a.keep), k);
  double *tv = a.tvec + (int64_t)s * a.nkcap * a.ps;
  double *tl = a.tvals + (int64_t)s * a.nkcap;
  for (int c = 0; c < nn; ++c) {
    const int o = ord[c];
    if (lane == 0) tl[c] = A[o * ld + o];
    for (int r = lane; r < k; r += kWave) tv[(int64_t)c * a.ps + r] = V[r * ld + o];
  }
  if (lane == 0) {
    BkState &Bo = a.bs[s];
    Bo.big = big;
    Bo.th1 = A[ord[0] * ld + ord[0]];
    Bo.th2 = A[ord[1] * ld + ord[1]];
    Bo.has2 = Bo.th2 < big;
  }
}

// ----------------------------------------------------------------------------
// Segmented reductions and the per-segment scalar work of each phase.
// ----------------------------------------------------------------------------
enum { BK_BEGIN = 0, BK_H1 = 1, BK_H2 = 2, BK_GRAM = 3, BK_RESID = 4 };

template <int OP>
__global__ __launch_bounds__(kBlock) void k_bk_reduce(BkArgs a, int jb) {
  __shared__ double vals[4 * (kBkMaxM / 2) + 16];
  const int g = blockIdx.x;
  const GrpDev G = a.grp[g];
  const int s = G.seg;
  const SegState S = a.st[s];
  const BkState B = a.bs[s];
  const SegDev sg = a.seg[s];
  const int nq = 2 * jb + 2;
  const int nval = (OP == BK_BEGIN) ? 5
                   : (OP == BK_H1)  ? 2 * nq + 7
                   : (OP == BK_H2)  ? 2 * nq + 2
                   : (OP == BK_GRAM) ? 3
                                     : 12;
  group_sums(a, G, vals, nval);
  bool take;
  switch (OP) {
    case BK_BEGIN: take = S.solve != 0; break;
    case BK_RESID: take = B.active != 0; break;
    default: take = bk_stepping(B, jb); break;
  }
  if (!take) return;
  if (!group_finish(a, g, G, sg, vals, nval)) return;
  const int t = threadIdx.x;
  BkState &Bo = a.bs[s];
  double *h1 = a.h + (int64_t)s * a.ps;
  double *h2 = h1 + a.hoff;
  if (OP == BK_BEGIN) {
    if (t == 0) {
      BkState n = {};
      n.c0 = vals[0];
      n.c1 = vals[1];
      const double raw = sqrt(fmax(vals[2], vals[4]));
      bk_factor(vals[2] - n.c0 * n.c0, vals[3] - n.c0 * n.c1, vals[4] - n.c1 * n.c1,
                kDeflAbs * raw, n.r00, n.r01, n.r11, n.z0, n.z1);
      n.cs = 1.0;
      n.active = 1;
      Bo = n;
    }
    return;
  }
  if (OP == BK_H1) {
    __shared__ double q[3];
    __shared__ int32_t zz[2];
    if (t == 0) {
      const double tn = fmax(B.tnorm, fmax(sqrt(vals[2 * nq + 2]), sqrt(vals[2 * nq + 3])));
      double q00, q01, q11;
      int32_t y0, y1;
      bk_factor(vals[2 * nq + 4], vals[2 * nq + 5], vals[2 * nq + 6], 0.5, q00, q01, q11, y0, y1);
      const int32_t z0 = B.z0 | y0, z1 = B.z1 | y1;
      Bo.tnorm = tn;
      Bo.q00 = q00;
      Bo.q01 = q01;
      Bo.q11 = q11;
      Bo.z0 = z0;
      Bo.z1 = z1;
      a.Zq[(int64_t)s * a.m + 2 * jb] = z0;
      a.Zq[(int64_t)s * a.m + 2 * jb + 1] = z1;
      q[0] = q00;
      q[1] = q01;
      q[2] = q11;
      zz[0] = z0;
      zz[1] = z1;
    }
    __syncthreads();
    // columns of W take the factor: (d0, d1) -> (d0, d1) Q^-1 for every row
    // of dots (basis vectors 0..nq-1 and u0); the rows of X_j then too
    for (int i = t; i < nq + 1; i += kBlock) {
      const int i0 = (i < nq) ? 4 * (i / 2) + (i % 2) : 2 * nq;
      const int st = (i < nq) ? 2 : 1;
      double o0, o1;
      bk_apply(q[0], q[1], q[2], zz[0], zz[1], vals[i0], vals[i0 + st], o0, o1);
      vals[i0] = o0;
      vals[i0 + st] = o1;
    }
    __syncthreads();
    if (t < 2) {
      // rows r = 0, 1 of X_j^T W for column c = t
      const int c = t;
      double o0, o1;
      bk_apply(q[0], q[1], q[2], zz[0], zz[1], vals[4 * jb + 2 * c], vals[4 * jb + 2 * c + 1],
               o0, o1);
      vals[4 * jb + 2 * c] = o0;
      vals[4 * jb + 2 * c + 1] = o1;
    }
    __syncthreads();
    for (int i = t; i < 2 * nq + 2; i += kBlock) h1[i] = vals[i];
    return;
  }
  if (OP == BK_H2) {
    double *T = a.Tm + (int64_t)s * a.m * a.m;
    const int c0 = 2 * jb;
    for (int k = t; k < c0; k += kBlock) {
      const int i = k / 2, r = k % 2;
      for (int c = 0; c < 2; ++c) {
        const double v = h1[4 * i + 2 * c + r] + vals[4 * i + 2 * c + r];
        T[(int64_t)k * a.m + c0 + c] = v;
        T[(int64_t)(c0 + c) * a.m + k] = v;
      }
    }
    if (t == 0) {
      const double d00 = h1[4 * jb] + vals[4 * jb];
      const double d10 = h1[4 * jb + 1] + vals[4 * jb + 1];
      const double d01 = h1[4 * jb + 2] + vals[4 * jb + 2];
      const double d11 = h1[4 * jb + 3] + vals[4 * jb + 3];
      T[(int64_t)c0 * a.m + c0] = d00;
      T[(int64_t)(c0 + 1) * a.m + c0 + 1] = d11;
      T[(int64_t)c0 * a.m + c0 + 1] = T[(int64_t)(c0 + 1) * a.m + c0] = 0.5 * (d01 + d10);
      Bo.nv = c0 + 2;
    }
    for (int i = t; i < 2 * nq + 2; i += kBlock) h2[i] = vals[i];
    return;
  }
  if (OP == BK_GRAM) {
    if (t == 0) {
      double r00, r01, r11;
      int32_t z0, z1;
      bk_factor(vals[0], vals[1], vals[2], kDeflAbs * B.tnorm, r00, r01, r11, z0, z1);
      Bo.r00 = r00;
      Bo.r01 = r01;
      Bo.r11 = r11;
      Bo.z0 = z0;
      Bo.z1 = z1;
      Bo.c0 = 0.0;
      Bo.c1 = 0.0;
      Bo.cur = B.cur ^ 1;
      Bo.steps = B.steps + 1;
      if (z0 && z1) {
        Bo.breakdown = 1;
        Bo.cycle_done = 1;
      } else if (jb == a.nb - 1) {
        Bo.cycle_done = 1;
      }
    }
    return;
  }
  // BK_RESID
  __shared__ int32_t thick_restart;
  if (t == 0) {
    thick_restart = 0;
    const double res1 = sqrt(vals[0]), res2 = sqrt(vals[1]);
    const int cycles = B.cycles + 1;
    const bool conv = res1 <= a.tol * B.th1 && (!B.has2 || res2 <= a.tol * B.th2);
    Bo.cycles = cycles;
    if (conv || cycles > a.max_restarts) {
      double cs = 1.0, sn = 0.0;
      if (a.sweep > 0 && B.has2 && B.th2 - B.th1 <= a.sweep_gap * B.th1) {
        const double cn = sqrt(vals[10] * vals[10] + vals[11] * vals[11]);
        if (cn > 0.0) {
          cs = vals[10] / cn;
          sn = vals[11] / cn;
        }
      }
      Bo.cs = cs;
      Bo.sn = sn;
      Bo.active = 0;
      Bo.converged = conv ? 1 : 0;
      // Rayleigh quotient of the returned vector cs y1 + sn y2
      const double num = cs * cs * vals[2] + 2.0 * cs * sn * vals[4] + sn * sn * vals[3];
      const double den = cs * cs * vals[5] + 2.0 * cs * sn * vals[6] + sn * sn * vals[7];
      SegState &So = a.st[s];
      So.rho = num / den;
      So.theta = B.th1;
      So.res = res1;
      So.converged = conv ? 1 : 0;
      So.active = 0;
      So.cycles = cycles;
      So.steps = B.steps;
      So.nnext = B.has2 ? 2 : 1;
      double *tl = a.tvals + (int64_t)s * a.nkcap;
      tl[0] = B.th1;
      tl[1] = B.has2 ? B.th2 : kNoSecond;
    } else if (a.keep == 0 || B.breakdown) {
      // explicit restart from the pair (copied into the raw block's buffer)
      Bo.c0 = vals[8];
      Bo.c1 = vals[9];
      double r00, r01, r11;
      int32_t z0, z1;
      bk_factor(vals[5] - vals[8] * vals[8], vals[6] - vals[8] * vals[9],
                vals[7] - vals[9] * vals[9], kDeflAbs, r00, r01, r11, z0, z1);
      Bo.r00 = r00;
      Bo.r01 = r01;
      Bo.r11 = r11;
      Bo.z0 = z0;
      Bo.z1 = z1;
      Bo.jb0 = 0;
      Bo.nv = 0;
      Bo.fresh = 1;
      Bo.cycle_done = 0;
      Bo.breakdown = 0;
      atomicAdd(&a.flags[0], 1);
    } else {
      // thick restart: the kept Ritz vectors head the basis, the cycle
      // continues from the last remainder block (its factor is current)
      Bo.jb0 = a.keep / 2;
      Bo.nv = a.keep;
      Bo.fresh = 0;
      Bo.cycle_done = 0;
      thick_restart = 1;
      atomicAdd(&a.flags[0], 1);
    }
  }
  __syncthreads();
  if (thick_restart) {
    double *T = a.Tm + (int64_t)s * a.m * a.m;
    const double *tl = a.tvals + (int64_t)s * a.nkcap;
    for (int i = t; i < a.keep * a.keep; i += kBlock) {
      const int r = i / a.keep, c = i % a.keep;
      T[(int64_t)r * a.m + c] = (r == c) ? tl[r] : 0.0;
    }
    for (int r = t; r < a.keep; r += kBlock) a.Zq[(int64_t)s * a.m + r] = !(tl[r] < B.big);
  }
}

__global__ void k_bk_flags_reset(int32_t *flags) { flags[0] = 0; }

template <int RPT>
int64_t block_impl(const LevelView &L, CompDev &C, SolveDev &S, const BlockParams &p,
                   double *y64, double *y2, Ctx &ctx) {
  const int64_t nr = std::max<int64_t>(L.nrows, 1);
  const int nb = p.m / 2;
  DevBuf<double> u0(ctx, nr), tm(ctx, (size_t)L.nseg * p.m * p.m);
  DevBuf<double2> w0(ctx, nr), w1(ctx, nr), yy(ctx, nr), bq(ctx, (size_t)nb * nr);
  DevBuf<int32_t> zq(ctx, (size_t)L.nseg * p.m), flags(ctx, 4);
  DevBuf<BkState> bs(ctx, L.nseg);
  RSB_HIP(hipMemsetAsync(bs.get(), 0, L.nseg * sizeof(BkState), ctx.stream));
  RSB_HIP(hipMemsetAsync(tm.get(), 0, (size_t)L.nseg * p.m * p.m * sizeof(double), ctx.stream));
  RSB_HIP(hipMemsetAsync(zq.get(), 0, (size_t)L.nseg * p.m * sizeof(int32_t), ctx.stream));
  BkArgs a{};
  a.blk = L.blk;
  a.grp = L.grp;
  a.seg = L.seg;
  a.st = S.st.get();
  a.bs = bs.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.h = S.h.get();
  a.hoff = 2 * p.m + 4;
  a.Tm = tm.get();
  a.Zq = zq.get();
  a.tvec = S.tvec.get();
  a.tvals = S.tvals.get();
  a.nkcap = S.nkcap;
  a.chunk_ptr = L.chunk_ptr;
  a.cols = L.cols;
  a.pk = L.pk;
  a.meta = L.pmeta;
  a.root = C.root.get();
  a.gid = L.gid;
  a.orig = L.orig;
  a.warm = p.warm;
  a.U0 = u0.get();
  a.W0 = w0.get();
  a.W1 = w1.get();
  a.Y = yy.get();
  a.Bq = bq.get();
  a.vs = nr;
  a.m = p.m;
  a.nb = nb;
  a.keep = p.keep;
  a.max_restarts = p.max_restarts;
  a.sweep = p.sweep;
  a.tol = p.tol;
  a.sweep_gap = p.sweep_gap;
  a.seed = p.seed;
  a.flags = flags.get();
  const int nblk = L.nblk, ngrp = L.ngrp;
  hipStream_t s = ctx.stream;
  k_bk_begin<RPT><<<nblk, kBlock, 0, s>>>(a);
  k_bk_reduce<BK_BEGIN><<<ngrp, kBlock, 0, s>>>(a, 0);
  RSB_LAUNCHED();
  int64_t steps = 0;
  for (int cycle = 0; cycle <= p.max_restarts; ++cycle) {
    for (int jb = 0; jb < nb; ++jb) {
      k_bk_step<RPT><<<nblk, kBlock, 0, s>>>(a, jb);
      k_bk_reduce<BK_H1><<<ngrp, kBlock, 0, s>>>(a, jb);
      k_bk_orth<RPT, 1><<<nblk, kBlock, 0, s>>>(a, jb);
      k_bk_reduce<BK_H2><<<ngrp, kBlock, 0, s>>>(a, jb);
      k_bk_orth<RPT, 2><<<nblk, kBlock, 0, s>>>(a, jb);
      k_bk_reduce<BK_GRAM><<<ngrp, kBlock, 0, s>>>(a, jb);
      RSB_LAUNCHED();
    }
    steps += nb;
    k_bk_eig<<<L.nseg, kWave, 0, s>>>(a);
    k_bk_ritz<RPT><<<nblk, kBlock, 0, s>>>(a);
    k_bk_resid<RPT><<<nblk, kBlock, 0, s>>>(a);
    k_bk_flags_reset<<<1, 1, 0, s>>>(a.flags);
    k_bk_reduce<BK_RESID><<<ngrp, kBlock, 0, s>>>(a, 0);
    k_bk_restart<RPT><<<nblk, kBlock, 0, s>>>(a);
    RSB_LAUNCHED();
    int32_t nact = 0;
    RSB_HIP(hipMemcpyAsync(&nact, a.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RSB_HIP(hipStreamSynchronize(s));
    if (nact == 0) break;
  }
  k_bk_output<RPT><<<nblk, kBlock, 0, s>>>(a, y64, y2);
  RSB_LAUNCHED();
  // segment steps: block steps summed over the segments
  std::vector<BkState> hb(L.nseg);
  RSB_HIP(hipMemcpyAsync(hb.data(), bs.get(), L.nseg * sizeof(BkState), hipMemcpyDeviceToHost, s));
  RSB_HIP(hipStreamSynchronize(s));
  int64_t segsteps = 0;
  for (const auto &b : hb) segsteps += b.steps;
  int64_t acc = 0;
  RSB_HIP(hipMemcpyAsync(&acc, S.counters.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RSB_HIP(hipStreamSynchronize(s));
  acc += segsteps;
  RSB_HIP(hipMemcpyAsync(S.counters.get(), &acc, sizeof(int64_t), hipMemcpyHostToDevice, s));
  RSB_HIP(hipStreamSynchronize(s));
  return steps;
}

}  // namespace

int64_t block_level(const LevelView &L, CompDev &C, SolveDev &S, const BlockParams &p,
                    double *y64, double *y2, Ctx &ctx) {
  if (L.nseg == 0) return 0;
  if (p.m < 4 || p.m > kBkMaxM || p.m % 2)
    fail(RSB_EINVAL, "block Lanczos: lanczos_m must be even and in [4, 48]");
  if (p.keep < 0 || p.keep % 2 || p.keep > p.m - 4 || p.keep > kMaxKeep)
    fail(RSB_EINVAL, "block Lanczos: lanczos_keep must be even and at most min(16, lanczos_m - 4)");
  if (S.nkcap < std::max(2, p.keep) || S.pstride < 4 * p.m + 8)
    fail(RSB_EINTERNAL, "block Lanczos: solver buffers too small");
  switch (L.rpt) {
    case 2: return block_impl<2>(L, C, S, p, y64, y2, ctx);
    case 4: return block_impl<4>(L, C, S, p, y64, y2, ctx);
    case 8: return block_impl<8>(L, C, S, p, y64, y2, ctx);
    default: fail(RSB_EINTERNAL, "unsupported rows-per-thread");
  }
}

}  // namespace rsb
