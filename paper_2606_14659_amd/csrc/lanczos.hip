// lanczos.hip -- batched restarted Lanczos with full reorthogonalisation
// (paper Sec. 6) for all segments of a bisection level.
//
// Every segment solves for the smallest eigenpair of its Laplacian restricted
// to the component being cut, orthogonal to the ones vector of that component
// (Sec. 4: L x = lambda x with 1^T x = 0).  Per Lanczos step j of a cycle:
//
//   project  (one launch): q_j = (w - c u0) s is written to the basis, the
//            Laplacian is applied in difference form (L q)_i = s sum_j w_ij
//            (w_i - w_j), and h = [u0, q_1 .. q_j]^T (L q_j) is reduced;
//   update   (one launch): w = L q_j - [u0, Q] h, ||w||^2 reduced; alpha_j =
//            h_j, beta_{j+1} = ||w||.  If the norm dropped below 1/sqrt(2) of
//            the three-term-recurrence norm a second Gram-Schmidt pass runs
//            (two more launches that return at once otherwise).
//
// q_{j+1} = w / beta_{j+1} is never formed as a separate pass: the next
// project launch reads w and applies the scale.  After m steps (or
// breakdown) the tridiagonal eigenproblem is solved on the device, the Ritz
// vector y = Q t becomes the next start vector and its residual decides
// convergence.  Reductions are two-level and in a fixed order (per block,
// per group of 32 blocks, per segment), done by the last block to finish.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

template <typename T>
struct LzArgs {
  const BlkDev *blk;
  const GrpDev *grp;
  const SegDev *seg;
  SegState *st;
  double *alpha, *beta, *h, *tvec;  // [nseg][ps]
  double *part, *gpart;             // [nblk][ps], [ngrp][ps]
  unsigned *gcnt, *scnt;
  int ps;
  const int64_t *chunk_ptr;
  const uint32_t *cols;
  const int32_t *root;
  const int32_t *gid;
  T *V;          // basis: V[k] at V + k * vs; V[0] = u0
  int64_t vs;
  T *W0, *W1;    // ping-pong work vectors
  int m;
  double tol;
  int max_restarts;
  int phase32;
  double brk;    // breakdown threshold relative to ||T||
  int32_t *flags;          // [0] active segments after the cycle, [1] max steps in the cycle
  unsigned long long *ctr; // [0] segment steps
  uint64_t seed;
};

// splitmix64 output for counter gid+1 of the stream started at seed
// (Steele, Lea, Flood 2014), mapped to [-1, 1).
__device__ inline double start_value(uint64_t seed, int64_t gid) {
  uint64_t z = seed + (uint64_t)(gid + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// Fixed-order two-level reduction of `nval` block values held in LDS
// `vals`.  Returns true in the one block that finishes the segment; there
// `vals` holds the segment totals.
template <typename A>
__device__ bool hier_reduce(const A &a, int lb, double *vals, int nval) {
  __shared__ int s_flag;
  const BlkDev b = a.blk[lb];
  const int t = threadIdx.x;
  for (int i = t; i < nval; i += kBlock) a.part[(int64_t)lb * a.ps + i] = vals[i];
  __threadfence();
  __syncthreads();
  if (t == 0) {
    unsigned prev = atomicAdd(&a.gcnt[b.grp], 1u);
    s_flag = (prev == (unsigned)a.grp[b.grp].nblk - 1u);
  }
  __syncthreads();
  if (!s_flag) return false;
  __threadfence();
  const GrpDev g = a.grp[b.grp];
  const SegDev sg = a.seg[b.seg];
  if (t == 0) a.gcnt[b.grp] = 0;
  for (int i = t; i < nval; i += kBlock) {
    double sum = 0.0;
    for (int q = 0; q < g.nblk; ++q) sum += a.part[(int64_t)(g.blk0 + q) * a.ps + i];
    vals[i] = sum;
  }
  __syncthreads();
  if (sg.ngrp == 1) return true;
  for (int i = t; i < nval; i += kBlock) a.gpart[(int64_t)b.grp * a.ps + i] = vals[i];
  __threadfence();
  __syncthreads();
  if (t == 0) {
    unsigned prev = atomicAdd(&a.scnt[b.seg], 1u);
    s_flag = (prev == (unsigned)sg.ngrp - 1u);
  }
  __syncthreads();
  if (!s_flag) return false;
  __threadfence();
  if (t == 0) a.scnt[b.seg] = 0;
  for (int i = t; i < nval; i += kBlock) {
    double sum = 0.0;
    for (int q = 0; q < sg.ngrp; ++q) sum += a.gpart[(int64_t)(sg.grp0 + q) * a.ps + i];
    vals[i] = sum;
  }
  __syncthreads();
  return true;
}

// Sum NV per-thread values over the block into vals[0..NV) (fixed order).
template <int NV>
__device__ inline void block_reduce_into(double (&v)[NV], double *red /* [4*NV] */,
                                         double *vals, int count) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)count) {
    double s = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) s += red[w * NV + threadIdx.x];
    vals[threadIdx.x] = s;
  }
  __syncthreads();
}

// Sliced-ELL Laplacian row in difference form: sum_j w_ij (x_i - x_j).
template <typename T>
__device__ inline T lap_row(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                            const T *__restrict__ x, int64_t row, T xi) {
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = chunk_ptr[c];
  const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
  const uint32_t *cp = cols + p + lane;
  T acc = 0;
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    uint32_t w0 = cp[(k + 0) * 64], w1 = cp[(k + 1) * 64], w2 = cp[(k + 2) * 64],
             w3 = cp[(k + 3) * 64];
    T x0 = x[colw_col(w0)], x1 = x[colw_col(w1)], x2 = x[colw_col(w2)], x3 = x[colw_col(w3)];
    acc += (T)colw_wt(w0) * (xi - x0);
    acc += (T)colw_wt(w1) * (xi - x1);
    acc += (T)colw_wt(w2) * (xi - x2);
    acc += (T)colw_wt(w3) * (xi - x3);
  }
  for (; k < width; ++k) {
    uint32_t w = cp[k * 64];
    acc += (T)colw_wt(w) * (xi - x[colw_col(w)]);
  }
  return acc;
}

// ----------------------------------------------------------------------------
// begin: u0 and the start vector of every segment with a component to cut.
// SRC 0: hashed random start (Sec. 7, Alg. 2 line 1; the Lanczos start);
// SRC 1: from the FP32 phase's final vector (mixed precision refinement).
// ----------------------------------------------------------------------------
template <typename T, int RPT, int SRC>
__global__ __launch_bounds__(kBlock) void k_lz_begin(LzArgs<T> a, const float *__restrict__ y32,
                                                     const SegState *__restrict__ st32,
                                                     const float *__restrict__ u32) {
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.solve) return;
  double c32 = 0, s32 = 0;
  if (SRC == 1) {
    c32 = st32[b.seg].c;
    s32 = st32[b.seg].s;
  }
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    const bool in = (a.root[row] == S.strad);
    const double u = in ? S.invsqrt_nc : 0.0;
    double x = 0.0;
    if (in) {
      if (SRC == 0) x = start_value(a.seed, a.gid[row]);
      else x = ((double)y32[row] - c32 * (double)u32[row]) * s32;
    }
    const T ut = (T)u, xt = (T)x;
    a.V[row] = ut;
    a.W0[row] = xt;
    acc[0] += (double)ut * (double)xt;
    acc[1] += (double)xt * (double)xt;
  }
  block_reduce_into<2>(acc, red, vals, 2);
  if (!hier_reduce(a, lb, vals, 2)) return;
  if (threadIdx.x == 0) {
    SegState &W = a.st[b.seg];
    const double c = vals[0];
    W.c = c;
    W.s = 1.0 / sqrt(fmax(vals[1] - c * c, 1e-300));
    W.active = 1;
    W.k = 0;
    W.cycle_done = 0;
    W.need2 = 0;
    W.converged = 0;
    W.restarts = 0;
    W.tnorm = 0.0;
    W.res = 0.0;
    W.cycles = 0;
    W.steps = 0;
  }
}

// ----------------------------------------------------------------------------
// project: MODE 0 = first pass of step j (SpMV of q_j, write q_j to V[j]);
//          MODE 1 = second Gram-Schmidt pass (project the current w again).
// ----------------------------------------------------------------------------
template <typename T, int RPT, int MODE>
__global__ __launch_bounds__(kBlock) void k_lz_project(LzArgs<T> a, int j) {
  __shared__ double red[4 * 8];
  __shared__ double vals[kMaxM + 8];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cycle_done) return;
  if (MODE == 1 && !S.need2) return;
  const T *Win = ((j - 1) & 1) ? a.W1 : a.W0;
  T *Wout = ((j - 1) & 1) ? a.W0 : a.W1;
  const double c = S.c, sc = S.s;
  double z[RPT], qv[RPT], uv[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    z[r] = qv[r] = uv[r] = 0.0;
    if (lr < b.nrows) {
      const int64_t row = b.row0 + lr;
      const double u = (double)a.V[row];
      uv[r] = u;
      if (MODE == 0) {
        const T wi = Win[row];
        const T q = (T)(((double)wi - c * u) * sc);
        a.V[(int64_t)j * a.vs + row] = q;
        qv[r] = (double)q;
        const T lq = (T)(sc * (double)lap_row<T>(a.chunk_ptr, a.cols, Win, row, wi));
        Wout[row] = lq;
        z[r] = (double)lq;
      } else {
        z[r] = (double)Wout[row];
      }
    }
  }
  // h_k = v_k^T z for k = 0..j, plus ||z||^2 at index j+1
  for (int k0 = 0; k0 <= j; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = r * kBlock + threadIdx.x;
      if (lr >= b.nrows) break;
      const int64_t row = b.row0 + lr;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = k0 + kk;
        if (k > j) break;
        double v;
        if (k == 0) v = uv[r];
        else if (MODE == 0 && k == j) v = qv[r];
        else v = (double)a.V[(int64_t)k * a.vs + row];
        acc[kk] += v * z[r];
      }
    }
    block_reduce_into<8>(acc, red, vals + k0, std::min(8, j + 1 - k0));
  }
  {
    double zz[1] = {0.0};
#pragma unroll
    for (int r = 0; r < RPT; ++r) zz[0] += z[r] * z[r];
    block_reduce_into<1>(zz, red, vals + j + 1, 1);
  }
  if (!hier_reduce(a, lb, vals, j + 2)) return;
  double *hs = a.h + (int64_t)b.seg * a.ps;
  for (int k = threadIdx.x; k <= j; k += kBlock) hs[k] = vals[k];
  if (threadIdx.x == 0 && MODE == 0) a.st[b.seg].lq2 = vals[j + 1];
}

// ----------------------------------------------------------------------------
// update: w -= [u0, Q] h; ||w||^2; finish the step (PASS 1 first pass,
// PASS 2 after the second Gram-Schmidt pass).
// ----------------------------------------------------------------------------
template <typename T, int RPT, int PASS>
__global__ __launch_bounds__(kBlock) void k_lz_update(LzArgs<T> a, int j) {
  __shared__ double red[4];
  __shared__ double vals[2];
  __shared__ double hs[kMaxM + 2];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active || S.cycle_done) return;
  if (PASS == 2 && !S.need2) return;
  const double *hg = a.h + (int64_t)b.seg * a.ps;
  for (int k = threadIdx.x; k <= j; k += kBlock) hs[k] = hg[k];
  __syncthreads();
  T *Wout = ((j - 1) & 1) ? a.W0 : a.W1;
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  for (int k = 0; k <= j; ++k) {
    const double hk = hs[k];
    const T *vk = a.V + (int64_t)k * a.vs + b.row0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = r * kBlock + threadIdx.x;
      if (lr < b.nrows) acc[r] += (double)vk[lr] * hk;
    }
  }
  double nn[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr < b.nrows) {
      const int64_t row = b.row0 + lr;
      const T zt = (T)((double)Wout[row] - acc[r]);
      Wout[row] = zt;
      nn[0] += (double)zt * (double)zt;
    }
  }
  block_reduce_into<1>(nn, red, vals, 1);
  if (!hier_reduce(a, lb, vals, 1)) return;
  if (threadIdx.x != 0) return;
  SegState &W = a.st[b.seg];
  const double w2 = vals[0];
  double alpha_j;
  if (PASS == 1) {
    const double hj = hs[j], hj1 = (j >= 2) ? hs[j - 1] : 0.0;
    const double ref2 = W.lq2 - hj * hj - hj1 * hj1;
    if (w2 < 0.5 * ref2) {
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
  double *al = a.alpha + (int64_t)b.seg * a.ps;
  double *be = a.beta + (int64_t)b.seg * a.ps;
  al[j - 1] = alpha_j;
  const double bprev = (j >= 2) ? be[j - 1] : 0.0;
  W.tnorm = fmax(W.tnorm, fabs(alpha_j) + beta + bprev);
  W.k = j;
  if (j >= a.m || beta <= a.brk * W.tnorm) {
    W.cycle_done = 1;
  } else {
    be[j] = beta;
    W.c = 0.0;
    W.s = 1.0 / beta;
  }
}

// ----------------------------------------------------------------------------
// Smallest eigenpair of T (Sturm multisection by one wavefront, then inverse
// iteration with partial pivoting by lane 0).  Ritz values below 1e-10 ||T||
// are taken as spurious null modes and skipped.
// ----------------------------------------------------------------------------
__device__ inline int sturm_count(const double *a, const double *b, int k, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = (i == 0) ? 0.0 : b[i] * b[i] / q;
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
  __shared__ double ad[kMaxM], bd[kMaxM];
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
  const int c0 = sturm_count(ad, bd, k, thr);
  const int target = std::min(c0 + 1, k);
  lo = fmax(lo, thr);
  hi = hi + 1e-12 * fabs(hi) + 1e-300;
  for (int it = 0; it < 40; ++it) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(kWave + 1);
    const bool ge = sturm_count(ad, bd, k, x) >= target;
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
    for (int it = 0; it < 4; ++it) {
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
// Ritz vector y = Q t into W0 (the next start vector) and its transform.
// ----------------------------------------------------------------------------
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_lz_ritz(LzArgs<T> a) {
  __shared__ double red[4 * 2];
  __shared__ double vals[2];
  __shared__ double ts[kMaxM];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  if (!S.active) return;
  const int k = S.k;
  const double *tg = a.tvec + (int64_t)b.seg * a.ps;
  for (int i = threadIdx.x; i < k; i += kBlock) ts[i] = tg[i];
  __syncthreads();
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  for (int c = 0; c < k; ++c) {
    const double tc = ts[c];
    const T *vc = a.V + (int64_t)(c + 1) * a.vs + b.row0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = r * kBlock + threadIdx.x;
      if (lr < b.nrows) acc[r] += (double)vc[lr] * tc;
    }
  }
  double p[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr < b.nrows) {
      const int64_t row = b.row0 + lr;
      const T y = (T)acc[r];
      a.W0[row] = y;
      p[0] += (double)a.V[row] * (double)y;
      p[1] += (double)y * (double)y;
    }
  }
  block_reduce_into<2>(p, red, vals, 2);
  if (!hier_reduce(a, lb, vals, 2)) return;
  if (threadIdx.x == 0) {
    SegState &W = a.st[b.seg];
    const double c = vals[0];
    W.c = c;
    W.s = 1.0 / sqrt(fmax(vals[1] - c * c, 1e-300));
    W.steps += k;
    atomicAdd(&a.ctr[0], (unsigned long long)k);
    atomicMax(&a.flags[1], k);
  }
}

// ----------------------------------------------------------------------------
// residual of the (projected, normalised) Ritz vector; convergence, restart.
// ||L y - rho y|| with rho the Rayleigh quotient, from ||L y - theta y||^2 =
// ||L y - rho y||^2 + (theta - rho)^2 ||y||^2.
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
  double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = r * kBlock + threadIdx.x;
    if (lr >= b.nrows) break;
    const int64_t row = b.row0 + lr;
    const T wi = a.W0[row];
    const double y = ((double)wi - c * (double)a.V[row]) * sc;
    const double ly = sc * (double)lap_row<T>(a.chunk_ptr, a.cols, a.W0, row, wi);
    const double rr = ly - th * y;
    p[0] += rr * rr;
    p[1] += y * ly;
    p[2] += y * y;
  }
  block_reduce_into<3>(p, red, vals, 3);
  if (!hier_reduce(a, lb, vals, 3)) return;
  if (threadIdx.x != 0) return;
  SegState &W = a.st[b.seg];
  const double rho = vals[1] / vals[2];
  const double dth = th - rho;
  const double res = sqrt(fmax(vals[0] - dth * dth * vals[2], 0.0));
  const double prev = W.res;
  W.res = res;
  W.rho = rho;
  W.cycles += 1;
  bool stop = false;
  if (res <= a.tol * rho) {
    W.converged = 1;
    stop = true;
  } else if (a.phase32 && W.cycles >= 2 && res > 0.9 * prev) {
    stop = true;  // FP32 floor reached: hand over to the FP64 refinement
  } else if (W.restarts >= a.max_restarts) {
    stop = true;
  }
  if (stop) {
    W.active = 0;
  } else {
    W.restarts += 1;
    W.k = 0;
    W.cycle_done = 0;
    W.need2 = 0;
    W.tnorm = 0.0;
    atomicAdd(&a.flags[0], 1);
  }
}

// final vector in FP64: y = (w - c u0) s on the component, 0 elsewhere
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
    if (S.solve) y = ((double)a.W0[row] - S.c * (double)a.V[row]) * S.s;
    y64[row] = y;
  }
}

__global__ void k_flags_reset(int32_t *flags) {
  flags[0] = 0;
  flags[1] = 0;
}

template <typename T, int RPT>
struct LzLaunch {
  static void begin(const LzArgs<T> &a, int nblk, const float *y32, const SegState *st32,
                    const float *u32, hipStream_t s) {
    if (y32)
      k_lz_begin<T, RPT, 1><<<nblk, kBlock, 0, s>>>(a, y32, st32, u32);
    else
      k_lz_begin<T, RPT, 0><<<nblk, kBlock, 0, s>>>(a, nullptr, nullptr, nullptr);
  }
  static void cycle(const LzArgs<T> &a, int nblk, int nseg, hipStream_t s) {
    k_flags_reset<<<1, 1, 0, s>>>(a.flags);
    for (int j = 1; j <= a.m; ++j) {
      k_lz_project<T, RPT, 0><<<nblk, kBlock, 0, s>>>(a, j);
      k_lz_update<T, RPT, 1><<<nblk, kBlock, 0, s>>>(a, j);
      k_lz_project<T, RPT, 1><<<nblk, kBlock, 0, s>>>(a, j);
      k_lz_update<T, RPT, 2><<<nblk, kBlock, 0, s>>>(a, j);
    }
    k_trieig<<<nseg, kWave, 0, s>>>(a.st, a.alpha, a.beta, a.tvec, a.ps, nseg);
    k_lz_ritz<T, RPT><<<nblk, kBlock, 0, s>>>(a);
    k_lz_residual<T, RPT><<<nblk, kBlock, 0, s>>>(a);
  }
  static void output(const LzArgs<T> &a, int nblk, double *y64, hipStream_t s) {
    k_lz_output<T, RPT><<<nblk, kBlock, 0, s>>>(a, y64);
  }
};

template <typename T, typename F>
void dispatch_rpt(int rpt, F &&f) {
  switch (rpt) {
    case 4: f(LzLaunch<T, 4>()); break;
    case 8: f(LzLaunch<T, 8>()); break;
    case 16: f(LzLaunch<T, 16>()); break;
    default: fail(RSB_EINTERNAL, "unsupported rows-per-thread " + std::to_string(rpt));
  }
}

}  // namespace

void solve_alloc(SolveDev &S, const Level &L, int m, Ctx &ctx) {
  S.m = m;
  S.pstride = m + 4;
  const size_t ns = std::max(L.nseg, 1), nb = std::max(L.nblk, 1), ng = std::max(L.ngrp, 1);
  if (!S.st.p || S.st.n < ns) S.st.alloc(ctx, ns);
  S.alpha.alloc(ctx, ns * S.pstride);
  S.beta.alloc(ctx, ns * S.pstride);
  S.h.alloc(ctx, ns * S.pstride);
  S.tvec.alloc(ctx, ns * S.pstride);
  S.part.alloc(ctx, nb * S.pstride);
  S.gpart.alloc(ctx, ng * S.pstride);
  S.gcnt.alloc(ctx, ng);
  S.scnt.alloc(ctx, ns);
  S.n_active.alloc(ctx, 4);
  S.counters.alloc(ctx, 4);
  RSB_HIP(hipMemsetAsync(S.gcnt.get(), 0, S.gcnt.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.scnt.get(), 0, S.scnt.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.counters.get(), 0, S.counters.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(S.beta.get(), 0, S.beta.bytes(), ctx.stream));
}

template <typename T>
int64_t lanczos_level(Level &L, CompDev &C, SolveDev &S, const LanczosParams &p,
                      const float *y32_in, const SolveDev *S32, T *basis, double *y64_out,
                      Ctx &ctx) {
  if (L.nseg == 0) return 0;
  if (p.m < 1 || p.m > kMaxM) fail(RSB_EINVAL, "lanczos_m must be in [1, 250]");
  LzArgs<T> a{};
  a.blk = L.d_blk.get();
  a.grp = L.d_grp.get();
  a.seg = L.d_seg.get();
  a.st = S.st.get();
  a.alpha = S.alpha.get();
  a.beta = S.beta.get();
  a.h = S.h.get();
  a.tvec = S.tvec.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.gcnt = S.gcnt.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.chunk_ptr = L.chunk_ptr.get();
  a.cols = L.cols.get();
  a.root = C.root.get();
  a.gid = L.gid.get();
  a.V = basis;
  a.vs = L.nrows;
  a.W0 = basis + (int64_t)(p.m + 1) * L.nrows;
  a.W1 = a.W0 + L.nrows;
  a.m = p.m;
  a.tol = p.tol;
  a.max_restarts = p.max_restarts;
  a.phase32 = p.phase32;
  a.brk = sizeof(T) == 4 ? 1e-5 : 1e-12;
  a.flags = S.n_active.get();
  a.ctr = (unsigned long long *)S.counters.get();
  a.seed = p.seed;
  const int nblk = L.nblk, nseg = L.nseg;
  const float *u32 = nullptr;
  const SegState *st32 = nullptr;
  if (y32_in) {
    // the FP32 phase's basis: u0 at its start, W0 after its m+1 vectors
    u32 = y32_in;
    st32 = S32->st.get();
  }
  int64_t level_steps = 0;
  dispatch_rpt<T>(L.rpt, [&](auto launcher) {
    using Lz = decltype(launcher);
    const float *y32 = y32_in ? y32_in + (int64_t)(S32->m + 1) * L.nrows : nullptr;
    Lz::begin(a, nblk, y32, st32, u32, ctx.stream);
    RSB_LAUNCHED();
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (p.use_graph) {
      RSB_HIP(hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal));
      Lz::cycle(a, nblk, nseg, ctx.stream);
      hipError_t e = hipStreamEndCapture(ctx.stream, &graph);
      if (e != hipSuccess) fail(RSB_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(RSB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
    }
    int32_t flags[2] = {0, 0};
    for (int cyc = 0; cyc <= p.max_restarts; ++cyc) {
      if (exec) {
        hipError_t e = hipGraphLaunch(exec, ctx.stream);
        if (e != hipSuccess) {
          (void)hipGraphExecDestroy(exec);
          (void)hipGraphDestroy(graph);
          fail(RSB_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
      } else {
        Lz::cycle(a, nblk, nseg, ctx.stream);
        RSB_LAUNCHED();
      }
      hipError_t e = hipMemcpyAsync(flags, a.flags, sizeof(flags), hipMemcpyDeviceToHost,
                                    ctx.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx.stream);
      if (e != hipSuccess) {
        if (exec) {
          (void)hipGraphExecDestroy(exec);
          (void)hipGraphDestroy(graph);
        }
        fail(RSB_EDEVICE, std::string("cycle: ") + hipGetErrorString(e));
      }
      level_steps += flags[1];
      if (flags[0] == 0) break;
    }
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
    }
    if (y64_out) {
      Lz::output(a, nblk, y64_out, ctx.stream);
      RSB_LAUNCHED();
    }
  });
  return level_steps;
}

template int64_t lanczos_level<float>(Level &, CompDev &, SolveDev &, const LanczosParams &,
                                      const float *, const SolveDev *, float *, double *, Ctx &);
template int64_t lanczos_level<double>(Level &, CompDev &, SolveDev &, const LanczosParams &,
                                       const float *, const SolveDev *, double *, double *,
                                       Ctx &);

}  // namespace rsb
