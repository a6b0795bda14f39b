// solver_dev.h -- device helpers shared by the eigen-solvers: the start
// vector, fixed-order segmented reductions and the Laplacian row.
#pragma once
#include "common.h"
#include "kernels.h"

namespace rsb {

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
// `vals` (A provides blk, grp, seg, part, gpart, gcnt, scnt, ps).  Returns
// true in the one block that finishes the segment; there `vals` holds the
// segment totals.  Block partials are published with a device-scope fence
// before the arrival counter is bumped, and read after an acquire fence.
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

// Sum NV per-thread values over the block into vals[0..count) (fixed order).
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

// Sliced-ELL Laplacian row in difference form: sum_j w_ij (x_i - x_j),
// accumulated in the vector type (paper Sec. 5: the action of L on x).
template <typename X>
__device__ inline X lap_row(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                            const X *__restrict__ x, int64_t row, X xi) {
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = chunk_ptr[c];
  const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
  const uint32_t *cp = cols + p + lane;
  X acc = 0;
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    uint32_t w0 = cp[(k + 0) * 64], w1 = cp[(k + 1) * 64], w2 = cp[(k + 2) * 64],
             w3 = cp[(k + 3) * 64];
    X x0 = x[colw_col(w0)], x1 = x[colw_col(w1)], x2 = x[colw_col(w2)], x3 = x[colw_col(w3)];
    acc += (X)colw_wt(w0) * (xi - x0);
    acc += (X)colw_wt(w1) * (xi - x1);
    acc += (X)colw_wt(w2) * (xi - x2);
    acc += (X)colw_wt(w3) * (xi - x3);
  }
  for (; k < width; ++k) {
    uint32_t w = cp[k * 64];
    acc += (X)colw_wt(w) * (xi - x[colw_col(w)]);
  }
  return acc;
}

}  // namespace rsb
