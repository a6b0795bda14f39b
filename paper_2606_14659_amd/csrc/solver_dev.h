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

// Segmented reductions are split in two launches.  The streaming kernel
// writes one partial vector per block (plain stores, no fence: a device-scope
// release in every block of a large launch would write back the L2 each
// time).  A small reduction kernel with one block per group of up to 32
// blocks then sums the partials in a fixed order; a segment with several
// groups is finished by its last group to arrive (its fences are cheap: at
// that point the L2 holds only the few group sums).
template <typename A>
__device__ inline void write_partials(const A &a, int lb, const double *vals, int nval) {
  for (int i = threadIdx.x; i < nval; i += kBlock) a.part[(int64_t)lb * a.ps + i] = vals[i];
}

// Sums over n rows of partials: vals[i] = sum_q src[q * ps + i], i < nval.
// K threads share a value (the largest power of two with K nval <= kBlock);
// thread sub of a value sums rows q = sub, sub + K, ... in increasing order,
// eight loads in flight at a time, then the K sums are added by a fixed tree,
// so the result does not depend on timing.
__device__ inline void sum_rows(const double *__restrict__ src, int n, int ps, int nval,
                                double *vals, double *lds /* [kBlock] */) {
  int K = 1;
  while (2 * K * nval <= kBlock) K *= 2;
  const int t = threadIdx.x;
  const int sub = t % K;
  for (int i0 = 0; i0 < nval; i0 += kBlock / K) {
    const int i = i0 + t / K;
    double acc = 0.0;
    if (i < nval) {
      for (int q0 = sub; q0 < n; q0 += 8 * K) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int q = q0 + u * K;
          v[u] = (q < n) ? src[(int64_t)q * ps + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
      }
    }
    lds[t] = acc;
    __syncthreads();
    for (int h = K / 2; h > 0; h >>= 1) {
      if (sub < h) lds[t] += lds[t + h];
      __syncthreads();
    }
    if (sub == 0 && i < nval) vals[i] = lds[t];
    __syncthreads();
  }
}

// Reduction-kernel side (block g = group g), first level: the group's
// block partials summed into vals[0..nval).  It only reads, so a caller may
// run it before it knows whether the segment takes part.
template <typename A>
__device__ inline void group_sums(const A &a, const GrpDev &G, double *vals, int nval) {
  __shared__ double lds[kBlock];
  sum_rows(a.part + (int64_t)G.blk0 * a.ps, G.nblk, a.ps, nval, vals, lds);
}

// Second level, after group_sums: returns true in the one block that
// finishes the segment; there vals[0..nval) holds the segment totals.
template <typename A>
__device__ bool group_finish(const A &a, int g, const GrpDev &G, const SegDev &sg, double *vals,
                             int nval) {
  __shared__ double lds[kBlock];
  __shared__ int s_flag;
  const int t = threadIdx.x;
  if (sg.ngrp == 1) return true;
  for (int i = t; i < nval; i += kBlock) a.gpart[(int64_t)g * a.ps + i] = vals[i];
  __threadfence();
  __syncthreads();
  if (t == 0) {
    unsigned prev = atomicAdd(&a.scnt[G.seg], 1u);
    s_flag = (prev == (unsigned)sg.ngrp - 1u);
  }
  __syncthreads();
  if (!s_flag) return false;
  __threadfence();
  if (t == 0) a.scnt[G.seg] = 0;
  sum_rows(a.gpart + (int64_t)sg.grp0 * a.ps, sg.ngrp, a.ps, nval, vals, lds);
  return true;
}

template <typename A>
__device__ bool group_reduce(const A &a, int g, double *vals, int nval) {
  const GrpDev G = a.grp[g];
  const SegDev sg = a.seg[G.seg];
  group_sums(a, G, vals, nval);
  return group_finish(a, g, G, sg, vals, nval);
}

// Rows of a block tile.  Thread t owns rows t, t + 256, ... (RPT of them); a
// row past the tile end is clamped to the tile's first row for its loads and
// its results are dropped, so the hot loops have no per-row branches and all
// their loads can be in flight together.
template <int RPT>
struct TileRows {
  int64_t row[RPT];
  bool ok[RPT];
  __device__ TileRows(const BlkDev &b) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = r * kBlock + (int)threadIdx.x;
      ok[r] = lr < b.nrows;
      row[r] = b.row0 + (ok[r] ? lr : 0);
    }
  }
};

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

// Load of data that a launch reads once (matrix words, basis vectors),
// marked non-temporal so that the stream does not push the gathered vector
// out of L2.
template <typename P>
__device__ inline P ld_stream(const P *p) {
  return __builtin_nontemporal_load(p);
}

// Sliced-ELL Laplacian row in difference form: sum_j w_ij (x_i - x_j),
// accumulated in the vector type (paper Sec. 5: the action of L on x).
template <int G, typename X>
__device__ inline void lap_slots(const uint32_t *__restrict__ cp, const X *__restrict__ x, int k0,
                                 int width, X xi, X &acc) {
  uint32_t w[G];
#pragma unroll
  for (int u = 0; u < G; ++u) w[u] = ld_stream(cp + (int64_t)(k0 + u) * 64);
#pragma unroll
  for (int u = 0; u < G; ++u) w[u] = (k0 + u < width) ? w[u] : 0u;
  X xv[G];
#pragma unroll
  for (int u = 0; u < G; ++u) xv[u] = x[colw_col(w[u])];
#pragma unroll
  for (int u = 0; u < G; ++u) acc += colw_wt(w[u]) ? (X)colw_wt(w[u]) * (xi - xv[u]) : (X)0;
}

template <typename X>
__device__ inline X lap_row(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                            const X *__restrict__ x, int64_t row, X xi) {
  // slots read at once: 16 for 4-byte values, 8 for 8-byte values (register
  // budget), and a group of 4 for a short remainder; never more than the
  // zero slack after the last slice
  constexpr int G = sizeof(X) == 8 ? kSlotGroup / 2 : kSlotGroup;
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = chunk_ptr[c];
  const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
  const uint32_t *cp = cols + p + lane;
  X acc = 0;
  // Groups of slots with unconditional loads (all column words, then all
  // gathers, so they are in flight together).  Slots past the row's width
  // read the next slice or the zero slack after the last one and are masked
  // to weight 0; a weight-0 slot contributes exactly 0 whatever it gathered.
  int k0 = 0;
  for (; k0 + 4 < width; k0 += G) lap_slots<G>(cp, x, k0, width, xi, acc);
  if (k0 < width) lap_slots<4>(cp, x, k0, width, xi, acc);
  return acc;
}

// The same row of L applied to two vectors from one read of the column words.
template <int G, typename X>
__device__ inline void lap_slots2(const uint32_t *__restrict__ cp, const X *__restrict__ x,
                                  const X *__restrict__ y, int k0, int width, X xi, X yi,
                                  X &ax, X &ay) {
  uint32_t w[G];
#pragma unroll
  for (int u = 0; u < G; ++u) w[u] = ld_stream(cp + (int64_t)(k0 + u) * 64);
#pragma unroll
  for (int u = 0; u < G; ++u) w[u] = (k0 + u < width) ? w[u] : 0u;
  X xv[G], yv[G];
#pragma unroll
  for (int u = 0; u < G; ++u) {
    xv[u] = x[colw_col(w[u])];
    yv[u] = y[colw_col(w[u])];
  }
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const X wt = (X)colw_wt(w[u]);
    ax += colw_wt(w[u]) ? wt * (xi - xv[u]) : (X)0;
    ay += colw_wt(w[u]) ? wt * (yi - yv[u]) : (X)0;
  }
}

template <typename X>
__device__ inline void lap_row2(const int64_t *__restrict__ chunk_ptr,
                                const uint32_t *__restrict__ cols, const X *__restrict__ x,
                                const X *__restrict__ y, int64_t row, X xi, X yi, X &ax, X &ay) {
  // 8 slots at a time: 8 words and 16 gathers in flight
  constexpr int G = kSlotGroup / 2;
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = chunk_ptr[c];
  const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
  const uint32_t *cp = cols + p + lane;
  ax = 0;
  ay = 0;
  int k0 = 0;
  for (; k0 + 4 < width; k0 += G) lap_slots2<G>(cp, x, y, k0, width, xi, yi, ax, ay);
  if (k0 < width) lap_slots2<4>(cp, x, y, k0, width, xi, yi, ax, ay);
}

// Gather-scatter row (Sec. 5): (L x)_e = deg_e x_e - sum of U over the row's
// vertex groups, U already holding the group sums of x.  Slots are read four
// at a time (loads in flight together); a slot without a group adds 0.
template <typename X>
__device__ inline X gs_row(const GsView &g, int64_t row, X xi) {
  const uint32_t *ep = g.ev + (row >> 6) * 64 * (int64_t)g.nv + (row & 63);
  double s = 0.0;
  for (int k0 = 0; k0 < g.nv; k0 += 4) {
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = (k0 + u < g.nv) ? ld_stream(ep + (int64_t)(k0 + u) * 64) : kGsNone;
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (w[u] != kGsNone) ? g.U[w[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u];
  }
  return (X)((double)g.deg[row] * (double)xi - s);
}

// U_gi = sum of x over the rows gent[a..b) of group gi, in ascending row
// order (FP64); four rows' loads are issued before they are added (eight
// measured slower: fewer waves in flight).
template <typename X>
__device__ inline void gs_group_sum(const GsView &g, int64_t gi, uint32_t a, uint32_t b,
                                    const X *__restrict__ x) {
  double s = 0.0;
  uint32_t k = a;
  for (; k + 4 <= b; k += 4) {
    int32_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = g.gent[k + u];
    X v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = x[r[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += (double)v[u];
  }
  for (; k < b; ++k) s += (double)x[g.gent[k]];
  g.U[gi] = s;
}

}  // namespace rsb
