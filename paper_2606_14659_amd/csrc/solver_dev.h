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

// The level's Laplacian as the row kernels read it: the sliced-ELL words and
// their packed copy (per-slice meta; kPlainSlice: words only).
struct SellRef {
  const int64_t *chunk_ptr;
  const uint32_t *cols;
  const uint32_t *pk;
  const int4 *meta;
  const TileStage *stage;  // null: no tile is staged
  const int4 *lmeta;
};

// The staging of the tile starting at row0, if it has one.
__device__ inline bool tile_staged(const SellRef &m, int64_t row0) {
  return m.stage != nullptr && m.stage[row0 >> 6].nint > 0;
}

// Copies the tile's intervals of x into xs (LDS); the caller synchronises.
template <typename X>
__device__ inline void stage_copy(const SellRef &m, int64_t row0, const X *__restrict__ x, X *xs,
                                  int tid, int nt) {
  const TileStage &ts = m.stage[row0 >> 6];
  const int nint = ts.nint;
  for (int k = 0; k < nint; ++k) {
    const X *src = x + ts.lo[k];
    X *dst = xs + ts.off[k];
    const int len = ts.len[k];
    for (int i = tid; i < len; i += nt) dst[i] = src[i];
  }
}

// Sliced-ELL Laplacian row in difference form: sum_j w_ij (x_i - x_j),
// accumulated in the vector type in slot order (paper Sec. 5: the action of L
// on x); a padding slot leaves the sum as it is.  The words are read in groups
// of G slots, exactly the row's width (loads past it masked off); the next
// group's words are issued before the current group's gathers are consumed,
// so words and gathers are in flight together.
template <int G>
__device__ inline void lap_words(const uint32_t *__restrict__ cp, int k0, int width,
                                 uint32_t (&w)[G]) {
#pragma unroll
  for (int u = 0; u < G; ++u) w[u] = (k0 + u < width) ? ld_stream(cp + (int64_t)(k0 + u) * 64) : 0u;
}

// w (x_i - x_j) added to the row's sum as one fused multiply-add, so that the
// 32-bit and the packed reading of a slice give the same bits.
__device__ inline float lap_fma(float w, float d, float acc) { return __builtin_fmaf(w, d, acc); }
__device__ inline double lap_fma(double w, double d, double acc) { return __builtin_fma(w, d, acc); }

// One slot entry of a packed slice: weight, and the column as an offset from
// the row (the slice's window base for its cluster added).
struct PkEntry {
  uint32_t wt;
  int32_t col;
};

__device__ inline PkEntry pk_entry(uint32_t half, int32_t row, const int4 &mb) {
  const uint32_t cid = (half >> kPackOffBits) & (kPackClusters - 1);
  const int32_t base = cid == 0 ? mb.x : cid == 1 ? mb.y : cid == 2 ? mb.z : mb.w;
  return {half >> 12, row + base + (int32_t)(half & ((1u << kPackOffBits) - 1))};
}

template <typename X, int G>
__device__ inline X lap_row_plain(const uint32_t *__restrict__ cp, int width,
                                  const X *__restrict__ x, X xi) {
  X acc = 0;
  uint32_t w[G];
  lap_words<G>(cp, 0, width, w);
  for (int k0 = 0; k0 < width; k0 += G) {
    X xv[G];
    uint32_t wc[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      wc[u] = w[u];
      xv[u] = colw_wt(wc[u]) ? x[colw_col(wc[u])] : (X)0;
    }
    lap_words<G>(cp, k0 + G, width, w);
#pragma unroll
    for (int u = 0; u < G; ++u)
      acc = colw_wt(wc[u]) ? lap_fma((X)colw_wt(wc[u]), xi - xv[u], acc) : acc;
  }
  return acc;
}

// Packed slice: GW words (2 GW slots) per group.
template <typename X, int GW>
__device__ inline X lap_row_packed(const uint32_t *__restrict__ cp, int nw, const int4 &mb,
                                   int32_t row, const X *__restrict__ x, X xi) {
  X acc = 0;
  uint32_t w[GW];
  lap_words<GW>(cp, 0, nw, w);
  for (int k0 = 0; k0 < nw; k0 += GW) {
    X xv[2 * GW];
    PkEntry e[2 * GW];
#pragma unroll
    for (int u = 0; u < GW; ++u) {
      e[2 * u] = pk_entry(w[u] & 0xffffu, row, mb);
      e[2 * u + 1] = pk_entry(w[u] >> 16, row, mb);
    }
#pragma unroll
    for (int u = 0; u < 2 * GW; ++u) xv[u] = e[u].wt ? x[e[u].col] : (X)0;
    lap_words<GW>(cp, k0 + GW, nw, w);
#pragma unroll
    for (int u = 0; u < 2 * GW; ++u) acc = e[u].wt ? lap_fma((X)e[u].wt, xi - xv[u], acc) : acc;
  }
  return acc;
}

// STAGED: the row's tile has its intervals of x in xs (LDS); a packed slice
// then gathers there through its LDS bases, a slice in words from x.
template <typename X, bool STAGED = false>
__device__ inline X lap_row(const SellRef &m, const X *__restrict__ x, const X *xs, int64_t row,
                            X xi) {
  constexpr int G = sizeof(X) == 8 ? kSlotGroup / 2 : kSlotGroup;
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = m.chunk_ptr[c];
  const int width = (int)((m.chunk_ptr[c + 1] - p) >> 6);
  const int4 mb = m.meta[c];
  if (mb.x != kPlainSlice) {
    const uint32_t *cp = m.pk + packed_slice_word(p, c) + lane;
    if (STAGED) return lap_row_packed<X, G / 2>(cp, (width + 1) >> 1, m.lmeta[c], (int32_t)row, xs, xi);
    return lap_row_packed<X, G / 2>(cp, (width + 1) >> 1, mb, (int32_t)row, x, xi);
  }
  return lap_row_plain<X, G>(m.cols + p + lane, width, x, xi);
}

template <typename X>
__device__ inline X lap_row(const SellRef &m, const X *__restrict__ x, int64_t row, X xi) {
  return lap_row<X, false>(m, x, nullptr, row, xi);
}

// The same row of L applied to two vectors from one read of the matrix.
template <typename X>
__device__ inline void lap_acc2(uint32_t wt, X xv, X yv, X xi, X yi, X &ax, X &ay) {
  ax = wt ? lap_fma((X)wt, xi - xv, ax) : ax;
  ay = wt ? lap_fma((X)wt, yi - yv, ay) : ay;
}

// Two FP64 vectors stored interleaved (x in .x, y in .y): one 16-byte gather
// per slot for both.
__device__ inline void lap_row2i(const SellRef &m, const double2 *__restrict__ xy, int64_t row,
                                 double xi, double yi, double &ax, double &ay) {
  constexpr int G = kSlotGroup / 2;
  const int64_t c = row >> 6;
  const int lane = (int)(row & 63);
  const int64_t p = m.chunk_ptr[c];
  const int width = (int)((m.chunk_ptr[c + 1] - p) >> 6);
  const int4 mb = m.meta[c];
  ax = 0;
  ay = 0;
  if (mb.x != kPlainSlice) {
    constexpr int GW = G / 2;
    const uint32_t *cp = m.pk + packed_slice_word(p, c) + lane;
    const int nw = (width + 1) >> 1;
    uint32_t w[GW];
    lap_words<GW>(cp, 0, nw, w);
    for (int k0 = 0; k0 < nw; k0 += GW) {
      double2 v[2 * GW];
      PkEntry e[2 * GW];
#pragma unroll
      for (int u = 0; u < GW; ++u) {
        e[2 * u] = pk_entry(w[u] & 0xffffu, (int32_t)row, mb);
        e[2 * u + 1] = pk_entry(w[u] >> 16, (int32_t)row, mb);
      }
#pragma unroll
      for (int u = 0; u < 2 * GW; ++u) v[u] = e[u].wt ? xy[e[u].col] : make_double2(0.0, 0.0);
      lap_words<GW>(cp, k0 + GW, nw, w);
#pragma unroll
      for (int u = 0; u < 2 * GW; ++u) lap_acc2(e[u].wt, v[u].x, v[u].y, xi, yi, ax, ay);
    }
    return;
  }
  const uint32_t *cp = m.cols + p + lane;
  uint32_t w[G];
  lap_words<G>(cp, 0, width, w);
  for (int k0 = 0; k0 < width; k0 += G) {
    double2 v[G];
    uint32_t wc[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      wc[u] = w[u];
      v[u] = colw_wt(wc[u]) ? xy[colw_col(wc[u])] : make_double2(0.0, 0.0);
    }
    lap_words<G>(cp, k0 + G, width, w);
#pragma unroll
    for (int u = 0; u < G; ++u) lap_acc2(colw_wt(wc[u]), v[u].x, v[u].y, xi, yi, ax, ay);
  }
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
