// sweep.hip -- sweep over the Fiedler pair for the smallest cut.
//
// The paper notes (Sec. 9) that on meshes with a degenerate or nearly
// degenerate Fiedler pair the eigen-solver returns whatever combination of
// the pair the start vector held, and suggests searching the combinations of
// the two eigenvectors for the minimum cut.  Thick-restart Lanczos already
// holds the second Ritz pair when the pair is nearly degenerate (an exactly
// degenerate pair has a single direction in one Krylov space).  For every
// segment whose second Ritz value lies within sweep_gap (relative) of the
// first: y2 is orthonormalised against u0 and y1, both vectors get the
// canonical sign, and for a = k pi / S, k = 0..S-1, the combination
// cos(a) y1 + sin(a) y2 is split by the usual rule and its cut weight summed
// (exact integer sums).  The combination with the smallest cut (ties: the
// smallest k) replaces y1.  All segments of a level are swept together.
//
// The same second Ritz vector also seeds the next level (warm start, an
// addition: the paper leaves the start vector open): scaled to unit
// root-mean-square on the segment's cut component, it is kept per element
// and the children's solves start from it plus a small random part.
#include <cmath>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

struct SweepSeg {
  int32_t on;                  // sweep this segment
  int32_t best;                // angle index of the smallest cut so far
  double a, b, inv;            // y2_hat = (y2 - a u0 - b y1) * inv
  unsigned long long cut;      // cut of the current angle (each edge twice)
  unsigned long long best_cut;
};

struct SwArgs {
  const BlkDev *blk;
  const GrpDev *grp;
  const SegDev *seg;
  const SegState *st;
  double *part, *gpart;
  unsigned *scnt;
  int ps;
  const int32_t *root;
  const double *tvals;
  int nkcap;
  double gap;
  double min_perp2;            // least squared norm of y2 off u0 and y1 to sweep
  SweepSeg *sw;
};

__device__ inline bool in_cut(const int32_t *root, const SegState &S, int64_t row) {
  return S.solve && S.strad >= 0 && root[row] == S.strad;
}

// partial sums over a tile: sum y2, sum y1 y2, sum y2^2 (rows being cut)
__global__ __launch_bounds__(kBlock) void k_sw_dots(SwArgs a, const double *__restrict__ y1,
                                                    const double *__restrict__ y2) {
  __shared__ double red[4 * 3];
  __shared__ double vals[3];
  const int lb = blockIdx.x;
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int lr = threadIdx.x; lr < b.nrows; lr += kBlock) {
    const int64_t row = b.row0 + lr;
    if (!in_cut(a.root, S, row)) continue;
    const double v = y2[row];
    acc[0] += v;
    acc[1] += y1[row] * v;
    acc[2] += v * v;
  }
  block_reduce_into<3>(acc, red, vals, 3);
  write_partials(a, lb, vals, 3);
}

// per segment: the orthonormalisation of y2 and the gap test
__global__ __launch_bounds__(kBlock) void k_sw_setup(SwArgs a) {
  __shared__ double vals[3];
  const int g = blockIdx.x;
  if (!group_reduce(a, g, vals, 3)) return;
  if (threadIdx.x != 0) return;
  const int s = a.grp[g].seg;
  const SegState &S = a.st[s];
  SweepSeg w{};
  const bool pair = S.solve && S.strad >= 0 && S.nnext >= 2 && a.nkcap >= 2;
  const double t1 = pair ? a.tvals[(int64_t)s * a.nkcap] : 0.0;
  const double t2 = pair ? a.tvals[(int64_t)s * a.nkcap + 1] : 0.0;
  if (pair && t2 - t1 <= a.gap * t1) {
    const double ca = S.invsqrt_nc * vals[0];  // u0^T y2
    const double cb = vals[1];                 // y1^T y2
    const double nn2 = vals[2] - ca * ca - cb * cb;
    if (nn2 > a.min_perp2) {
      w.on = 1;
      w.a = ca;
      w.b = cb;
      w.inv = 1.0 / sqrt(nn2);
    }
  }
  a.sw[s] = w;
}

__global__ void k_sw_y2hat(SwArgs a, const SegDev *__restrict__ segs, int nseg,
                           const int32_t *__restrict__ row_seg, const double *__restrict__ y1,
                           const double *__restrict__ y2, int64_t nrows, double *__restrict__ y2h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int s = row_seg[i];
  double v = 0.0;
  if (s >= 0) {
    const SweepSeg w = a.sw[s];
    const SegState &S = a.st[s];
    if (w.on && in_cut(a.root, S, i)) v = (y2[i] - w.a * S.invsqrt_nc - w.b * y1[i]) * w.inv;
  }
  y2h[i] = v;
}

// y = c y1 + s y2_hat on swept segments (per-segment angle when coef_best)
__global__ void k_sw_combine(const SwArgs a, const int32_t *__restrict__ row_seg,
                             const double *__restrict__ y1, const double *__restrict__ y2h,
                             double c, double sn, const double *__restrict__ coef, int nangles,
                             int64_t nrows, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int s = row_seg[i];
  double v = y1[i];
  if (s >= 0 && a.sw[s].on && in_cut(a.root, a.st[s], i)) {
    double cc = c, ss = sn;
    if (coef) {
      const int k = a.sw[s].best;
      cc = coef[k];
      ss = coef[nangles + k];
    }
    v = cc * y1[i] + ss * y2h[i];
  }
  out[i] = v;
}

__global__ void k_sw_cut_reset(SweepSeg *sw, int nseg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) sw[s].cut = 0;
}

// cut weight of the sides on swept segments (each edge from both ends)
__global__ __launch_bounds__(kBlock) void k_sw_cut(SwArgs a, const int32_t *__restrict__ row_seg,
                                                   const int64_t *__restrict__ chunk_ptr,
                                                   const uint32_t *__restrict__ cols,
                                                   const uint8_t *__restrict__ side,
                                                   int64_t nrows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int s = i < nrows ? row_seg[i] : -1;
  unsigned long long cw = 0;
  if (s >= 0 && a.sw[s].on) {
    const int64_t c = i >> 6;
    const int64_t p = chunk_ptr[c];
    const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
    const uint32_t *cp = cols + p + (i & 63);
    const uint8_t si = side[i];
    for (int k = 0; k < width; ++k) {
      const uint32_t word = cp[(int64_t)k * 64];
      const uint32_t w = colw_wt(word);
      if (w && side[colw_col(word)] != si) cw += w;
    }
  }
  // rows of a wavefront belong to one segment (segments are 64-row aligned)
  for (int off = kWave / 2; off > 0; off >>= 1) cw += __shfl_xor(cw, off, kWave);
  if (lane == 0 && cw) atomicAdd(&a.sw[s].cut, cw);
}

__global__ void k_sw_pick(SweepSeg *sw, int nseg, int k) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg || !sw[s].on) return;
  if (k == 0 || sw[s].cut < sw[s].best_cut) {
    sw[s].best = k;
    sw[s].best_cut = sw[s].cut;
  }
}

__global__ void k_sw_row_seg(const BlkDev *__restrict__ blk, int32_t *__restrict__ row_seg) {
  const BlkDev b = blk[blockIdx.x];
  for (int lr = threadIdx.x; lr < b.nrows; lr += kBlock) row_seg[b.row0 + lr] = b.seg;
}

// warm start: partial sums of y2^2 over the rows being cut of a tile
__global__ __launch_bounds__(kBlock) void k_wu_dots(SwArgs a, const double *__restrict__ y2) {
  __shared__ double red[4];
  __shared__ double vals[1];
  const int lb = blockIdx.x;
  const BlkDev b = a.blk[lb];
  const SegState S = a.st[b.seg];
  double acc[1] = {0.0};
  for (int lr = threadIdx.x; lr < b.nrows; lr += kBlock) {
    const int64_t row = b.row0 + lr;
    if (in_cut(a.root, S, row)) acc[0] += y2[row] * y2[row];
  }
  block_reduce_into<1>(acc, red, vals, 1);
  write_partials(a, lb, vals, 1);
}

// scale = sqrt(component size) / ||y2|| (0: no second Ritz vector)
__global__ __launch_bounds__(kBlock) void k_wu_scale(SwArgs a, double *__restrict__ scale) {
  __shared__ double vals[1];
  const int g = blockIdx.x;
  if (!group_reduce(a, g, vals, 1)) return;
  if (threadIdx.x != 0) return;
  const int s = a.grp[g].seg;
  const SegState &S = a.st[s];
  const bool pair = S.solve && S.strad >= 0 && S.nnext >= 2 && vals[0] > 0.0;
  scale[s] = pair ? 1.0 / (S.invsqrt_nc * sqrt(vals[0])) : 0.0;
}

__global__ void k_wu_scatter(SwArgs a, const int32_t *__restrict__ row_seg,
                             const int32_t *__restrict__ orig, const double *__restrict__ scale,
                             const double *__restrict__ y2, int64_t nrows,
                             double *__restrict__ warm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int s = row_seg[i];
  if (s < 0 || orig[i] < 0) return;
  const double sc = scale[s];
  if (sc > 0.0 && in_cut(a.root, a.st[s], i)) warm[orig[i]] = y2[i] * sc;
}

}  // namespace

void warm_update(Level &L, CompDev &C, SolveDev &S, const double *y2, double *warm, Ctx &ctx) {
  const int64_t n = L.nrows;
  if (n == 0 || L.nseg == 0) return;
  hipStream_t st = ctx.stream;
  DevBuf<double> scale(ctx, L.nseg);
  DevBuf<int32_t> row_seg(ctx, n);
  SwArgs a{};
  a.blk = L.d_blk.get();
  a.grp = L.d_grp.get();
  a.seg = L.d_seg.get();
  a.st = S.st.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.root = C.root.get();
  k_sw_row_seg<<<L.nblk, kBlock, 0, st>>>(L.d_blk.get(), row_seg.get());
  k_wu_dots<<<L.nblk, kBlock, 0, st>>>(a, y2);
  k_wu_scale<<<L.ngrp, kBlock, 0, st>>>(a, scale.get());
  k_wu_scatter<<<grid_for(n, kBlock), kBlock, 0, st>>>(a, row_seg.get(), L.orig.get(),
                                                       scale.get(), y2, n, warm);
  RSB_LAUNCHED();
}

void fiedler_sweep(Level &L, CompDev &C, SolveDev &S, double *y64, const double *y2, int nangles,
                   double sweep_gap, int *swept, int *moved, Ctx &ctx, double min_perp2,
                   std::vector<int32_t> *on_out) {
  const int64_t n = L.nrows;
  if (on_out) on_out->assign(L.nseg, 0);
  if (n == 0 || L.nseg == 0 || nangles < 1) return;
  hipStream_t st = ctx.stream;
  DevBuf<SweepSeg> sw(ctx, L.nseg);
  DevBuf<int32_t> row_seg(ctx, n);
  SwArgs a{};
  a.blk = L.d_blk.get();
  a.grp = L.d_grp.get();
  a.seg = L.d_seg.get();
  a.st = S.st.get();
  a.part = S.part.get();
  a.gpart = S.gpart.get();
  a.scnt = S.scnt.get();
  a.ps = S.pstride;
  a.root = C.root.get();
  a.tvals = S.tvals.get();
  a.nkcap = S.nkcap;
  a.gap = sweep_gap;
  a.min_perp2 = min_perp2;
  a.sw = sw.get();
  // tiles cover every row of the level
  k_sw_row_seg<<<L.nblk, kBlock, 0, st>>>(L.d_blk.get(), row_seg.get());
  k_sw_dots<<<L.nblk, kBlock, 0, st>>>(a, y64, y2);
  k_sw_setup<<<L.ngrp, kBlock, 0, st>>>(a);
  RSB_LAUNCHED();
  std::vector<SweepSeg> hs(L.nseg);
  RSB_HIP(hipMemcpyAsync(hs.data(), sw.get(), L.nseg * sizeof(SweepSeg), hipMemcpyDeviceToHost,
                         st));
  RSB_HIP(hipStreamSynchronize(st));
  int on = 0;
  for (auto &w : hs) on += w.on;
  if (swept) *swept += on;
  if (on_out)
    for (int i = 0; i < L.nseg; ++i) (*on_out)[i] = hs[i].on;
  if (on == 0) return;
  const unsigned g = grid_for(n, kBlock), gs = grid_for(L.nseg, 64);
  DevBuf<double> y2h(ctx, n), yk(ctx, n);
  DevBuf<uint8_t> side(ctx, n);
  k_sw_y2hat<<<g, kBlock, 0, st>>>(a, L.d_seg.get(), L.nseg, row_seg.get(), y64, y2, n,
                                   y2h.get());
  RSB_LAUNCHED();
  canonical_sign_level(L, C, S, y64, ctx);
  canonical_sign_level(L, C, S, y2h.get(), ctx);
  std::vector<double> coef(2 * nangles);
  for (int k = 0; k < nangles; ++k) {
    const double ang = M_PI * (double)k / (double)nangles;
    coef[k] = std::cos(ang);
    coef[nangles + k] = std::sin(ang);
  }
  for (int k = 0; k < nangles; ++k) {
    k_sw_combine<<<g, kBlock, 0, st>>>(a, row_seg.get(), y64, y2h.get(), coef[k],
                                       coef[nangles + k], nullptr, nangles, n, yk.get());
    RSB_LAUNCHED();
    split_level(L, C, S, yk.get(), side.get(), ctx);
    k_sw_cut_reset<<<gs, 64, 0, st>>>(sw.get(), L.nseg);
    k_sw_cut<<<g, kBlock, 0, st>>>(a, row_seg.get(), L.chunk_ptr.get(), L.cols.get(), side.get(),
                                   n);
    k_sw_pick<<<gs, 64, 0, st>>>(sw.get(), L.nseg, k);
    RSB_LAUNCHED();
  }
  DevBuf<double> dcoef(ctx, 2 * nangles);
  RSB_HIP(hipMemcpyAsync(dcoef.get(), coef.data(), 2 * nangles * sizeof(double),
                         hipMemcpyHostToDevice, st));
  k_sw_combine<<<g, kBlock, 0, st>>>(a, row_seg.get(), y64, y2h.get(), 0.0, 0.0, dcoef.get(),
                                     nangles, n, yk.get());
  RSB_LAUNCHED();
  RSB_HIP(hipMemcpyAsync(y64, yk.get(), n * sizeof(double), hipMemcpyDeviceToDevice, st));
  RSB_HIP(hipMemcpyAsync(hs.data(), sw.get(), L.nseg * sizeof(SweepSeg), hipMemcpyDeviceToHost,
                         st));
  RSB_HIP(hipStreamSynchronize(st));
  if (moved)
    for (auto &w : hs) *moved += (w.on && w.best != 0);
}

}  // namespace rsb
