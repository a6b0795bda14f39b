// amg.hip -- aggregation multigrid preconditioner of the inverse-iteration
// solves (paper Sec. 7, Alg. 3) for all segments of a bisection level.
//
// Hierarchy.  Level 0 is the bisection level itself (its sliced-ELL
// Laplacian with packed weights); only the rows of each segment's component
// being cut take part ("live" rows).  Level l+1 collapses pairs of level-l
// rows: J is the Boolean piecewise-constant prolongation and J^T L J is again
// a graph Laplacian whose weight between two aggregates is the sum of the
// weights between their members (edges inside an aggregate drop out), so all
// levels hold exact integer weights.  The pairs come from a handshake
// matching (the paper pairs consecutive elements of an RCB order, which
// needs coordinates the partitioner does not have): in each of kMatchRounds
// rounds every unmatched live row proposes to its unmatched neighbour of
// largest (weight, pair hash), ties to the smaller global id, and mutual
// proposals are matched.  The pair hash is the splitmix64 output for counter
// max(gid) of the stream started at min(gid), so both ends rank an edge
// alike and the hierarchy does not depend on row numbering or on which
// other segments share the level.  A coarse row is numbered by its first
// member and carries the smaller global id of its members.  A segment stops
// coarsening when the next level would keep more than 90% of its rows, when
// a pair has more than kAmgCandCap entries in its two rows, or after
// kAmgMaxLevels levels; coarse levels hold only the segments still
// coarsening.  Coarse levels are sliced ELL (64-row slices, slot-major) with
// separate column and 32-bit weight words, columns ascending in every row.
//
// V-cycle (Alg. 3, damped Jacobi with weight sigma): u = sigma D f, r = f - Lu,
// then nsmooth times u += sigma D r, r = f - L u; restrict f_c = J^T r; the
// coarse cycle; u += J e_c; then nsmooth times r = f - L u, u += sigma D r
// (the printed algorithm subtracts L u from an already updated residual
// after the coarse correction; the true residual is used here).  A segment's
// coarsest level runs only the first part (smoothing).  Every launch covers
// all segments; rows of segments whose solve has ended are skipped.  Each
// smoothing step is one launch: the Jacobi update of a neighbour (and the
// coarse correction before the first post-smoothing step) is formed on the
// fly where the residual gathers it, and results alternate between two
// buffers per level.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

constexpr int kMatchRounds = 4;
constexpr int kAmgMaxLevels = 40;
constexpr int kAmgCandCap = 1024;

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

// Laplacian slots of one row, level 0 (packed words) or coarse (separate).
struct MatDev {
  const int64_t *chunk_ptr;
  const uint32_t *packed;  // level 0
  const int32_t *col;      // coarse levels
  const uint32_t *wgt;
};

template <bool PACKED>
struct RowSlots {
  const int64_t base;
  const int width;
  const MatDev &m;
  __device__ RowSlots(const MatDev &mm, int64_t row)
      : base(mm.chunk_ptr[row >> 6] + (row & 63)),
        width((int)((mm.chunk_ptr[(row >> 6) + 1] - mm.chunk_ptr[row >> 6]) >> 6)),
        m(mm) {}
  // column and weight of slot k (weight 0: padding)
  __device__ void get(int k, int64_t &j, uint32_t &w) const {
    if (PACKED) {
      const uint32_t word = m.packed[base + (int64_t)k * 64];
      j = colw_col(word);
      w = colw_wt(word);
    } else {
      j = m.col[base + (int64_t)k * 64];
      w = m.wgt[base + (int64_t)k * 64];
    }
  }
};

// sum_j w_ij (u_i - v(j)) over the row's slots in slot (ascending column)
// order, as the oracle sums it.  Slots are taken in groups: the group's
// column words first, then its gathers, so that they are in flight
// together.  Padding slots gather the row itself and add nothing.
template <bool PACKED, typename V>
__device__ inline double row_diff_sum(const MatDev &m, int64_t i, double ui, V v) {
  constexpr int G = 8;
  const RowSlots<PACKED> rs(m, i);
  double acc = 0.0;
  for (int k0 = 0; k0 < rs.width; k0 += G) {
    int64_t j[G];
    uint32_t w[G];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      j[t] = i;
      w[t] = 0;
      if (k0 + t < rs.width) rs.get(k0 + t, j[t], w[t]);
      if (w[t] == 0) j[t] = i;
    }
    double x[G];
#pragma unroll
    for (int t = 0; t < G; ++t) x[t] = v(j[t]);
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (w[t]) acc += (double)w[t] * (ui - x[t]);
  }
  return acc;
}

__device__ inline uint32_t pair_priority(int64_t ga, int64_t gb) {
  const uint64_t lo = (uint64_t)(ga < gb ? ga : gb), hi = (uint64_t)(ga < gb ? gb : ga);
  uint64_t z = lo + hi * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)(z >> 32);
}

// Row is solved (its segment's CG still runs); st == nullptr: always.
__device__ inline bool seg_running(const SegState *st, int32_t seg) {
  if (seg < 0) return false;
  if (!st) return true;
  const SegState &S = st[seg];
  return S.active && !S.cg_done;
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// Level 0: segment of every live row (-1 otherwise), row length, 1/L_ii.
__global__ __launch_bounds__(kBlock) void k_amg_init0(const BlkDev *__restrict__ blk,
                                                      const SegState *__restrict__ st,
                                                      const int32_t *__restrict__ root,
                                                      MatDev m, int32_t *__restrict__ seg,
                                                      int32_t *__restrict__ rowlen,
                                                      double *__restrict__ dinv) {
  const BlkDev b = blk[blockIdx.x];
  for (int lr = threadIdx.x; lr < b.nrows; lr += kBlock) {
    const int64_t row = b.row0 + lr;
    const SegState &S = st[b.seg];
    const bool live = S.solve && root[row] == S.strad;
    int len = 0;
    uint64_t deg = 0;
    if (live) {
      RowSlots<true> rs(m, row);
      for (int k = 0; k < rs.width; ++k) {
        int64_t j;
        uint32_t w;
        rs.get(k, j, w);
        len += (w != 0);
        deg += w;
      }
    }
    seg[row] = live ? b.seg : -1;
    rowlen[row] = len;
    dinv[row] = deg ? 1.0 / (double)deg : 0.0;
  }
}

__global__ void k_amg_fill(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_amg_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// mate: -2 not taking part, -1 unmatched, else the partner (itself: single).
__global__ void k_amg_match_init(const int32_t *__restrict__ seg, int64_t n,
                                 int32_t *__restrict__ mate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) mate[i] = seg[i] >= 0 ? -1 : -2;
}

template <bool PACKED>
__global__ void k_amg_propose(MatDev m, const int32_t *__restrict__ gid,
                              const int32_t *__restrict__ mate, int64_t n,
                              int32_t *__restrict__ prop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t best = -1;
  if (mate[i] == -1) {
    uint32_t bw = 0, bh = 0;
    int32_t bg = 0;
    const int32_t gi = gid[i];
    RowSlots<PACKED> rs(m, i);
    for (int k = 0; k < rs.width; ++k) {
      int64_t j;
      uint32_t w;
      rs.get(k, j, w);
      if (w == 0 || mate[j] != -1) continue;
      const int32_t gj = gid[j];
      const uint32_t h = pair_priority(gi, gj);
      const bool better = best < 0 || w > bw || (w == bw && h > bh) ||
                          (w == bw && h == bh && gj < bg);
      if (better) {
        best = (int32_t)j;
        bw = w;
        bh = h;
        bg = gj;
      }
    }
  }
  prop[i] = best;
}

__global__ void k_amg_accept(const int32_t *__restrict__ prop, int64_t n,
                             int32_t *__restrict__ mate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || mate[i] != -1) return;
  const int32_t p = prop[i];
  if (p >= 0 && prop[p] == (int32_t)i) mate[i] = p;
}

// Unmatched rows become single; per-segment counts of live rows, coarse
// rows and pairs too wide for the coarse-row kernel.  A wavefront whose
// rows all belong to one segment adds its totals with one atomic each.
__global__ __launch_bounds__(kBlock) void k_amg_count(
    const int32_t *__restrict__ seg, const int32_t *__restrict__ rowlen, int64_t n,
    int32_t *__restrict__ mate, int32_t *__restrict__ nrow_s, int32_t *__restrict__ ncoarse_s,
    int32_t *__restrict__ wide_s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t s = i < n ? seg[i] : -1;
  int live = 0, lead = 0, wide = 0;
  if (s >= 0) {
    int32_t p = mate[i];
    if (p == -1) {
      p = (int32_t)i;
      mate[i] = p;
    }
    live = 1;
    if (p >= i) {
      lead = 1;
      wide = (rowlen[i] + (p != i ? rowlen[p] : 0) > kAmgCandCap) ? 1 : 0;
    }
  }
  const uint64_t act = __ballot(s >= 0);
  if (act == 0) return;
  const int first = __ffsll((unsigned long long)act) - 1;
  const int32_t s0 = __shfl(s, first, kWave);
  const bool uniform = __ballot(s >= 0 && s != s0) == 0;
  if (uniform) {
    const int nl = wave_sum_i(live), nc = wave_sum_i(lead), nw = wave_sum_i(wide);
    if (lane == first) {
      atomicAdd(&nrow_s[s0], nl);
      atomicAdd(&ncoarse_s[s0], nc);
      if (nw) atomicOr(&wide_s[s0], 1);
    }
  } else if (s >= 0) {
    atomicAdd(&nrow_s[s], live);
    if (lead) atomicAdd(&ncoarse_s[s], 1);
    if (wide) atomicOr(&wide_s[s], 1);
  }
}

__global__ void k_amg_decide(int nseg, int level, const int32_t *__restrict__ nrow_s,
                             const int32_t *__restrict__ ncoarse_s,
                             const int32_t *__restrict__ wide_s, int32_t *__restrict__ cont) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int64_t nr = nrow_s[s], nc = ncoarse_s[s];
  cont[s] = (nr > 0 && !wide_s[s] && 10 * nc <= 9 * nr && level + 1 < kAmgMaxLevels) ? 1 : 0;
}

__global__ void k_amg_leaders(const int32_t *__restrict__ seg, const int32_t *__restrict__ mate,
                              const int32_t *__restrict__ cont, int64_t n,
                              int32_t *__restrict__ lead) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = seg[i];
  lead[i] = (s >= 0 && cont[s] && mate[i] >= i) ? 1 : 0;
}

// agg of every row of a continuing segment (-1 otherwise); the coarse rows'
// members, global ids and segments.
__global__ void k_amg_link(const int32_t *__restrict__ seg, const int32_t *__restrict__ gid,
                           const int32_t *__restrict__ mate, const int32_t *__restrict__ cont,
                           const int64_t *__restrict__ cidx, int64_t n, int32_t *__restrict__ agg,
                           int32_t *__restrict__ mem1, int32_t *__restrict__ gid1,
                           int32_t *__restrict__ seg1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = seg[i];
  if (s < 0 || !cont[s]) {
    agg[i] = -1;
    return;
  }
  const int32_t p = mate[i];
  const int64_t first = p < i ? p : i;
  const int64_t I = cidx[first];
  agg[i] = (int32_t)I;
  if (first == i) {
    mem1[2 * I] = (int32_t)i;
    mem1[2 * I + 1] = p != i ? p : -1;
    gid1[I] = p != i ? min(gid[i], gid[p]) : gid[i];
    seg1[I] = s;
  }
}

// Coarse rows, one wavefront each: the (aggregate, weight) entries of both
// members' rows into LDS, equal aggregates merged by summing their weights.
// Launched over the padded row count: padding rows (no members) get empty
// rows whose slots are all padding.
// PASS 0 writes the row length; PASS 1 the slots at their rank (ascending
// columns), padding slots up to the slice width, and 1/L_II.
template <bool PACKED, int PASS>
__global__ __launch_bounds__(kBlock) void k_amg_coarse(
    MatDev m, const int32_t *__restrict__ agg, const int32_t *__restrict__ mem1, int64_t n1,
    int32_t *__restrict__ rowlen1, const int64_t *__restrict__ chunk_ptr1,
    int32_t *__restrict__ col1, uint32_t *__restrict__ wgt1, double *__restrict__ dinv1,
    int *__restrict__ err) {
  constexpr int W = kBlock / kWave;
  __shared__ int32_t cc[W][kAmgCandCap];
  __shared__ uint32_t cw[W][kAmgCandCap];
  __shared__ uint64_t sumw[W][kAmgCandCap];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t I = (int64_t)blockIdx.x * W + wave;
  if (I >= n1) return;
  int32_t *c = cc[wave];
  uint32_t *cwt = cw[wave];
  uint64_t *sw = sumw[wave];
  int total = 0;
  for (int t = 0; t < 2; ++t) {
    const int32_t a = mem1[2 * I + t];
    if (a < 0) continue;
    RowSlots<PACKED> rs(m, a);
    for (int k0 = 0; k0 < rs.width; k0 += kWave) {
      const int k = k0 + lane;
      int64_t j = 0;
      uint32_t w = 0;
      if (k < rs.width) rs.get(k, j, w);
      const int32_t cj = w ? agg[j] : -1;
      const bool keep = w != 0 && cj != (int32_t)I;
      const uint64_t mask = __ballot(keep);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      // the wide-pair check at coarsening keeps total below the capacity
      if (keep && total + before < kAmgCandCap) {
        c[total + before] = cj;
        cwt[total + before] = w;
      }
      total += __popcll(mask);
    }
  }
  if (total > kAmgCandCap) {
    if (lane == 0) atomicOr(err, 1);
    return;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // first occurrence of each aggregate gets the summed weight, others 0
  for (int i = lane; i < total; i += kWave) {
    const int32_t v = c[i];
    uint64_t s = 0;
    bool first = true;
    for (int j = 0; j < total; ++j) {
      if (c[j] == v) {
        s += cwt[j];
        if (j < i) first = false;
      }
    }
    sw[i] = first ? s : 0;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int cnt = 0;
  uint64_t deg = 0;
  for (int i = lane; i < total; i += kWave) {
    cnt += (sw[i] != 0);
    deg += sw[i];
  }
  cnt = wave_sum_i(cnt);
  if (PASS == 0) {
    if (lane == 0) rowlen1[I] = cnt;
    return;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) deg += __shfl_xor(deg, off, kWave);
  const int64_t cb = chunk_ptr1[I >> 6] + (I & 63);
  const int width = (int)((chunk_ptr1[(I >> 6) + 1] - chunk_ptr1[I >> 6]) >> 6);
  for (int i = lane; i < total; i += kWave) {
    if (sw[i] == 0) continue;
    const int32_t v = c[i];
    int rank = 0;
    for (int j = 0; j < total; ++j) rank += (sw[j] != 0 && c[j] < v);
    if (sw[i] > 0xFFFFFFFFull) atomicOr(err, 2);
    col1[cb + (int64_t)rank * 64] = v;
    wgt1[cb + (int64_t)rank * 64] = (uint32_t)sw[i];
  }
  for (int k = cnt + lane; k < width; k += kWave) {
    col1[cb + (int64_t)k * 64] = (int32_t)I;
    wgt1[cb + (int64_t)k * 64] = 0u;
  }
  if (lane == 0) dinv1[I] = deg ? 1.0 / (double)deg : 0.0;
}

// Slots of every 64-row slice (its widest row) for a coarse level; padding
// rows past n1 have length 0 and no segment.
__global__ void k_amg_slice_slots(const int32_t *__restrict__ rowlen, int64_t n1, int64_t nchunks,
                                  int64_t *__restrict__ slots) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  int w = 0;
  for (int r = 0; r < 64; ++r) {
    const int64_t I = c * 64 + r;
    if (I < n1) w = max(w, rowlen[I]);
  }
  slots[c] = (int64_t)w * 64;
}

__global__ void k_amg_pad_rows(int64_t n1, int64_t n1pad, int32_t *__restrict__ seg1,
                               int32_t *__restrict__ rowlen1, double *__restrict__ dinv1,
                               int32_t *__restrict__ gid1, int32_t *__restrict__ mem1) {
  const int64_t I = n1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n1pad) return;
  seg1[I] = -1;
  rowlen1[I] = 0;
  dinv1[I] = 0.0;
  gid1[I] = 0;
  mem1[2 * I] = -1;
  mem1[2 * I + 1] = -1;
}

// ---------------------------------------------------------------------------
// V-cycle kernels (one thread per row of a level)
// ---------------------------------------------------------------------------

// Pre-smoothing, first step: u = sigma D f and r = f - L u, the neighbours'
// u_j = sigma D_j f_j formed from f_j on the fly.
template <bool PACKED>
__global__ void k_vc_pre0(MatDev m, const int32_t *__restrict__ seg,
                          const SegState *__restrict__ st, const double *__restrict__ dinv,
                          const double *__restrict__ f, double sigma, int64_t n,
                          double *__restrict__ u_out, double *__restrict__ r_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!seg_running(st, seg[i])) return;
  const double fi = f[i];
  const double ui = sigma * dinv[i] * fi;
  const double acc =
      row_diff_sum<PACKED>(m, i, ui, [&](int64_t j) { return sigma * dinv[j] * f[j]; });
  u_out[i] = ui;
  r_out[i] = fi - acc;
}

// Pre-smoothing step: u' = u + sigma D r and r' = f - L u' (neighbours' u'
// formed on the fly; new values go to the other buffers).
template <bool PACKED>
__global__ void k_vc_pre(MatDev m, const int32_t *__restrict__ seg,
                         const SegState *__restrict__ st, const double *__restrict__ dinv,
                         const double *__restrict__ f, const double *__restrict__ u_in,
                         const double *__restrict__ r_in, double sigma, int64_t n,
                         double *__restrict__ u_out, double *__restrict__ r_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!seg_running(st, seg[i])) return;
  const double ui = u_in[i] + sigma * dinv[i] * r_in[i];
  const double acc = row_diff_sum<PACKED>(
      m, i, ui, [&](int64_t j) { return u_in[j] + sigma * dinv[j] * r_in[j]; });
  u_out[i] = ui;
  r_out[i] = f[i] - acc;
}

// f_c = J^T r (coarse rows)
__global__ void k_vc_restrict(const int32_t *__restrict__ seg1, const int32_t *__restrict__ mem1,
                              const SegState *__restrict__ st, const double *__restrict__ r,
                              int64_t n1, double *__restrict__ f1) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n1) return;
  if (!seg_running(st, seg1[I])) return;
  const int32_t a = mem1[2 * I], b = mem1[2 * I + 1];
  f1[I] = b >= 0 ? r[a] + r[b] : r[a];
}

// u += J e_c in place (no smoothing steps after the coarse correction)
__global__ void k_vc_prolong(const int32_t *__restrict__ seg, const int32_t *__restrict__ agg,
                             const SegState *__restrict__ st, const double *__restrict__ e1,
                             int64_t n, double *__restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!seg_running(st, seg[i]) || agg[i] < 0) return;
  u[i] += e1[agg[i]];
}

// Post-smoothing step: r = f - L u, u' = u + sigma D r; with PROLONG the
// coarse correction u += J e_c is applied first (to the row and, on the
// fly, to its neighbours).  Rows whose segment stopped coarsening at this
// level keep u (copied to the output buffer).
template <bool PACKED, bool PROLONG>
__global__ void k_vc_post(MatDev m, const int32_t *__restrict__ seg,
                          const int32_t *__restrict__ agg, const SegState *__restrict__ st,
                          const double *__restrict__ dinv, const double *__restrict__ f,
                          const double *__restrict__ u_in, const double *__restrict__ e1,
                          double sigma, int64_t n, double *__restrict__ u_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!seg_running(st, seg[i])) return;
  const int32_t ai = agg[i];
  if (ai < 0) {
    u_out[i] = u_in[i];
    return;
  }
  const double ui = PROLONG ? u_in[i] + e1[ai] : u_in[i];
  // (neighbours of a row whose segment continues have an aggregate)
  const double acc = row_diff_sum<PACKED>(
      m, i, ui, [&](int64_t j) { return PROLONG ? u_in[j] + e1[agg[j]] : u_in[j]; });
  const double ri = f[i] - acc;
  u_out[i] = ui + sigma * dinv[i] * ri;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

void amg_setup(const LevelView &L, const int32_t *d_root, const SegState *d_st, AmgDev &A,
               Ctx &ctx) {
  A.lv.clear();
  A.lv.reserve(kAmgMaxLevels);
  hipStream_t s = ctx.stream;
  const int nseg = std::max(L.nseg, 1);
  A.lv.emplace_back();
  {
    AmgLevelDev &z = A.lv.back();
    z.n = L.nrows;
    z.mat = MatDevHost{L.chunk_ptr, L.cols, nullptr, nullptr};
    z.gid = L.gid;
    z.seg.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.rowlen.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.dinv.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.agg.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.u.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.u2.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.r.alloc(ctx, std::max<int64_t>(z.n, 1));
    z.r2.alloc(ctx, std::max<int64_t>(z.n, 1));
    if (z.n > 0) {
      // the cycle writes only live rows: the level-0 correction is zero on
      // every other row (other components, padding) for its callers
      k_amg_fill<<<grid_for(z.n, kBlock), kBlock, 0, s>>>(z.seg.get(), z.n, -1);
      k_amg_zero<<<grid_for(z.n, kBlock), kBlock, 0, s>>>(z.u.get(), z.n);
      k_amg_zero<<<grid_for(z.n, kBlock), kBlock, 0, s>>>(z.u2.get(), z.n);
      RSB_LAUNCHED();
    }
    if (L.nblk > 0) {
      MatDev m{L.chunk_ptr, L.cols, nullptr, nullptr};
      k_amg_init0<<<L.nblk, kBlock, 0, s>>>(L.blk, d_st, d_root, m, z.seg.get(), z.rowlen.get(),
                                            z.dinv.get());
      RSB_LAUNCHED();
    }
  }
  DevBuf<int32_t> mate, prop, nrow_s(ctx, nseg), ncoarse_s(ctx, nseg), wide_s(ctx, nseg),
      cont(ctx, nseg), lead;
  DevBuf<int64_t> cidx, ntot(ctx, 1);
  DevBuf<int> err(ctx, 1);
  k_amg_fill<<<1, 1, 0, s>>>(err.get(), 1, 0);
  RSB_LAUNCHED();
  for (int l = 0; l + 1 < kAmgMaxLevels; ++l) {
    AmgLevelDev &F = A.lv.back();
    const int64_t n = F.n;
    if (n == 0) break;
    const bool packed = (l == 0);
    MatDev m{F.mat.chunk_ptr, F.mat.packed, F.mat.col, F.mat.wgt};
    mate.alloc(ctx, n);
    prop.alloc(ctx, n);
    const unsigned g = grid_for(n, kBlock);
    k_amg_match_init<<<g, kBlock, 0, s>>>(F.seg.get(), n, mate.get());
    for (int round = 0; round < kMatchRounds; ++round) {
      if (packed)
        k_amg_propose<true><<<g, kBlock, 0, s>>>(m, F.gid, mate.get(), n, prop.get());
      else
        k_amg_propose<false><<<g, kBlock, 0, s>>>(m, F.gid, mate.get(), n, prop.get());
      k_amg_accept<<<g, kBlock, 0, s>>>(prop.get(), n, mate.get());
    }
    const unsigned gs = grid_for(nseg, kBlock);
    k_amg_fill<<<gs, kBlock, 0, s>>>(nrow_s.get(), nseg, 0);
    k_amg_fill<<<gs, kBlock, 0, s>>>(ncoarse_s.get(), nseg, 0);
    k_amg_fill<<<gs, kBlock, 0, s>>>(wide_s.get(), nseg, 0);
    k_amg_count<<<g, kBlock, 0, s>>>(F.seg.get(), F.rowlen.get(), n, mate.get(), nrow_s.get(),
                                     ncoarse_s.get(), wide_s.get());
    k_amg_decide<<<gs, kBlock, 0, s>>>(L.nseg, l, nrow_s.get(), ncoarse_s.get(), wide_s.get(),
                                       cont.get());
    lead.alloc(ctx, n);
    cidx.alloc(ctx, n);
    k_amg_leaders<<<g, kBlock, 0, s>>>(F.seg.get(), mate.get(), cont.get(), n, lead.get());
    RSB_LAUNCHED();
    scan_exclusive(lead.get(), n, cidx.get(), ntot.get(), ctx);
    int64_t n1 = 0;
    RSB_HIP(hipMemcpyAsync(&n1, ntot.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RSB_HIP(hipStreamSynchronize(s));
    if (n1 == 0) {
      k_amg_fill<<<g, kBlock, 0, s>>>(F.agg.get(), n, -1);
      RSB_LAUNCHED();
      break;
    }
    const int64_t n1pad = round_up(n1, 64);
    AmgLevelDev C;
    C.n = n1pad;
    C.gid_own.alloc(ctx, n1pad);
    C.gid = C.gid_own.get();
    C.seg.alloc(ctx, n1pad);
    C.rowlen.alloc(ctx, n1pad);
    C.dinv.alloc(ctx, n1pad);
    C.agg.alloc(ctx, n1pad);
    C.mem.alloc(ctx, 2 * n1pad);
    C.f.alloc(ctx, n1pad);
    C.u.alloc(ctx, n1pad);
    C.u2.alloc(ctx, n1pad);
    C.r.alloc(ctx, n1pad);
    C.r2.alloc(ctx, n1pad);
    k_amg_link<<<g, kBlock, 0, s>>>(F.seg.get(), F.gid, mate.get(), cont.get(), cidx.get(), n,
                                    F.agg.get(), C.mem.get(), C.gid_own.get(), C.seg.get());
    if (n1pad > n1)
      k_amg_pad_rows<<<grid_for(n1pad - n1, kBlock), kBlock, 0, s>>>(
          n1, n1pad, C.seg.get(), C.rowlen.get(), C.dinv.get(), C.gid_own.get(), C.mem.get());
    const unsigned gw = grid_for(n1pad, kBlock / kWave);
    if (packed)
      k_amg_coarse<true, 0><<<gw, kBlock, 0, s>>>(m, F.agg.get(), C.mem.get(), n1pad,
                                                   C.rowlen.get(), nullptr, nullptr, nullptr,
                                                   nullptr, err.get());
    else
      k_amg_coarse<false, 0><<<gw, kBlock, 0, s>>>(m, F.agg.get(), C.mem.get(), n1pad,
                                                    C.rowlen.get(), nullptr, nullptr, nullptr,
                                                    nullptr, err.get());
    RSB_LAUNCHED();
    const int64_t nch = n1pad / 64;
    DevBuf<int64_t> slots(ctx, nch);
    C.chunk_ptr.alloc(ctx, nch + 1);
    k_amg_slice_slots<<<grid_for(nch, kBlock), kBlock, 0, s>>>(C.rowlen.get(), n1, nch,
                                                               slots.get());
    RSB_LAUNCHED();
    scan_exclusive(slots.get(), nch, C.chunk_ptr.get(), C.chunk_ptr.get() + nch, ctx);
    int64_t words = 0;
    int herr = 0;
    RSB_HIP(hipMemcpyAsync(&words, C.chunk_ptr.get() + nch, sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    RSB_HIP(hipMemcpyAsync(&herr, err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    RSB_HIP(hipStreamSynchronize(s));
    if (herr) fail(RSB_EINTERNAL, "AMG coarse row: candidate capacity exceeded");
    C.col.alloc(ctx, std::max<int64_t>(words, 1));
    C.wgt.alloc(ctx, std::max<int64_t>(words, 1));
    C.words = words;
    if (packed)
      k_amg_coarse<true, 1><<<gw, kBlock, 0, s>>>(m, F.agg.get(), C.mem.get(), n1pad, nullptr,
                                                   C.chunk_ptr.get(), C.col.get(), C.wgt.get(),
                                                   C.dinv.get(), err.get());
    else
      k_amg_coarse<false, 1><<<gw, kBlock, 0, s>>>(m, F.agg.get(), C.mem.get(), n1pad, nullptr,
                                                    C.chunk_ptr.get(), C.col.get(), C.wgt.get(),
                                                    C.dinv.get(), err.get());
    RSB_LAUNCHED();
    RSB_HIP(hipMemcpyAsync(&herr, err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    RSB_HIP(hipStreamSynchronize(s));
    if (herr & 2) fail(RSB_EINTERNAL, "AMG coarse weight above 2^32 - 1");
    C.mat = MatDevHost{C.chunk_ptr.get(), nullptr, C.col.get(), C.wgt.get()};
    A.lv.push_back(std::move(C));
  }
  // the coarsest level has no next level
  {
    AmgLevelDev &B = A.lv.back();
    if (B.n > 0) {
      k_amg_fill<<<grid_for(B.n, kBlock), kBlock, 0, s>>>(B.agg.get(), B.n, -1);
      RSB_LAUNCHED();
    }
  }
  RSB_HIP(hipStreamSynchronize(s));
}

namespace {

// Launches of one level (and, recursively, the levels below).  Returns the
// buffer (0 or 1) that holds the level's result u.
int vc_level(AmgDev &A, size_t l, const double *f, const SegState *st, hipStream_t s) {
  AmgLevelDev &Z = A.lv[l];
  const unsigned g = grid_for(Z.n, kBlock);
  const bool packed = (l == 0);
  MatDev m{Z.mat.chunk_ptr, Z.mat.packed, Z.mat.col, Z.mat.wgt};
  double *u[2] = {Z.u.get(), Z.u2.get()};
  double *r[2] = {Z.r.get(), Z.r2.get()};
  const double sg = A.sigma;
  if (packed)
    k_vc_pre0<true><<<g, kBlock, 0, s>>>(m, Z.seg.get(), st, Z.dinv.get(), f, sg, Z.n, u[0], r[0]);
  else
    k_vc_pre0<false><<<g, kBlock, 0, s>>>(m, Z.seg.get(), st, Z.dinv.get(), f, sg, Z.n, u[0],
                                          r[0]);
  int cur = 0;
  for (int k = 0; k < A.nsmooth; ++k, cur ^= 1) {
    if (packed)
      k_vc_pre<true><<<g, kBlock, 0, s>>>(m, Z.seg.get(), st, Z.dinv.get(), f, u[cur], r[cur],
                                          sg, Z.n, u[cur ^ 1], r[cur ^ 1]);
    else
      k_vc_pre<false><<<g, kBlock, 0, s>>>(m, Z.seg.get(), st, Z.dinv.get(), f, u[cur], r[cur],
                                           sg, Z.n, u[cur ^ 1], r[cur ^ 1]);
  }
  if (l + 1 >= A.lv.size()) return cur;
  AmgLevelDev &C = A.lv[l + 1];
  k_vc_restrict<<<grid_for(C.n, kBlock), kBlock, 0, s>>>(C.seg.get(), C.mem.get(), st, r[cur],
                                                         C.n, C.f.get());
  const int cb = vc_level(A, l + 1, C.f.get(), st, s);
  const double *e1 = cb ? C.u2.get() : C.u.get();
  if (A.nsmooth == 0) {
    k_vc_prolong<<<g, kBlock, 0, s>>>(Z.seg.get(), Z.agg.get(), st, e1, Z.n, u[cur]);
    return cur;
  }
  for (int k = 0; k < A.nsmooth; ++k, cur ^= 1) {
    const double *ui = u[cur];
    double *uo = u[cur ^ 1];
    if (packed && k == 0)
      k_vc_post<true, true><<<g, kBlock, 0, s>>>(m, Z.seg.get(), Z.agg.get(), st, Z.dinv.get(), f,
                                                 ui, e1, sg, Z.n, uo);
    else if (packed)
      k_vc_post<true, false><<<g, kBlock, 0, s>>>(m, Z.seg.get(), Z.agg.get(), st, Z.dinv.get(),
                                                  f, ui, e1, sg, Z.n, uo);
    else if (k == 0)
      k_vc_post<false, true><<<g, kBlock, 0, s>>>(m, Z.seg.get(), Z.agg.get(), st, Z.dinv.get(),
                                                  f, ui, e1, sg, Z.n, uo);
    else
      k_vc_post<false, false><<<g, kBlock, 0, s>>>(m, Z.seg.get(), Z.agg.get(), st, Z.dinv.get(),
                                                   f, ui, e1, sg, Z.n, uo);
  }
  return cur;
}

}  // namespace

const double *amg_vcycle(AmgDev &A, const double *d_f, const SegState *d_st, hipStream_t s) {
  if (A.lv.empty()) return nullptr;
  const int b = vc_level(A, 0, d_f, d_st, s);
  RSB_LAUNCHED();
  return b ? A.lv[0].u2.get() : A.lv[0].u.get();
}

const double *amg_result(const AmgDev &A) {
  // pre-smoothing leaves a level's result in buffer nsmooth % 2; on a level
  // with a level below, nsmooth post-smoothing steps (or the in-place
  // correction when nsmooth = 0) bring it back to buffer 0
  if (A.lv.empty()) return nullptr;
  const bool second = A.lv.size() == 1 && (A.nsmooth & 1);
  return second ? A.lv[0].u2.get() : A.lv[0].u.get();
}

}  // namespace rsb
