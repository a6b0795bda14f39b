// reorder.hip -- locality order of the level-0 rows.
//
// The solver streams every row of a level once per Lanczos step and gathers
// the vector at each row's neighbours.  With elements in an arbitrary order
// those gathers touch the whole vector.  The paper's partitioner also starts
// from an effectively random distribution and pre-sorts it by recursive
// coordinate bisection for locality (Sec. 5, Sec. 8).  Coordinates are not
// part of the input, so the rows are ordered by the graph instead, in
// Cuthill-McKee order: a first search from row 0 finds the farthest row
// (smallest index among the farthest), a second search from there gives
// every row its level; rows are grouped by level (stable radix sort), and
// level by level each row is placed by the least position of its neighbours
// in the level before (ties in input order), so that a run of rows in one
// level gathers from a run in the next; rows the search does not reach go
// last in their old order.  The order changes only where rows live: element
// ids, start vectors, tie-breaks and outputs still follow the input
// numbering.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

__global__ void k_bfs_init(int32_t *__restrict__ dist, int64_t n, int64_t src,
                           int32_t *__restrict__ frontier) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dist[i] = (i == src) ? 0 : -1;
  if (i == 0) frontier[0] = (int32_t)src;
}

// One level of the search from the frontier (rows at level L, *nf of them,
// a count the previous level's launch left on the device): unreached
// neighbours get level L + 1 (first claim wins; every claimant writes the
// same level, so the levels do not depend on timing) and join the next
// frontier, whose order may vary and is not used.  A fixed grid strides over
// the frontier, so levels can be launched back to back without the host
// reading their sizes.
__global__ void k_bfs_top(const int32_t *__restrict__ frontier, const int32_t *__restrict__ nf,
                          const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                          int32_t *__restrict__ dist, int32_t L, int32_t *__restrict__ next,
                          int32_t *__restrict__ nnext) {
  const int64_t n = *nf;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = frontier[k];
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int32_t j = col[p];
      if (dist[j] == -1 && atomicCAS(&dist[j], -1, L + 1) == -1) next[atomicAdd(nnext, 1)] = j;
    }
  }
}

__global__ void k_bfs_count_set(int32_t *__restrict__ c, int32_t v) { c[0] = v; }

// farthest reached row, smallest index among ties: max of (dist, ~row)
__global__ void k_bfs_far(const int32_t *__restrict__ dist, int64_t n,
                          unsigned long long *__restrict__ best) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long key = 0;
  if (i < n && dist[i] >= 0)
    key = ((unsigned long long)dist[i] << 32) | (0xFFFFFFFFull - (unsigned long long)i);
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(key, off, kWave);
    key = key > o ? key : o;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && key) atomicMax(best, key);
}

__global__ void k_order_keys(const int32_t *__restrict__ dist, int64_t n,
                             uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = dist[i] >= 0 ? (uint64_t)dist[i] : 0xFFFFFFFFull;
  vals[i] = (uint32_t)i;
}

__global__ void k_level_count(const int32_t *__restrict__ dist, int64_t n,
                              int32_t *__restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && dist[i] >= 0) atomicAdd(&cnt[dist[i]], 1);
}

// rows of level L + 1 (order[a..b)): key = least position of a neighbour in
// level L (positions [a0, a0 + m)), relative to a0; every such row has one,
// m would sort last
__global__ void k_cm_keys(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ dist, const int32_t *__restrict__ pos,
                          const uint32_t *__restrict__ order, int64_t a, int64_t b, int32_t L,
                          int64_t a0, int64_t m, uint64_t *__restrict__ keys) {
  const int64_t k = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= b) return;
  const int64_t i = order[k];
  int64_t best = a0 + m;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t j = col[p];
    if (dist[j] == L) best = min(best, (int64_t)pos[j]);
  }
  keys[k] = (uint64_t)(best - a0);
}

__global__ void k_cm_pos(const uint32_t *__restrict__ order, int64_t a, int64_t b,
                         int32_t *__restrict__ pos) {
  const int64_t k = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < b) pos[order[k]] = (int32_t)k;
}

__global__ void k_perm_finish(const uint32_t *__restrict__ vals, int64_t n,
                              int32_t *__restrict__ perm, int32_t *__restrict__ iperm,
                              const int64_t *__restrict__ rp, int64_t *__restrict__ newlen) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t old = (int32_t)vals[k];
  perm[k] = old;
  iperm[old] = (int32_t)k;
  newlen[k] = rp[old + 1] - rp[old];
}

__global__ void k_perm_csr(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ w, const int32_t *__restrict__ perm,
                           const int32_t *__restrict__ iperm, const int64_t *__restrict__ nrp,
                           int64_t n, int32_t *__restrict__ ncol, int32_t *__restrict__ nw) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t old = perm[k];
  const int64_t a = rp[old], len = rp[old + 1] - a, b = nrp[k];
  for (int64_t t = 0; t < len; ++t) {
    ncol[b + t] = iperm[col[a + t]];
    nw[b + t] = w[a + t];
  }
}

// Breadth-first levels from src into dist; returns the number of levels
// (the largest distance + 1).  Levels go out in batches of kBfsBatch
// launches; lc[i] holds the frontier size of the batch's level i, and the
// host reads the batch's sizes once to find where the search ended (the
// launches after that found an empty frontier and did nothing).
constexpr int kBfsBatch = 16;

int bfs(const DevCsr &g, int64_t src, int32_t *dist, int32_t *fa, int32_t *fb, Ctx &ctx) {
  const int64_t n = g.n;
  k_bfs_init<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(dist, n, src, fa);
  RSB_LAUNCHED();
  DevBuf<int32_t> lc(ctx, kBfsBatch + 1);
  const unsigned grid = std::min<unsigned>(grid_for(n, kBlock), 1024u);
  int32_t L = 0;
  int32_t start = 1;  // frontier size at the batch's first level
  for (;;) {
    RSB_HIP(hipMemsetAsync(lc.get(), 0, (kBfsBatch + 1) * sizeof(int32_t), ctx.stream));
    k_bfs_count_set<<<1, 1, 0, ctx.stream>>>(lc.get(), start);
    for (int i = 0; i < kBfsBatch; ++i) {
      k_bfs_top<<<grid, kBlock, 0, ctx.stream>>>(fa, lc.get() + i, g.row_ptr.get(), g.col.get(),
                                                 dist, L + i, fb, lc.get() + i + 1);
      std::swap(fa, fb);
    }
    RSB_LAUNCHED();
    int32_t h[kBfsBatch + 1];
    RSB_HIP(hipMemcpyAsync(h, lc.get(), sizeof(h), hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    for (int i = 1; i <= kBfsBatch; ++i)
      if (h[i] == 0) return L + i;
    L += kBfsBatch;
    start = h[kBfsBatch];
  }
}

// Row count and the exact integer sums of the reached rows' distances (per
// block, then one atomic add per block).
__global__ void k_bfs_sums(const int32_t *__restrict__ dist, int64_t n,
                           unsigned long long *__restrict__ sums) {
  __shared__ unsigned long long red[3][kBlock / kWave];
  unsigned long long c = 0, s1 = 0, s2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = dist[i];
    if (d >= 0) {
      c += 1;
      s1 += (unsigned long long)d;
      s2 += (unsigned long long)d * (unsigned long long)d;
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, kWave);
    s1 += __shfl_xor(s1, off, kWave);
    s2 += __shfl_xor(s2, off, kWave);
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][w] = c;
    red[1][w] = s1;
    red[2][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / kWave; ++k) {
      c += red[0][k];
      s1 += red[1][k];
      s2 += red[2][k];
    }
    atomicAdd(&sums[0], c);
    atomicAdd(&sums[1], s1);
    atomicAdd(&sums[2], s2);
  }
}

__global__ void k_bfs_warm(const int32_t *__restrict__ dist, int64_t n, double mean, double sd,
                           double *__restrict__ warm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && dist[i] >= 0) warm[i] = ((double)dist[i] - mean) / sd;
}

}  // namespace

void bfs_start_values(const DevCsr &g, double *warm, Ctx &ctx) {
  const int64_t n = g.n;
  if (n < 2) return;
  const unsigned gr = grid_for(n, kBlock);
  DevBuf<int32_t> dist(ctx, n), fa(ctx, n), fb(ctx, n);
  DevBuf<unsigned long long> best(ctx, 1), sums(ctx, 3);
  bfs(g, 0, dist.get(), fa.get(), fb.get(), ctx);
  RSB_HIP(hipMemsetAsync(best.get(), 0, sizeof(unsigned long long), ctx.stream));
  k_bfs_far<<<gr, kBlock, 0, ctx.stream>>>(dist.get(), n, best.get());
  RSB_LAUNCHED();
  unsigned long long hb = 0;
  RSB_HIP(hipMemcpyAsync(&hb, best.get(), sizeof(hb), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  const int64_t far = hb ? (int64_t)(0xFFFFFFFFull - (hb & 0xFFFFFFFFull)) : 0;
  bfs(g, far, dist.get(), fa.get(), fb.get(), ctx);
  RSB_HIP(hipMemsetAsync(sums.get(), 0, 3 * sizeof(unsigned long long), ctx.stream));
  k_bfs_sums<<<std::min<unsigned>(gr, 1024u), kBlock, 0, ctx.stream>>>(dist.get(), n, sums.get());
  RSB_LAUNCHED();
  unsigned long long h[3] = {0, 0, 0};
  RSB_HIP(hipMemcpyAsync(h, sums.get(), sizeof(h), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  const int64_t cnt = (int64_t)h[0];
  if (cnt < 2) return;
  // the same arithmetic on the exact sums as the reference definition
  const double mean = (double)(int64_t)h[1] / (double)cnt;
  const double var = (double)(int64_t)h[2] / (double)cnt - mean * mean;
  if (!(var > 0.0)) return;
  k_bfs_warm<<<gr, kBlock, 0, ctx.stream>>>(dist.get(), n, mean, std::sqrt(var), warm);
  RSB_LAUNCHED();
  RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void locality_order(DevCsr &g, DevBuf<int32_t> &perm, Ctx &ctx) {
  const int64_t n = g.n;
  perm.alloc(ctx, std::max<int64_t>(n, 1));
  if (n == 0) return;
  const unsigned gr = grid_for(n, kBlock);
  DevBuf<int32_t> dist(ctx, n), fa(ctx, n), fb(ctx, n);
  DevBuf<unsigned long long> best(ctx, 1);
  bfs(g, 0, dist.get(), fa.get(), fb.get(), ctx);
  RSB_HIP(hipMemsetAsync(best.get(), 0, sizeof(unsigned long long), ctx.stream));
  k_bfs_far<<<gr, kBlock, 0, ctx.stream>>>(dist.get(), n, best.get());
  RSB_LAUNCHED();
  unsigned long long hb = 0;
  RSB_HIP(hipMemcpyAsync(&hb, best.get(), sizeof(hb), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  const int64_t far = hb ? (int64_t)(0xFFFFFFFFull - (hb & 0xFFFFFFFFull)) : 0;
  const int nlev = bfs(g, far, dist.get(), fa.get(), fb.get(), ctx);
  DevBuf<uint64_t> keys(ctx, n);
  DevBuf<uint32_t> vals(ctx, n);
  k_order_keys<<<gr, kBlock, 0, ctx.stream>>>(dist.get(), n, keys.get(), vals.get());
  RSB_LAUNCHED();
  sort_pairs(keys.get(), vals.get(), n, 32, ctx);
  // level sizes, then Cuthill-McKee placement level by level
  {
    DevBuf<int32_t> cnt(ctx, std::max(nlev, 1));
    fill_i32(cnt.get(), std::max(nlev, 1), 0, ctx);
    k_level_count<<<gr, kBlock, 0, ctx.stream>>>(dist.get(), n, cnt.get());
    RSB_LAUNCHED();
    std::vector<int32_t> hc(std::max(nlev, 1));
    RSB_HIP(hipMemcpyAsync(hc.data(), cnt.get(), hc.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    DevBuf<int32_t> pos(ctx, n);
    int64_t a = 0, a0 = 0;
    for (int L = 0; L < nlev; ++L) {
      const int64_t b = a + hc[L];
      if (L > 0 && b - a > 1) {
        const int64_t m = hc[L - 1];
        int bits = 1;
        while ((1ll << bits) <= m) ++bits;
        k_cm_keys<<<grid_for(b - a, kBlock), kBlock, 0, ctx.stream>>>(
            g.row_ptr.get(), g.col.get(), dist.get(), pos.get(), vals.get(), a, b, L - 1, a0, m,
            keys.get());
        RSB_LAUNCHED();
        sort_pairs(keys.get() + a, vals.get() + a, b - a, bits, ctx, false);
      }
      k_cm_pos<<<grid_for(b - a, kBlock), kBlock, 0, ctx.stream>>>(vals.get(), a, b, pos.get());
      RSB_LAUNCHED();
      a0 = a;
      a = b;
    }
  }
  DevBuf<int32_t> iperm(ctx, n);
  DevBuf<int64_t> newlen(ctx, n);
  k_perm_finish<<<gr, kBlock, 0, ctx.stream>>>(vals.get(), n, perm.get(), iperm.get(),
                                               g.row_ptr.get(), newlen.get());
  RSB_LAUNCHED();
  DevCsr out;
  out.n = n;
  out.nnz = g.nnz;
  out.row_ptr.alloc(ctx, n + 1);
  out.col.alloc(ctx, std::max<int64_t>(g.nnz, 1));
  out.wgt.alloc(ctx, std::max<int64_t>(g.nnz, 1));
  scan_exclusive(newlen.get(), n, out.row_ptr.get(), out.row_ptr.get() + n, ctx);
  k_perm_csr<<<gr, kBlock, 0, ctx.stream>>>(g.row_ptr.get(), g.col.get(), g.wgt.get(), perm.get(),
                                            iperm.get(), out.row_ptr.get(), n, out.col.get(),
                                            out.wgt.get());
  RSB_LAUNCHED();
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  g.row_ptr = std::move(out.row_ptr);
  g.col = std::move(out.col);
  g.wgt = std::move(out.wgt);
}

}  // namespace rsb
