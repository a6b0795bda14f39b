// gather_scatter.hip -- the Laplacian in gather-scatter form (Sec. 5).
//
// The paper never assembles the Laplacian: an element's value is copied to
// its vertices (P), the copies of each vertex are summed (Q Q^T) and copied
// back (P^T), A_w = P^T Q Q^T P, and L = diag(A_w 1) - A_w.  For element e of
// a subgraph, with U_v the sum of x over the subgraph's elements containing
// vertex v and size_v their number,
//     (L x)_e = sum over the distinct vertices v of e of (size_v x_e - U_v)
//             = sum over the other elements j of s_ej (x_e - x_j),
// s_ej the number of vertices e and j share: the weighted dual graph's
// Laplacian (Sec. 2, Sec. 4), restricted to the subgraph.  A vertex shared
// by elements of different subgraphs is a separate "group" in each.
//
// Built once per call: the vertex -> (element, slot) incidence, by a radix
// sort of the (vertex id, pair index) pairs.  Built per level from it: the
// groups (each vertex's rows sorted, split where the subgraph changes), the
// group of every (row, slot) in a 64-row chunked layout, and each row's
// degree.  Each multiply is one launch forming U over the groups followed by
// the row pass inside the solver's own kernel.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

__device__ inline int gs_seg_of(const SegDev *seg, int nseg, int64_t row) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid].row0 <= row) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_gs_pairs(const int64_t *__restrict__ ids, int64_t n, uint32_t p0,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                           int *__restrict__ neg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (ids[i] < 0) atomicOr(neg, 1);
  keys[i] = (uint64_t)ids[i];
  vals[i] = p0 + (uint32_t)i;
}

__global__ void k_gs_maxkey(const uint64_t *__restrict__ keys, int64_t n,
                            unsigned long long *__restrict__ mx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = i < n ? keys[i] : 0ull;
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, kWave);
    v = v > o ? v : o;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicMax(mx, v);
}

// first pair of every vertex; a pair repeating its element's vertex (the
// stable sort keeps an element's pairs adjacent) loses its entry
__global__ void k_gs_mark(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                          int64_t n, int nv, int32_t *__restrict__ first,
                          uint32_t *__restrict__ vent) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const bool f = (k == 0) || keys[k] != keys[k - 1];
  first[k] = f ? 1 : 0;
  const bool dup = !f && (vals[k] / (uint32_t)nv == vals[k - 1] / (uint32_t)nv);
  vent[k] = dup ? kGsNone : vals[k];
}

__global__ void k_gs_vptr(const int32_t *__restrict__ first, const int64_t *__restrict__ idx,
                          int64_t n, int64_t nvert, int64_t *__restrict__ vptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (first[k]) vptr[idx[k]] = k;
  if (k == 0) vptr[nvert] = n;
}

__global__ void k_gs_maxdeg(const int64_t *__restrict__ vptr, int64_t nvert, int *__restrict__ mx) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int d = v < nvert ? (int)min<int64_t>(vptr[v + 1] - vptr[v], 1 << 30) : 0;
  for (int off = kWave / 2; off > 0; off >>= 1) d = max(d, __shfl_xor(d, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0 && d) atomicMax(mx, d);
}

// vertex order key: the least rank (first-level row) of its elements
__global__ void k_gs_vkey(const int64_t *__restrict__ vptr, const uint32_t *__restrict__ vent,
                          int64_t nvert, int nv, const int32_t *__restrict__ rank,
                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvert) return;
  uint32_t best = 0xFFFFFFFFu;
  for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
    const uint32_t p = vent[k];
    if (p == kGsNone) continue;
    const uint32_t e = p / (uint32_t)nv;
    const uint32_t r = rank ? (uint32_t)rank[e] : e;
    best = min(best, r);
  }
  keys[v] = best;
  vals[v] = (uint32_t)v;
}

__global__ void k_gs_vlen(const uint32_t *__restrict__ order, const int64_t *__restrict__ vptr,
                          int64_t nvert, int64_t *__restrict__ len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nvert) len[i] = vptr[order[i] + 1] - vptr[order[i]];
}

__global__ void k_gs_vmove(const uint32_t *__restrict__ order, const int64_t *__restrict__ vptr,
                           const uint32_t *__restrict__ vent, const int64_t *__restrict__ nptr,
                           int64_t nvert, uint32_t *__restrict__ nvent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvert) return;
  const int64_t a = vptr[order[i]], n = vptr[order[i] + 1] - a, b = nptr[i];
  for (int64_t t = 0; t < n; ++t) nvent[b + t] = vent[a + t];
}

__global__ void k_gs_rowof(const int32_t *__restrict__ orig, int64_t nrows,
                           int32_t *__restrict__ row_of) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrows && orig[r] >= 0) row_of[orig[r]] = (int32_t)r;
}

__global__ void k_gs_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The live rows of vertex v at this level, ascending, with their slots.
__device__ inline int gs_collect(const int64_t *__restrict__ vptr, const uint32_t *__restrict__ vent,
                                 int64_t v, int nv, const int32_t *__restrict__ row_of,
                                 int32_t *rows, int32_t *slots) {
  int n = 0;
  for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
    const uint32_t p = vent[k];
    if (p == kGsNone) continue;
    const int32_t r = row_of[p / (uint32_t)nv];
    if (r < 0) continue;
    // insertion in ascending row order (a vertex has at most kGsMaxDeg entries)
    int i = n++;
    while (i > 0 && rows[i - 1] > r) {
      rows[i] = rows[i - 1];
      slots[i] = slots[i - 1];
      --i;
    }
    rows[i] = r;
    slots[i] = (int32_t)(p % (uint32_t)nv);
  }
  return n;
}

__global__ void k_gs_count(const int64_t *__restrict__ vptr, const uint32_t *__restrict__ vent,
                           int64_t nvert, int nv, const int32_t *__restrict__ row_of,
                           const SegDev *__restrict__ seg, int nseg, int32_t *__restrict__ cnt_g,
                           int32_t *__restrict__ cnt_e) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvert) return;
  int32_t rows[kGsMaxDeg], slots[kGsMaxDeg];
  const int n = gs_collect(vptr, vent, v, nv, row_of, rows, slots);
  int ng = 0, prev = -1;
  for (int i = 0; i < n; ++i) {
    const int s = gs_seg_of(seg, nseg, rows[i]);
    if (s != prev) {
      ++ng;
      prev = s;
    }
  }
  cnt_g[v] = ng;
  cnt_e[v] = n;
}

__global__ void k_gs_fill(const int64_t *__restrict__ vptr, const uint32_t *__restrict__ vent,
                          int64_t nvert, int nv, const int32_t *__restrict__ row_of,
                          const SegDev *__restrict__ seg, int nseg,
                          const int64_t *__restrict__ goff, const int64_t *__restrict__ eoff,
                          uint32_t *__restrict__ gptr, int32_t *__restrict__ gent,
                          int32_t *__restrict__ gseg, uint32_t *__restrict__ ev) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvert) return;
  int32_t rows[kGsMaxDeg], slots[kGsMaxDeg];
  const int n = gs_collect(vptr, vent, v, nv, row_of, rows, slots);
  const int64_t e0 = eoff[v];
  int64_t g = goff[v] - 1;
  int prev = -1;
  for (int i = 0; i < n; ++i) {
    const int s = gs_seg_of(seg, nseg, rows[i]);
    if (s != prev) {
      ++g;
      gptr[g] = (uint32_t)(e0 + i);
      gseg[g] = s;
      prev = s;
    }
    gent[e0 + i] = rows[i];
    const int64_t r = rows[i];
    ev[(r >> 6) * 64 * (int64_t)nv + (int64_t)slots[i] * 64 + (r & 63)] = (uint32_t)g;
  }
}

__global__ void k_gs_end(uint32_t *__restrict__ gptr, int64_t ngroups, int64_t nent) {
  gptr[ngroups] = (uint32_t)nent;
}

__global__ void k_gs_deg(const uint32_t *__restrict__ ev, const uint32_t *__restrict__ gptr,
                         int64_t nrows, int nv, int32_t *__restrict__ deg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const uint32_t *ep = ev + (r >> 6) * 64 * (int64_t)nv + (r & 63);
  int64_t d = 0;
  for (int k = 0; k < nv; ++k) {
    const uint32_t g = ep[(int64_t)k * 64];
    if (g != kGsNone) d += (int64_t)gptr[g + 1] - gptr[g];
  }
  deg[r] = (int32_t)d;
}

__global__ void k_gs_sums(GsView g, const double *__restrict__ x) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi < g.ngroups) gs_group_sum(g, gi, g.gptr[gi], g.gptr[gi + 1], x);
}

__global__ void k_gs_rows(GsView g, int64_t nrows, const double *__restrict__ x,
                          double *__restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrows) y[r] = gs_row<double>(g, r, x[r]);
}

}  // namespace

void gs_base_build(const std::vector<const int64_t *> &ids, const std::vector<int64_t> &nelem,
                   int nv, const int32_t *rank, GsBase &B, Ctx &ctx) {
  int64_t npairs = 0;
  for (int64_t e : nelem) npairs += e * nv;
  if (nv < 1 || npairs >= (int64_t)kGsNone)
    fail(RSB_EINVAL, "gather-scatter operator: too many (element, vertex) pairs (limit 2^32 - 1)");
  B.nv = nv;
  B.npairs = npairs;
  DevBuf<uint64_t> keys(ctx, std::max<int64_t>(npairs, 1));
  DevBuf<uint32_t> vals(ctx, std::max<int64_t>(npairs, 1));
  DevBuf<int> neg(ctx, 1);
  RSB_HIP(hipMemsetAsync(neg.get(), 0, sizeof(int), ctx.stream));
  int64_t off = 0;
  for (size_t b = 0; b < ids.size(); ++b) {
    const int64_t n = nelem[b] * nv;
    if (n > 0) {
      k_gs_pairs<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(
          ids[b], n, (uint32_t)off, keys.get() + off, vals.get() + off, neg.get());
      RSB_LAUNCHED();
    }
    off += n;
  }
  DevBuf<unsigned long long> mx(ctx, 1);
  RSB_HIP(hipMemsetAsync(mx.get(), 0, sizeof(unsigned long long), ctx.stream));
  if (npairs > 0) {
    k_gs_maxkey<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(keys.get(), npairs, mx.get());
    RSB_LAUNCHED();
  }
  unsigned long long hmx = 0;
  int hneg = 0;
  RSB_HIP(hipMemcpyAsync(&hmx, mx.get(), sizeof(hmx), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipMemcpyAsync(&hneg, neg.get(), sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  if (hneg) fail(RSB_EINVAL, "negative vertex id");
  const int bits = hmx ? 64 - __builtin_clzll(hmx) : 1;
  sort_pairs(keys.get(), vals.get(), npairs, bits, ctx);
  DevBuf<int32_t> first(ctx, std::max<int64_t>(npairs, 1));
  DevBuf<int64_t> idx(ctx, npairs + 1);
  B.vent.alloc(ctx, std::max<int64_t>(npairs, 1));
  if (npairs > 0) {
    k_gs_mark<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(keys.get(), vals.get(), npairs,
                                                                  nv, first.get(), B.vent.get());
    RSB_LAUNCHED();
  }
  scan_exclusive(first.get(), npairs, idx.get(), idx.get() + npairs, ctx);
  RSB_HIP(hipMemcpyAsync(&B.nvert, idx.get() + npairs, sizeof(int64_t), hipMemcpyDeviceToHost,
                         ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  B.vptr.alloc(ctx, B.nvert + 1);
  if (npairs > 0) {
    k_gs_vptr<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(first.get(), idx.get(), npairs,
                                                                  B.nvert, B.vptr.get());
    RSB_LAUNCHED();
  } else {
    RSB_HIP(hipMemsetAsync(B.vptr.get(), 0, sizeof(int64_t), ctx.stream));
  }
  DevBuf<int> md(ctx, 1);
  RSB_HIP(hipMemsetAsync(md.get(), 0, sizeof(int), ctx.stream));
  if (B.nvert > 0) {
    k_gs_maxdeg<<<grid_for(B.nvert, kBlock), kBlock, 0, ctx.stream>>>(B.vptr.get(), B.nvert,
                                                                      md.get());
    RSB_LAUNCHED();
  }
  int hmd = 0;
  RSB_HIP(hipMemcpyAsync(&hmd, md.get(), sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  if (hmd > kGsMaxDeg)
    fail(RSB_EINVAL, "gather-scatter operator: a vertex id appears in more than 64 slots (" +
                         std::to_string(hmd) + ")");
  // Vertices in order of their first element's row (stable, ties by id), so
  // that groups numbered in vertex order lie close to the rows that use them
  // and the group sums and the row pass both touch memory in row order.
  const int64_t nvert = B.nvert;
  {
    DevBuf<uint64_t> vk(ctx, nvert);
    DevBuf<uint32_t> order(ctx, nvert);
    const unsigned gv = grid_for(nvert, kBlock);
    k_gs_vkey<<<gv, kBlock, 0, ctx.stream>>>(B.vptr.get(), B.vent.get(), nvert, nv, rank, vk.get(),
                                            order.get());
    RSB_LAUNCHED();
    sort_pairs(vk.get(), order.get(), nvert, 32, ctx);
    DevBuf<int64_t> len(ctx, nvert), nptr(ctx, nvert + 1);
    k_gs_vlen<<<gv, kBlock, 0, ctx.stream>>>(order.get(), B.vptr.get(), nvert, len.get());
    RSB_LAUNCHED();
    scan_exclusive(len.get(), nvert, nptr.get(), nptr.get() + nvert, ctx);
    DevBuf<uint32_t> nvent(ctx, std::max<int64_t>(npairs, 1));
    k_gs_vmove<<<gv, kBlock, 0, ctx.stream>>>(order.get(), B.vptr.get(), B.vent.get(), nptr.get(),
                                             nvert, nvent.get());
    RSB_LAUNCHED();
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    B.vptr = std::move(nptr);
    B.vent = std::move(nvent);
  }
}

void gs_rank_of_rows(const int32_t *orig, int64_t nrows, int32_t *rank, Ctx &ctx) {
  if (nrows <= 0) return;
  k_gs_rowof<<<grid_for(nrows, kBlock), kBlock, 0, ctx.stream>>>(orig, nrows, rank);
  RSB_LAUNCHED();
}

void gs_level_build(const GsBase &B, const Level &L, int64_t nelem_total, GsLevel &G, Ctx &ctx) {
  const int64_t n = L.nrows, nv = B.nv;
  G.nv = B.nv;
  G.ev.alloc(ctx, std::max<int64_t>(n * nv, 1));
  G.deg.alloc(ctx, std::max<int64_t>(n, 1));
  if (n > 0) {
    k_gs_fill_u32<<<grid_for(n * nv, kBlock), kBlock, 0, ctx.stream>>>(G.ev.get(), n * nv, kGsNone);
    RSB_LAUNCHED();
  }
  DevBuf<int32_t> row_of(ctx, std::max<int64_t>(nelem_total, 1));
  fill_i32(row_of.get(), nelem_total, -1, ctx);
  if (n > 0) {
    k_gs_rowof<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(L.orig.get(), n, row_of.get());
    RSB_LAUNCHED();
  }
  const int64_t nvert = B.nvert;
  DevBuf<int32_t> cg(ctx, std::max<int64_t>(nvert, 1)), ce(ctx, std::max<int64_t>(nvert, 1));
  DevBuf<int64_t> goff(ctx, nvert + 1), eoff(ctx, nvert + 1);
  const unsigned gv = grid_for(nvert, kBlock);
  if (nvert > 0 && L.nseg > 0) {
    k_gs_count<<<gv, kBlock, 0, ctx.stream>>>(B.vptr.get(), B.vent.get(), nvert, B.nv,
                                              row_of.get(), L.d_seg.get(), L.nseg, cg.get(),
                                              ce.get());
    RSB_LAUNCHED();
  } else if (nvert > 0) {
    fill_i32(cg.get(), nvert, 0, ctx);
    fill_i32(ce.get(), nvert, 0, ctx);
  }
  scan_exclusive(cg.get(), nvert, goff.get(), goff.get() + nvert, ctx);
  scan_exclusive(ce.get(), nvert, eoff.get(), eoff.get() + nvert, ctx);
  int64_t tot[2] = {0, 0};
  RSB_HIP(hipMemcpyAsync(&tot[0], goff.get() + nvert, sizeof(int64_t), hipMemcpyDeviceToHost,
                         ctx.stream));
  RSB_HIP(hipMemcpyAsync(&tot[1], eoff.get() + nvert, sizeof(int64_t), hipMemcpyDeviceToHost,
                         ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  G.ngroups = tot[0];
  G.nent = tot[1];
  G.gptr.alloc(ctx, G.ngroups + 1);
  G.gent.alloc(ctx, std::max<int64_t>(G.nent, 1));
  G.gseg.alloc(ctx, std::max<int64_t>(G.ngroups, 1));
  G.U.alloc(ctx, std::max<int64_t>(G.ngroups, 1));
  if (nvert > 0 && L.nseg > 0) {
    k_gs_fill<<<gv, kBlock, 0, ctx.stream>>>(B.vptr.get(), B.vent.get(), nvert, B.nv, row_of.get(),
                                             L.d_seg.get(), L.nseg, goff.get(), eoff.get(),
                                             G.gptr.get(), G.gent.get(), G.gseg.get(), G.ev.get());
    RSB_LAUNCHED();
  }
  k_gs_end<<<1, 1, 0, ctx.stream>>>(G.gptr.get(), G.ngroups, G.nent);
  RSB_LAUNCHED();
  if (n > 0) {
    k_gs_deg<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(G.ev.get(), G.gptr.get(), n, B.nv,
                                                             G.deg.get());
    RSB_LAUNCHED();
  }
  RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void gs_apply(const GsView &g, int64_t nrows, const double *x, double *y, Ctx &ctx) {
  if (g.ngroups > 0) {
    k_gs_sums<<<grid_for(g.ngroups, kBlock), kBlock, 0, ctx.stream>>>(g, x);
    RSB_LAUNCHED();
  }
  if (nrows > 0) {
    k_gs_rows<<<grid_for(nrows, kBlock), kBlock, 0, ctx.stream>>>(g, nrows, x, y);
    RSB_LAUNCHED();
  }
}

}  // namespace rsb
