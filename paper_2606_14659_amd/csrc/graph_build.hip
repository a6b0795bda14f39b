// graph_build.hip -- element dual graph on the GPU (paper Sec. 2, Sec. 4).
//
// s_ij = number of distinct vertex ids elements i and j share; the Laplacian
// has off-diagonal -w_ij with w from s (weighted: s, unit: 1, face: s >= nv/2).
//
// Algorithm:
//  1. one (vertex id, slot = e*nv + l) pair per element vertex; an id repeated
//     inside an element keeps only its first slot (set semantics);
//  2. stable LSD radix sort of the pairs by vertex id, 8-bit digits, only as
//     many passes as the largest id needs;
//  3. runs of equal ids give, for every vertex, the elements touching it;
//  4. one wavefront per element gathers the elements of its vertices' runs
//     into LDS and counts multiplicities: that count is s_ij.  Distinct
//     neighbours are ranked to get ascending columns; a counting pass gives
//     row lengths, an exclusive scan the row pointers, a second pass the
//     columns and weights.
#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

constexpr int kIpt = 16;                 // keys per thread in a radix tile
constexpr int kTile = kBlock * kIpt;     // 4096 keys per tile
constexpr int kCandCap = 1024;           // candidate entries per element (LDS)
constexpr uint64_t kInvalid = ~uint64_t(0);

__global__ void k_id_stats(const int64_t *__restrict__ ids, int64_t count,
                           unsigned long long *__restrict__ maxid, int *__restrict__ neg) {
  unsigned long long m = 0;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = ids[i];
    if (v < 0) bad = 1;
    else m = m > (unsigned long long)v ? m : (unsigned long long)v;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(m, off, kWave);
    m = m > o ? m : o;
    bad |= __shfl_xor(bad, off, kWave);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(maxid, m);
    if (bad) atomicOr(neg, 1);
  }
}

__global__ void k_make_pairs(const int64_t *__restrict__ ids, int64_t nelem, int nv,
                             uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nelem * nv) return;
  int64_t e = s / nv;
  int l = (int)(s - e * nv);
  int64_t v = ids[s];
  bool dup = false;
  for (int k = 0; k < l; ++k) dup |= (ids[e * nv + k] == v);
  keys[s] = dup ? kInvalid : (uint64_t)v;
  vals[s] = (uint32_t)s;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                       int64_t n, int shift, int64_t nblocks,
                                                       int64_t *__restrict__ hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int r = 0; r < kIpt; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one digit pass.  Items of the tile are taken in rounds
// of 256 (item index = round*256 + thread), so the stable order is (round,
// wave, lane).  Within a wave, lanes with the same digit are found with
// eight ballots (one per digit bit).
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n, int shift,
    int64_t nblocks, const int64_t *__restrict__ offs, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout) {
  constexpr int W = kBlock / kWave;
  __shared__ int64_t running[256];
  __shared__ int wcnt[W][256];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  running[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  for (int w = 0; w < W; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kIpt; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    int d = valid ? (int)((key >> shift) & 255) : 255;
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    int rank = __popcll(peers & lt);
    int leader = __ffsll((unsigned long long)peers) - 1;
    if (lane == leader) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    int64_t pos = running[d] + rank;
    for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int tot = 0;
    for (int w = 0; w < W; ++w) {
      tot += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    running[threadIdx.x] += tot;
    __syncthreads();
  }
}

__global__ void k_run_heads(const uint64_t *__restrict__ keys, int64_t n,
                            int32_t *__restrict__ head) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// run id of each sorted position (inclusive count of heads - 1); slot -> run
// map; run start positions.
// Slots of the invalid (duplicate) key keep slot_run = -1; that run, if
// present, is the last one and only bounds the run before it.
__global__ void k_run_index(const int32_t *__restrict__ head, const int64_t *__restrict__ excl,
                            const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                            int64_t n, int32_t *__restrict__ slot_run,
                            int64_t *__restrict__ run_start) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t run = excl[i] + head[i] - 1;
  if (keys[i] != kInvalid) slot_run[vals[i]] = (int32_t)run;
  if (head[i]) run_start[run] = i;
  if (i == n - 1) run_start[run + 1] = n;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One wavefront per element.  PASS 0 writes row lengths, PASS 1 columns and
// weights at row_ptr.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_elem_neighbors(
    int64_t nelem, int nv, int graph, const int32_t *__restrict__ slot_run,
    const int64_t *__restrict__ run_start, const uint32_t *__restrict__ sorted_vals,
    int32_t *__restrict__ row_len, const int64_t *__restrict__ row_ptr,
    int32_t *__restrict__ col, int32_t *__restrict__ wgt, int *__restrict__ err) {
  constexpr int W = kBlock / kWave;
  __shared__ int32_t cand[W][kCandCap];
  __shared__ uint8_t keepw[W][kCandCap];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t e = (int64_t)blockIdx.x * W + wave;
  if (e >= nelem) return;
  int32_t *c = cand[wave];
  uint8_t *kw = keepw[wave];
  int total = 0;
  for (int l = 0; l < nv; ++l) {
    int32_t r = slot_run[e * nv + l];
    if (r < 0) continue;
    int64_t a = run_start[r], b = run_start[r + 1];
    int len = (int)(b - a);
    if (total + len > kCandCap) {
      if (lane == 0) atomicOr(err, 1);
      return;
    }
    for (int t = lane; t < len; t += kWave) c[total + t] = (int32_t)(sorted_vals[a + t] / nv);
    total += len;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // per candidate: 1st occurrence of a kept neighbour -> weight, else 0
  for (int i = lane; i < total; i += kWave) {
    int32_t v = c[i];
    int cnt = 0;
    bool first = true;
    for (int j = 0; j < total; ++j) {
      bool same = (c[j] == v);
      cnt += same;
      if (same && j < i) first = false;
    }
    int w = 0;
    if (first && v != (int32_t)e) {
      if (graph == RSB_GRAPH_WEIGHTED) w = cnt;
      else if (graph == RSB_GRAPH_UNIT) w = 1;
      else w = (cnt >= nv / 2) ? 1 : 0;
    }
    if (w > (int)kWeightMask) atomicOr(err, 2);
    kw[i] = (uint8_t)(w > 255 ? 255 : w);
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (PASS == 0) {
    int k = 0;
    for (int i = lane; i < total; i += kWave) k += (kw[i] != 0);
    k = wave_sum_i(k);
    if (lane == 0) row_len[e] = k;
  } else {
    int64_t rp = row_ptr[e];
    for (int i = lane; i < total; i += kWave) {
      if (!kw[i]) continue;
      int32_t v = c[i];
      int rank = 0;
      for (int j = 0; j < total; ++j) rank += (kw[j] != 0 && c[j] < v);
      col[rp + rank] = v;
      wgt[rp + rank] = kw[i];
    }
  }
}

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// keys, 8 bits per pass; the sorted pairs end in keys/vals.
void sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int bits, Ctx &ctx, bool sync) {
  if (n <= 1 || bits <= 0) return;
  const int passes = (bits + 7) / 8;
  DevBuf<uint64_t> kb(ctx, n);
  DevBuf<uint32_t> vb(ctx, n);
  const int64_t nblocks = (n + kTile - 1) / kTile;
  DevBuf<int64_t> hist(ctx, 256 * nblocks), offs(ctx, 256 * nblocks);
  uint64_t *kin = keys, *kout = kb.get();
  uint32_t *vin = vals, *vout = vb.get();
  for (int p = 0; p < passes; ++p) {
    k_radix_hist<<<(unsigned)nblocks, kBlock, 0, ctx.stream>>>(kin, n, 8 * p, nblocks, hist.get());
    RSB_LAUNCHED();
    scan_exclusive(hist.get(), 256 * nblocks, offs.get(), nullptr, ctx);
    k_radix_scatter<<<(unsigned)nblocks, kBlock, 0, ctx.stream>>>(kin, vin, n, 8 * p, nblocks,
                                                                  offs.get(), kout, vout);
    RSB_LAUNCHED();
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kin != keys) {
    RSB_HIP(hipMemcpyAsync(keys, kin, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx.stream));
    RSB_HIP(hipMemcpyAsync(vals, vin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx.stream));
  }
  if (sync) RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void fill_f64(double *p, int64_t n, double v, Ctx &ctx) {
  if (n <= 0) return;
  k_fill_f64<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(p, n, v);
  RSB_LAUNCHED();
}

void fill_i32(int32_t *p, int64_t n, int32_t v, Ctx &ctx) {
  if (n <= 0) return;
  k_fill_i32<<<grid_for(n, kBlock), kBlock, 0, ctx.stream>>>(p, n, v);
  RSB_LAUNCHED();
}

void build_dual_graph(const int64_t *d_ids, int64_t nelem, int nv, int graph, DevCsr &out,
                      Ctx &ctx) {
  const int64_t npairs = nelem * nv;
  // 1. id range and validity
  DevBuf<unsigned long long> d_max(ctx, 1);
  DevBuf<int> d_neg(ctx, 1);
  RSB_HIP(hipMemsetAsync(d_max.get(), 0, sizeof(unsigned long long), ctx.stream));
  RSB_HIP(hipMemsetAsync(d_neg.get(), 0, sizeof(int), ctx.stream));
  {
    unsigned g = (unsigned)std::min<int64_t>(grid_for(npairs, kBlock), 4096);
    k_id_stats<<<g, kBlock, 0, ctx.stream>>>(d_ids, npairs, d_max.get(), d_neg.get());
    RSB_LAUNCHED();
  }
  unsigned long long maxid = 0;
  int neg = 0;
  RSB_HIP(hipMemcpyAsync(&maxid, d_max.get(), sizeof(maxid), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipMemcpyAsync(&neg, d_neg.get(), sizeof(neg), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  if (neg) fail(RSB_EINVAL, "negative vertex id");
  // bits so that every valid id is below the all-ones pattern of the digits
  int bits = 64 - __builtin_clzll(maxid + 1ull);
  int passes = (bits + 7) / 8;

  // 2. pairs and radix sort
  DevBuf<uint64_t> ka(ctx, npairs), kb(ctx, npairs);
  DevBuf<uint32_t> va(ctx, npairs), vb(ctx, npairs);
  k_make_pairs<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(d_ids, nelem, nv, ka.get(),
                                                                     va.get());
  RSB_LAUNCHED();
  const int64_t nblocks = (npairs + kTile - 1) / kTile;
  DevBuf<int64_t> hist(ctx, 256 * nblocks), offs(ctx, 256 * nblocks);
  uint64_t *kin = ka.get(), *kout = kb.get();
  uint32_t *vin = va.get(), *vout = vb.get();
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    k_radix_hist<<<(unsigned)nblocks, kBlock, 0, ctx.stream>>>(kin, npairs, shift, nblocks,
                                                               hist.get());
    RSB_LAUNCHED();
    scan_exclusive(hist.get(), 256 * nblocks, offs.get(), nullptr, ctx);
    k_radix_scatter<<<(unsigned)nblocks, kBlock, 0, ctx.stream>>>(
        kin, vin, npairs, shift, nblocks, offs.get(), kout, vout);
    RSB_LAUNCHED();
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  hist.release();
  offs.release();
  // 3. runs; invalid (duplicate) slots sort last and are dropped
  DevBuf<int32_t> head(ctx, npairs);
  DevBuf<int64_t> hexcl(ctx, npairs);
  k_run_heads<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(kin, npairs, head.get());
  RSB_LAUNCHED();
  DevBuf<int64_t> d_nruns(ctx, 1);
  scan_exclusive(head.get(), npairs, hexcl.get(), d_nruns.get(), ctx);
  DevBuf<int32_t> slot_run(ctx, npairs);
  DevBuf<int64_t> run_start(ctx, npairs + 1);
  fill_i32(slot_run.get(), npairs, -1, ctx);
  k_run_index<<<grid_for(npairs, kBlock), kBlock, 0, ctx.stream>>>(
      head.get(), hexcl.get(), kin, vin, npairs, slot_run.get(), run_start.get());
  RSB_LAUNCHED();
  head.release();
  hexcl.release();
  d_nruns.release();
  // 4. neighbours: lengths, row pointers, columns
  out.n = nelem;
  out.row_ptr.alloc(ctx, nelem + 1);
  DevBuf<int32_t> rowlen(ctx, nelem);
  DevBuf<int> d_err(ctx, 1);
  RSB_HIP(hipMemsetAsync(d_err.get(), 0, sizeof(int), ctx.stream));
  const unsigned eg = grid_for(nelem, kBlock / kWave);
  k_elem_neighbors<0><<<eg, kBlock, 0, ctx.stream>>>(
      nelem, nv, graph, slot_run.get(), run_start.get(), vin, rowlen.get(), nullptr, nullptr,
      nullptr, d_err.get());
  RSB_LAUNCHED();
  DevBuf<int64_t> d_nnz(ctx, 1);
  scan_exclusive(rowlen.get(), nelem, out.row_ptr.get(), out.row_ptr.get() + nelem, ctx);
  int err = 0;
  RSB_HIP(hipMemcpyAsync(&err, d_err.get(), sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipMemcpyAsync(&out.nnz, out.row_ptr.get() + nelem, sizeof(int64_t),
                         hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  if (err & 1) fail(RSB_EINVAL, "an element has more than 1024 candidate neighbour entries");
  if (err & 2) fail(RSB_EINVAL, "edge weight above 15 (too many shared vertex ids)");
  out.col.alloc(ctx, std::max<int64_t>(out.nnz, 1));
  out.wgt.alloc(ctx, std::max<int64_t>(out.nnz, 1));
  k_elem_neighbors<1><<<eg, kBlock, 0, ctx.stream>>>(
      nelem, nv, graph, slot_run.get(), run_start.get(), vin, nullptr, out.row_ptr.get(),
      out.col.get(), out.wgt.get(), d_err.get());
  RSB_LAUNCHED();
}

}  // namespace rsb
