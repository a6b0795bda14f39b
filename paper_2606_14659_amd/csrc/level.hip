// level.hip -- bisection-level bookkeeping on the GPU: the sliced-ELL
// Laplacian of level 0, connected components and cut targets (disconnected
// rule), the split (sign rule + radix select, Sec. 4 / Alg. 1), compaction
// into the next level's induced subgraphs, and partition metrics.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)std::max<int64_t>(1, (n + per_block - 1) / per_block);
}

__device__ inline int seg_of_row(const SegDev *seg, int nseg, int64_t row) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg[mid].row0 <= row) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Level 0 from CSR
// ---------------------------------------------------------------------------
__global__ void k_chunk_words_csr(const int64_t *__restrict__ row_ptr, int64_t n, int64_t row_base,
                                  int64_t chunk_base, int64_t nchunks_mesh,
                                  int64_t *__restrict__ words) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // row within the mesh segment
  int64_t c = r / kWave;
  if (c >= nchunks_mesh) return;
  int len = (r < n) ? (int)(row_ptr[r + 1] - row_ptr[r]) : 0;
  for (int off = kWave / 2; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) words[chunk_base + c] = (int64_t)len * kWave;
}

__global__ void k_fill_sell_csr(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                const int32_t *__restrict__ wgt, int64_t n, int64_t row_base,
                                int64_t chunk_base, int64_t nchunks_mesh,
                                const int64_t *__restrict__ chunk_ptr, uint32_t *__restrict__ cols,
                                int32_t *__restrict__ orig, int32_t *__restrict__ gid,
                                int64_t orig_base, const int32_t *__restrict__ perm) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = r / kWave;
  if (c >= nchunks_mesh) return;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[chunk_base + c];
  int width = (int)((chunk_ptr[chunk_base + c + 1] - p) / kWave);
  int len = 0;
  int64_t a = 0;
  if (r < n) {
    a = row_ptr[r];
    len = (int)(row_ptr[r + 1] - a);
  }
  for (int k = 0; k < width; ++k) {
    uint32_t word = 0;
    if (k < len) word = pack_colw((uint32_t)(row_base + col[a + k]), (uint32_t)wgt[a + k]);
    cols[p + (int64_t)k * kWave + lane] = word;
  }
  const int64_t e = (r < n) ? (perm ? perm[r] : r) : -1;  // element of this row
  orig[row_base + r] = (r < n) ? (int32_t)(orig_base + e) : -1;
  gid[row_base + r] = (r < n) ? (int32_t)e : -1;
}

// ---------------------------------------------------------------------------
// Connected components (lock-free union-find, links point to lower rows)
// ---------------------------------------------------------------------------
__device__ inline int cc_load(int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cc_store(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving; parent[x] <= x always holds.
__device__ inline int cc_rep(int32_t *parent, int x) {
  int curr = cc_load(&parent[x]);
  if (curr != x) {
    int prev = x, next;
    while (curr > (next = cc_load(&parent[curr]))) {
      cc_store(&parent[prev], next);
      prev = curr;
      curr = next;
    }
  }
  return curr;
}

// Root of x by a read-only walk (no writes), for use once hooking is done:
// every parent pointer leads to the same root, whatever other threads store.
__device__ inline int cc_root(int32_t *parent, int x) {
  int curr = x, next;
  while ((next = cc_load(&parent[curr])) != curr) curr = next;
  return curr;
}

__global__ void k_cc_init(int32_t *__restrict__ parent, int32_t *__restrict__ size, int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  parent[i] = (int32_t)i;
  size[i] = 0;
}

// Each live row starts linked to its least neighbour when that is below it
// (a forest, since links only go down), so that most of the hooking below
// finds both ends already joined.
__global__ void k_cc_init_link(const int64_t *__restrict__ chunk_ptr,
                               const uint32_t *__restrict__ cols, const int32_t *__restrict__ orig,
                               int32_t *__restrict__ parent, int64_t nrows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows || orig[r] < 0) return;
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  int best = (int)r;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) != 0) best = min(best, (int)colw_col(w));
  }
  parent[r] = best;
}

// Every row first points at the root of its tree (read-only walk, each row
// storing only its own pointer).
__global__ void k_cc_flatten(int32_t *parent, const int32_t *__restrict__ orig, int64_t nrows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows || orig[i] < 0) return;
  const int r = cc_root(parent, (int)i);
  cc_store(&parent[i], r);
}

// Hooking over the edges still needed (the sampling idea of Sutton et al.,
// "Optimizing parallel graph connectivity computation via subgraph
// sampling", 2018).  After the initial links every segment's first row is a
// root (it has no lower neighbour in its segment) and most rows hang under
// it.  A row whose pointer is that root skips all its edges: it is in that
// component, and any edge to a row outside it is hooked by the other end,
// which walks all its edges.  The component only grows during the launch,
// so a row that sees the root is in it whenever it looks.
// Join the trees of rows v and j: the larger root is linked under the
// smaller by compare-and-swap, retried from whatever root it met.
__device__ inline void cc_hook_pair(int32_t *parent, int v, int j) {
  int a = cc_rep(parent, v), b = cc_rep(parent, j);
  while (a != b) {
    if (a < b) {
      int ret = atomicCAS(&parent[b], b, a);
      if (ret == b) break;
      b = ret;
    } else {
      int ret = atomicCAS(&parent[a], a, b);
      if (ret == a) break;
      a = ret;
    }
  }
}

// SAMPLE: one more sampled edge per row, its greatest neighbour, which
// joins most trees whose root has no lower neighbour (rows just past a
// hole) to the rest.
template <bool SAMPLE>
__global__ void k_cc_hook(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                          const int32_t *__restrict__ orig, const SegDev *__restrict__ seg,
                          int nseg, int32_t *parent, int64_t nrows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  if (orig[r] < 0) return;
  if (!SAMPLE) {
    const int64_t first = seg[seg_of_row(seg, nseg, r)].row0;
    if (cc_load(&parent[r]) == (int32_t)first) return;
  }
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  int v = (int)r;
  int top = -1;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) == 0) continue;
    int j = (int)colw_col(w);
    if (SAMPLE) top = max(top, j);
    else cc_hook_pair(parent, v, j);
  }
  if (SAMPLE && top > v) cc_hook_pair(parent, v, top);
}

__global__ void k_cc_compress(int32_t *parent, int32_t *__restrict__ size,
                              const int32_t *__restrict__ orig, int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  // A walk that halved paths here could store an intermediate node over the
  // root that another row just stored for itself; the read-only walk leaves
  // every pointer an ancestor, and each row then stores only its own root.
  int r = cc_root(parent, (int)i);
  cc_store(&parent[i], r);
  // component sizes: lanes sharing the root of lane 0 add together
  const bool real = orig[i] >= 0;
  const int r0 = __shfl(r, 0, kWave);
  const unsigned long long same = __ballot(real && r == r0);
  if ((threadIdx.x & (kWave - 1)) == 0 && same) atomicAdd(&size[r0], (int)__popcll(same));
  if (real && r != r0) atomicAdd(&size[r], 1);
}

// Least global id of every component, at its root.  Most lanes of a wave
// share one component: those reduce over the wave and make one atomic; the
// others make theirs only when they lower the stored value.
__global__ void k_cc_mingid(const int32_t *__restrict__ root, const int32_t *__restrict__ gid,
                            const int32_t *__restrict__ orig, int64_t nrows,
                            int32_t *__restrict__ mingid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool real = i < nrows && orig[i] >= 0;
  const int r = real ? root[i] : -1;
  const int g = real ? gid[i] : 0x7fffffff;
  const int r0 = __shfl(r, 0, kWave);
  int m = (r == r0) ? g : 0x7fffffff;
  for (int off = kWave / 2; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0 && r0 >= 0 && m < mingid[r0]) atomicMin(&mingid[r0], m);
  if (real && r != r0 && g < mingid[r]) atomicMin(&mingid[r], g);
}

__global__ void k_cc_root_flag(const int32_t *__restrict__ root, const int32_t *__restrict__ orig,
                               int64_t nrows, int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  flag[i] = (orig[i] >= 0 && root[i] == (int32_t)i) ? 1 : 0;
}

// roots as (segment, least gid) keys and their rows
__global__ void k_cc_root_keys(const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                               const int32_t *__restrict__ mingid, const SegDev *__restrict__ seg,
                               int nseg, int64_t nrows, uint64_t *__restrict__ keys,
                               uint32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows || !flag[i]) return;
  const int s = seg_of_row(seg, nseg, i);
  keys[pos[i]] = ((uint64_t)s << 32) | (uint32_t)mingid[i];
  vals[pos[i]] = (uint32_t)i;
}

__global__ void k_cc_root_sizes(const uint32_t *__restrict__ vals,
                                const int32_t *__restrict__ size, int64_t nroots,
                                int64_t *__restrict__ sz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nroots) sz[k] = size[vals[k]];
}

// base[segment] = prefix at the segment's first root in sorted order
__global__ void k_cc_seg_base(const uint64_t *__restrict__ keys, const int64_t *__restrict__ off,
                              int64_t nroots, int64_t *__restrict__ base) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nroots) return;
  if (k == 0 || (keys[k - 1] >> 32) != (keys[k] >> 32)) base[keys[k] >> 32] = off[k];
}

// pre[root] = offset of the component among its segment's components taken
// in order of least global id (roots sorted by (segment, least gid))
__global__ void k_cc_root_pre(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                              const int64_t *__restrict__ off, const int64_t *__restrict__ base,
                              int64_t nroots, int64_t *__restrict__ pre) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nroots) return;
  pre[vals[k]] = off[k] - base[keys[k] >> 32];
}

__global__ void k_seg_state_init(SegState *__restrict__ st, const SegDev *__restrict__ seg,
                                 int nseg) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  SegState z = {};
  z.strad = -1;
  z.first = 0x7fffffff;
  st[s] = z;
}

// pre[root] is the segment-relative offset of the component (the elements of
// the segment's components with a smaller least global id); pick the
// component that straddles the low-side count of each segment.
__global__ void k_cc_targets(const int32_t *__restrict__ parent, const int32_t *__restrict__ size,
                             int64_t *__restrict__ pre, const int32_t *__restrict__ orig,
                             const SegDev *__restrict__ seg, int nseg, SegState *__restrict__ st,
                             int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  if (orig[i] < 0 || parent[i] != (int32_t)i) return;
  int s = seg_of_row(seg, nseg, i);
  int64_t rel = pre[i];
  int64_t sz = size[i];
  int64_t nlow = seg[s].nlow;
  atomicAdd(&st[s].ncomp, 1);
  if (rel < nlow && nlow < rel + sz) {
    st[s].strad = (int32_t)i;
    st[s].nlow2 = (int32_t)(nlow - rel);
    st[s].solve = 1;
    st[s].invsqrt_nc = 1.0 / sqrt((double)sz);
  }
}

// ---------------------------------------------------------------------------
// Split: sign rule and radix select
// ---------------------------------------------------------------------------
__device__ inline uint64_t ordered_bits(double v) {
  uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline bool in_solve(const int32_t *root, const SegState &s, int64_t row) {
  return s.strad >= 0 && root[row] == s.strad;
}

// Rows are handled one per thread; a wavefront covers 64 rows of a single
// segment (segments are 64-row aligned), so values are reduced over the
// wavefront first and one lane does the atomic.
__global__ void k_sign_max(const double *__restrict__ y, const int32_t *__restrict__ root,
                           const SegDev *__restrict__ seg, int nseg,
                           const SegState *__restrict__ st, unsigned long long *__restrict__ ymax,
                           int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;  // whole wavefronts (nrows is a multiple of 64)
  int s = seg_of_row(seg, nseg, i);
  unsigned long long v =
      in_solve(root, st[s], i) ? (unsigned long long)__double_as_longlong(fabs(y[i])) : 0ull;
  for (int off = kWave / 2; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, kWave);
    v = v > o ? v : o;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicMax(&ymax[s], v);
}

// The deciding element is the one of least global id among the large
// entries (rows need not be in global-id order): min of (gid, row).
__global__ void k_sign_first(const double *__restrict__ y, const int32_t *__restrict__ root,
                             const int32_t *__restrict__ gid, const SegDev *__restrict__ seg,
                             int nseg, const SegState *__restrict__ st,
                             const unsigned long long *__restrict__ ymax, int64_t nrows,
                             unsigned long long *__restrict__ firstkey) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;  // whole wavefronts
  int s = seg_of_row(seg, nseg, i);
  unsigned long long cand = ~0ull;
  if (in_solve(root, st[s], i)) {
    double m = __longlong_as_double((long long)ymax[s]);
    if (fabs(y[i]) >= 1e-3 * m)
      cand = ((unsigned long long)(uint32_t)gid[i] << 32) | (unsigned long long)(uint32_t)i;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(cand, off, kWave);
    cand = cand < o ? cand : o;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && cand != ~0ull) atomicMin(&firstkey[s], cand);
}

// y <- -y on the rows being cut of every segment whose sign pass flipped.
__global__ void k_sign_apply(double *__restrict__ y, const int32_t *__restrict__ root,
                             const SegDev *__restrict__ seg, int nseg,
                             const SegState *__restrict__ st, int64_t nrows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int s = seg_of_row(seg, nseg, i);
  if (in_solve(root, st[s], i) && st[s].flip) y[i] = -y[i];
}

__global__ void k_sign_flip(const double *__restrict__ y, SegState *__restrict__ st, int nseg,
                            uint64_t *__restrict__ pk, uint32_t *__restrict__ pg,
                            int64_t *__restrict__ rank,
                            const unsigned long long *__restrict__ firstkey) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const unsigned long long fk = firstkey[s];
  st[s].first = (fk == ~0ull) ? 0x7fffffff : (int32_t)(fk & 0xffffffffull);
  int f = 0;
  if (st[s].strad >= 0 && st[s].first != 0x7fffffff) f = (y[st[s].first] > 0.0) ? 1 : 0;
  st[s].flip = f;
  pk[s] = 0;
  pg[s] = 0;
  rank[s] = (int64_t)st[s].nlow2 - 1;  // 0-based rank of the last low element
}

// Composite key (ordered bits of the signed vector, gid): 12 digits of 8
// bits, most significant first.
__device__ inline int key_digit(uint64_t key, uint32_t g, int pass) {
  return pass < 8 ? (int)((key >> (56 - 8 * pass)) & 255) : (int)((g >> (24 - 8 * (pass - 8))) & 255);
}

__device__ inline bool key_matches(uint64_t key, uint32_t g, uint64_t pk, uint32_t pg, int pass) {
  if (pass <= 8) {
    if (pass == 0) return true;
    int sh = 64 - 8 * pass;
    return (sh == 0) ? key == pk : (key >> sh) == (pk >> sh);
  }
  if (key != pk) return false;
  int sh = 32 - 8 * (pass - 8);
  return (g >> sh) == (pg >> sh);
}

__global__ __launch_bounds__(kBlock) void k_sel_hist(
    const double *__restrict__ y, const int32_t *__restrict__ gid,
    const int32_t *__restrict__ root, const BlkDev *__restrict__ blk,
    const SegState *__restrict__ st, const uint64_t *__restrict__ pk,
    const uint32_t *__restrict__ pg, unsigned *__restrict__ hist, int pass) {
  __shared__ unsigned h[256];
  const BlkDev b = blk[blockIdx.x];
  const SegState ss = st[b.seg];
  if (ss.strad < 0) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t kp = pk[b.seg];
  const uint32_t gp = pg[b.seg];
  for (int r = threadIdx.x; r < b.nrows; r += kBlock) {
    int64_t row = b.row0 + r;
    if (root[row] != ss.strad) continue;
    double v = ss.flip ? -y[row] : y[row];
    uint64_t key = ordered_bits(v);
    uint32_t g = (uint32_t)gid[row];
    if (key_matches(key, g, kp, gp, pass)) atomicAdd(&h[key_digit(key, g, pass)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[(int64_t)b.seg * 256 + threadIdx.x], h[threadIdx.x]);
}

// One wavefront per segment: find the digit holding the target rank.
__global__ void k_sel_pick(unsigned *__restrict__ hist, const SegState *__restrict__ st,
                           uint64_t *__restrict__ pk, uint32_t *__restrict__ pg,
                           int64_t *__restrict__ rank, int nseg, int pass) {
  int s = blockIdx.x;
  if (s >= nseg || st[s].strad < 0) return;
  int lane = threadIdx.x;
  unsigned *hs = hist + (int64_t)s * 256;
  // each lane owns 4 consecutive bins
  unsigned c[4];
  unsigned tot = 0;
  for (int q = 0; q < 4; ++q) {
    c[q] = hs[lane * 4 + q];
    tot += c[q];
  }
  // inclusive scan of lane totals
  unsigned inc = tot;
  for (int off = 1; off < kWave; off <<= 1) {
    unsigned o = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += o;
  }
  unsigned excl = inc - tot;
  int64_t want = rank[s];
  int found = -1;
  int64_t below = 0;
  if ((int64_t)excl <= want && want < (int64_t)inc) {
    unsigned run = excl;
    for (int q = 0; q < 4; ++q) {
      if (want < (int64_t)(run + c[q])) {
        found = lane * 4 + q;
        below = run;
        break;
      }
      run += c[q];
    }
  }
  for (int q = 0; q < 4; ++q) hs[lane * 4 + q] = 0;
  if (found >= 0) {
    rank[s] = want - below;
    if (pass < 8) pk[s] |= (uint64_t)found << (56 - 8 * pass);
    else pg[s] |= (uint32_t)found << (24 - 8 * (pass - 8));
  }
}

__global__ void k_side(const double *__restrict__ y, const int32_t *__restrict__ gid,
                       const int32_t *__restrict__ root, const int32_t *__restrict__ size,
                       const int64_t *__restrict__ pre, const int32_t *__restrict__ orig,
                       const SegDev *__restrict__ seg, int nseg, const SegState *__restrict__ st,
                       const uint64_t *__restrict__ pk, const uint32_t *__restrict__ pg,
                       uint8_t *__restrict__ side, int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  if (orig[i] < 0) {
    side[i] = 2;
    return;
  }
  int s = seg_of_row(seg, nseg, i);
  const SegState ss = st[s];
  int r = root[i];
  if (ss.strad >= 0 && r == ss.strad) {
    double v = ss.flip ? -y[i] : y[i];
    uint64_t key = ordered_bits(v);
    uint32_t g = (uint32_t)gid[i];
    uint64_t kp = pk[s];
    uint32_t gp = pg[s];
    bool low = (key < kp) || (key == kp && g <= gp);
    side[i] = low ? 0 : 1;
  } else {
    int64_t rel = pre[r];
    side[i] = (rel + size[r] <= seg[s].nlow) ? 0 : 1;
  }
}

// Stand-alone split of one vector (test entry point): all rows one segment.
__global__ void k_split_keys(const double *__restrict__ y, const int64_t *__restrict__ gid,
                             int64_t n, uint64_t *__restrict__ key, uint64_t *__restrict__ g64) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = ordered_bits(y[i]);
  g64[i] = (uint64_t)gid[i];
}

// ---------------------------------------------------------------------------
// Compaction
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_block_low_count(const uint8_t *__restrict__ side,
                                                            const BlkDev *__restrict__ blk,
                                                            int64_t *__restrict__ cnt) {
  __shared__ int lds[kBlock / kWave];
  const BlkDev b = blk[blockIdx.x];
  int c = 0;
  for (int r = threadIdx.x; r < b.nrows; r += kBlock) c += (side[b.row0 + r] == 0);
  c = wave_sum_i(c);
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += lds[w];
    cnt[blockIdx.x] = t;
  }
}

// New row of every old row (-1: leaf or padding); leaves write their part.
__global__ __launch_bounds__(kBlock) void k_new_index(
    const uint8_t *__restrict__ side, const BlkDev *__restrict__ blk,
    const SegDev *__restrict__ seg, const int64_t *__restrict__ blk_excl,
    const int64_t *__restrict__ child_row0 /* [nseg][2], -1 leaf */,
    const int32_t *__restrict__ child_part /* [nseg][2] */, const int32_t *__restrict__ orig,
    int32_t *__restrict__ newidx, int32_t *__restrict__ part_out) {
  __shared__ int lds[kBlock];
  const BlkDev b = blk[blockIdx.x];
  const SegDev sg = seg[b.seg];
  // low rows before this block within the segment
  int64_t low_before = blk_excl[blockIdx.x] - blk_excl[sg.blk0];
  int64_t pos_before = b.row0 - sg.row0;
  for (int r0 = 0; r0 < b.nrows; r0 += kBlock) {
    int r = r0 + threadIdx.x;
    int64_t row = b.row0 + r;
    int sd = (r < b.nrows) ? side[row] : 2;
    int isl = (sd == 0);
    // block-wide inclusive scan of isl
    lds[threadIdx.x] = isl;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      int add = (threadIdx.x >= (unsigned)off) ? lds[threadIdx.x - off] : 0;
      __syncthreads();
      lds[threadIdx.x] += add;
      __syncthreads();
    }
    int incl = lds[threadIdx.x];
    int tot = lds[kBlock - 1];
    __syncthreads();
    if (r < b.nrows) {
      int ni = -1;
      if (sd < 2) {
        int64_t rank0 = low_before + incl - isl;
        int64_t p = pos_before + r;            // position in the segment
        int64_t rank = sd == 0 ? rank0 : p - rank0;
        int64_t base = child_row0[2 * b.seg + sd];
        if (base >= 0) ni = (int)(base + rank);
        else part_out[orig[row]] = child_part[2 * b.seg + sd];
      }
      newidx[row] = ni;
    }
    low_before += tot;
  }
}

__global__ void k_new_rowlen(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                             const uint8_t *__restrict__ side, const int32_t *__restrict__ newidx,
                             int32_t *__restrict__ newlen, int64_t nrows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int ni = newidx[r];
  if (ni < 0) return;
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  int sd = side[r];
  int len = 0;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) != 0 && side[colw_col(w)] == sd) ++len;
  }
  newlen[ni] = len;
}

__global__ void k_chunk_words(const int32_t *__restrict__ len, int64_t nchunks,
                              int64_t *__restrict__ words) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = r / kWave;
  if (c >= nchunks) return;
  int l = len[r];
  for (int off = kWave / 2; off > 0; off >>= 1) l = max(l, __shfl_xor(l, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) words[c] = (int64_t)l * kWave;
}

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_new_fill(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                           const uint8_t *__restrict__ side, const int32_t *__restrict__ newidx,
                           const int32_t *__restrict__ orig, const int32_t *__restrict__ gid,
                           const int64_t *__restrict__ nchunk_ptr, uint32_t *__restrict__ ncols,
                           int32_t *__restrict__ norig, int32_t *__restrict__ ngid, int64_t nrows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int ni = newidx[r];
  if (ni < 0) return;
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  int sd = side[r];
  int64_t np = nchunk_ptr[ni / kWave];
  int nlane = ni & (kWave - 1);
  int k2 = 0;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) == 0) continue;
    uint32_t j = colw_col(w);
    if (side[j] != sd) continue;
    ncols[np + (int64_t)k2 * kWave + nlane] = pack_colw((uint32_t)newidx[j], colw_wt(w));
    ++k2;
  }
  norig[ni] = orig[r];
  ngid[ni] = gid[r];
}

__global__ void k_fill_pad_rows(int32_t *__restrict__ orig, int32_t *__restrict__ gid,
                                int32_t *__restrict__ len, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  orig[i] = -1;
  gid[i] = -1;
  len[i] = 0;
}

// ---------------------------------------------------------------------------
// Laplacian apply on a level (FP64), the SpMV of the test entry point
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spmv64(const int64_t *__restrict__ chunk_ptr,
                                                   const uint32_t *__restrict__ cols,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y, int64_t nrows) {
  int64_t r = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (r >= nrows) return;
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  double xi = x[r], acc = 0.0;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) == 0) continue;  // padding slot
    acc += (double)colw_wt(w) * (xi - x[colw_col(w)]);
  }
  y[r] = acc;
}

// ---------------------------------------------------------------------------
// Metrics
// ---------------------------------------------------------------------------
__global__ void k_metrics(const int64_t *__restrict__ chunk_ptr, const uint32_t *__restrict__ cols,
                          const int32_t *__restrict__ orig, const int32_t *__restrict__ part,
                          const int32_t *__restrict__ poff /* per row global part offset */,
                          unsigned long long *__restrict__ acc, unsigned *__restrict__ bits,
                          int32_t nparts, int64_t nrows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;  // whole wavefronts
  int64_t c = r / kWave;
  int lane = (int)(r & (kWave - 1));
  int64_t p = chunk_ptr[c];
  int width = (int)((chunk_ptr[c + 1] - p) / kWave);
  const bool real = orig[r] >= 0;
  int pi = real ? part[orig[r]] + poff[r] : -1;
  if (real && (pi < 0 || pi >= nparts)) {
    atomicAdd(&acc[4], 1ull);  // unassigned element: reported as an internal error
    pi = -1;
  }
  if (pi < 0) width = 0;
  unsigned long long wcut = 0, pairs = 0;
  for (int k = 0; k < width; ++k) {
    uint32_t w = cols[p + (int64_t)k * kWave + lane];
    if (colw_wt(w) == 0) continue;
    int64_t j = colw_col(w);
    int pj = part[orig[j]] + poff[j];
    if (pj == pi || pj < 0 || pj >= nparts) continue;
    if (bits) {
      const int64_t bit = (int64_t)pi * nparts + pj;
      atomicOr(&bits[bit >> 5], 1u << (bit & 31));
    }
    if (j > r) {
      wcut += colw_wt(w);
      pairs += 1;
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    wcut += __shfl_xor(wcut, off, kWave);
    pairs += __shfl_xor(pairs, off, kWave);
  }
  if (lane == 0 && wcut) {
    atomicAdd(&acc[0], wcut);
    atomicAdd(&acc[1], pairs);
  }
}

__global__ void k_neighbor_counts(const unsigned *__restrict__ bits, int32_t nparts,
                                  unsigned long long *__restrict__ acc) {
  int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= nparts) return;
  // rows are bit-packed contiguously; count bits [pidx*nparts, (pidx+1)*nparts)
  int64_t b0 = (int64_t)pidx * nparts, b1 = b0 + nparts;
  unsigned cnt = 0;
  for (int64_t b = b0; b < b1;) {
    int64_t wi = b >> 5;
    int off = (int)(b & 31);
    int take = (int)std::min<int64_t>(32 - off, b1 - b);
    unsigned v = bits[wi] >> off;
    if (take < 32) v &= (1u << take) - 1u;
    cnt += __popc(v);
    b += take;
  }
  atomicMax(&acc[2], (unsigned long long)cnt);
  atomicAdd(&acc[3], (unsigned long long)cnt);
}

__global__ void k_row_part_offset(const int32_t *__restrict__ orig, const SegDev *__restrict__ seg,
                                  int nseg, const int32_t *__restrict__ mesh_off,
                                  int32_t *__restrict__ poff, int64_t nrows) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int s = seg_of_row(seg, nseg, i);
  poff[i] = mesh_off[seg[s].mesh];
}

// Packed copy of the slices (the layout is described with kPackOffBits):
// one wavefront per slice.  The window bases cover the slice's deltas
// (column - row) greedily from the least one (each base is the least delta
// the windows before it leave uncovered), which needs the fewest windows; a
// slice that needs more than kPackClusters keeps only its 32-bit words.  The
// exact column range of each window (least and greatest column, over the
// slice's rows) goes to crlo / crhi for the staging of tiles.
__device__ inline int32_t wave_min_i32(int32_t v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ inline int32_t wave_max_i32(int32_t v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

constexpr int kPackRegSlots = 32;  // slots a row keeps in registers while packing

template <bool REG>
__device__ inline uint32_t pack_word(const uint32_t *cp, const uint32_t (&wr)[kPackRegSlots], int k) {
  if (REG) {
    uint32_t w = 0;
#pragma unroll
    for (int u = 0; u < kPackRegSlots; ++u) w = (u == k) ? wr[u] : w;
    return w;
  }
  return cp[(int64_t)k * kWave];
}

// Returns the slice's nonzeros when it is packed, -1 when it stays in words.
template <bool REG>
__device__ int pack_one_slice(const uint32_t *cp, int width, int32_t row, int lane,
                              uint32_t *out, int4 *meta, int4 *crlo, int4 *crhi, int64_t c) {
  uint32_t wr[kPackRegSlots];
#pragma unroll
  for (int u = 0; u < kPackRegSlots; ++u) wr[u] = (REG && u < width) ? cp[(int64_t)u * kWave] : 0u;
  int32_t b[kPackClusters] = {0, 0, 0, 0};
  int nb = 0;
  bool fits = true;
  int32_t covered = INT32_MIN;  // deltas <= covered lie in a window
  for (;;) {
    int32_t mn = INT32_MAX;
    for (int k = 0; k < width; ++k) {
      const uint32_t w = pack_word<REG>(cp, wr, k);
      const int32_t d = (int32_t)colw_col(w) - row;
      if (colw_wt(w) && d > covered && d < mn) mn = d;
    }
    mn = wave_min_i32(mn);
    if (mn == INT32_MAX) break;
    if (nb == kPackClusters) {
      fits = false;
      break;
    }
#pragma unroll
    for (int i = 0; i < kPackClusters; ++i) b[i] = (i == nb) ? mn : b[i];
    ++nb;
    covered = mn + ((1 << kPackOffBits) - 1);
  }
  if (!fits) {
    if (lane == 0) {
      meta[c] = make_int4(kPlainSlice, 0, 0, 0);
      crlo[c] = make_int4(INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX);
      crhi[c] = make_int4(INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN);
    }
    return -1;
  }
  int32_t lo[kPackClusters] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  int32_t hi[kPackClusters] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
  int nz = 0;
  for (int q = 0; 2 * q < width; ++q) {
    uint32_t h[2] = {0u, 0u};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = 2 * q + t;
      const uint32_t w = k < width ? pack_word<REG>(cp, wr, k) : 0u;
      if (colw_wt(w)) {
        const int32_t col = (int32_t)colw_col(w);
        const int32_t d = col - row;
        // window: the last base <= d (bases ascending, unused ones never match)
        const int i = (nb > 1 && d >= b[1]) + (nb > 2 && d >= b[2]) + (nb > 3 && d >= b[3]);
        const int32_t base = i == 0 ? b[0] : i == 1 ? b[1] : i == 2 ? b[2] : b[3];
        h[t] = (colw_wt(w) << 12) | ((uint32_t)i << kPackOffBits) | (uint32_t)(d - base);
#pragma unroll
        for (int u = 0; u < kPackClusters; ++u) {
          lo[u] = (u == i) ? min(lo[u], col) : lo[u];
          hi[u] = (u == i) ? max(hi[u], col) : hi[u];
        }
        ++nz;
      }
    }
    out[(int64_t)q * kWave] = h[0] | (h[1] << 16);
  }
#pragma unroll
  for (int u = 0; u < kPackClusters; ++u) {
    lo[u] = wave_min_i32(lo[u]);
    hi[u] = wave_max_i32(hi[u]);
  }
  nz = wave_sum_i(nz);
  if (lane == 0) {
    meta[c] = make_int4(b[0], b[1], b[2], b[3]);
    crlo[c] = make_int4(lo[0], lo[1], lo[2], lo[3]);
    crhi[c] = make_int4(hi[0], hi[1], hi[2], hi[3]);
  }
  return nz;
}

__global__ __launch_bounds__(kBlock) void k_pack_slices(const int64_t *__restrict__ chunk_ptr,
                                                       const uint32_t *__restrict__ cols,
                                                       int64_t nchunks, uint32_t *__restrict__ pk,
                                                       int4 *__restrict__ meta,
                                                       int4 *__restrict__ crlo,
                                                       int4 *__restrict__ crhi,
                                                       unsigned long long *__restrict__ cnt) {
  // slices strided over the grid's wavefronts; the counts summed per block
  // (one pair of atomics per block)
  __shared__ unsigned long long red[2][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  unsigned long long nz = 0, ns = 0;
  for (int64_t c = (int64_t)blockIdx.x * (kBlock / kWave) + wave; c < nchunks; c += nwaves) {
    const int64_t p = chunk_ptr[c];
    const int width = (int)((chunk_ptr[c + 1] - p) >> 6);
    const int32_t row = (int32_t)(c * kWave + lane);
    const uint32_t *cp = cols + p + lane;
    uint32_t *out = pk + packed_slice_word(p, c) + lane;
    const int r = width <= kPackRegSlots
                      ? pack_one_slice<true>(cp, width, row, lane, out, meta, crlo, crhi, c)
                      : pack_one_slice<false>(cp, width, row, lane, out, meta, crlo, crhi, c);
    if (r >= 0) {
      nz += (unsigned long long)r;
      ns += 1;
    }
  }
  if (lane == 0) {
    red[0][wave] = nz;
    red[1][wave] = ns;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      nz += red[0][w];
      ns += red[1][w];
    }
    atomicAdd(&cnt[0], nz);
    atomicAdd(&cnt[1], ns);
  }
}

__global__ void k_meta_plain(int4 *meta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) meta[i] = make_int4(kPlainSlice, 0, 0, 0);
}

// Staging of a tile's gathers (one wavefront per tile): the column ranges of
// the windows of its packed slices, merged where they overlap or lie within
// kStageGap of each other, become at most kStageMaxInt intervals of the
// vector that the tile's launch copies into LDS (at most kStageCap values
// together); lmeta then holds, per slice and window, the base that turns a
// packed entry into an LDS index (interval offset - interval start + window
// base).  A tile whose ranges need more is not staged (nint = 0).
__global__ __launch_bounds__(kBlock) void k_stage_tiles(const BlkDev *__restrict__ blk, int nblk,
                                                       const int4 *__restrict__ meta,
                                                       const int4 *__restrict__ crlo,
                                                       const int4 *__restrict__ crhi,
                                                       TileStage *__restrict__ stage,
                                                       int4 *__restrict__ lmeta,
                                                       unsigned *__restrict__ nstaged) {
  const int t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (t >= nblk) return;  // the whole wavefront
  const int lane = threadIdx.x & (kWave - 1);
  const BlkDev bk = blk[t];
  const int64_t c0 = bk.row0 >> 6;
  const int ns = bk.nrows >> 6;
  // range r = 4 (slice) + window; a lane holds ranges lane + 64 i
  constexpr int kR = 4;  // ranges per lane: tiles of up to 64 slices
  int32_t rlo[kR], rhi[kR], rk[kR];
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int r = lane + kWave * i;
    rlo[i] = INT32_MAX;
    rhi[i] = INT32_MIN;
    rk[i] = -1;
    if (r < 4 * ns) {
      const int64_t c = c0 + (r >> 2);
      const int4 lo = crlo[c], hi = crhi[c];
      const int u = r & 3;
      rlo[i] = u == 0 ? lo.x : u == 1 ? lo.y : u == 2 ? lo.z : lo.w;
      rhi[i] = u == 0 ? hi.x : u == 1 ? hi.y : u == 2 ? hi.z : hi.w;
      if (rlo[i] > rhi[i]) rk[i] = kStageMaxInt;  // empty (or a slice in words)
    } else {
      rk[i] = kStageMaxInt;
    }
  }
  TileStage ts{};
  int32_t off = 0;
  bool ok = ns <= kR * kWave / 4;
  for (int k = 0; ok; ++k) {
    int32_t lo = INT32_MAX;
#pragma unroll
    for (int i = 0; i < kR; ++i) lo = (rk[i] < 0) ? min(lo, rlo[i]) : lo;
    lo = wave_min_i32(lo);
    if (lo == INT32_MAX) break;  // every range placed
    if (k == kStageMaxInt) {
      ok = false;
      break;
    }
    int32_t hi = lo;
    for (;;) {
      int32_t h = hi;
#pragma unroll
      for (int i = 0; i < kR; ++i)
        h = (rk[i] < 0 && rlo[i] <= hi + kStageGap) ? max(h, rhi[i]) : h;
      h = wave_max_i32(h);
      if (h == hi) break;
      hi = h;
    }
#pragma unroll
    for (int i = 0; i < kR; ++i) rk[i] = (rk[i] < 0 && rlo[i] <= hi + kStageGap) ? k : rk[i];
    ts.lo[k] = lo;
    ts.len[k] = hi - lo + 1;
    ts.off[k] = off;
    off += hi - lo + 1;
    ts.nint = k + 1;
    if (off > kStageCap) ok = false;
  }
  ts.total = off;
  if (!ok) ts.nint = 0;
  if (lane == 0) {
    stage[c0] = ts;
    if (ts.nint > 0) atomicAdd(nstaged, 1u);
  }
  // the LDS bases of the tile's packed slices
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int r = lane + kWave * i;
    if (r < 4 * ns) {
      const int64_t c = c0 + (r >> 2);
      const int u = r & 3;
      const int4 mb = meta[c];
      const int32_t base = u == 0 ? mb.x : u == 1 ? mb.y : u == 2 ? mb.z : mb.w;
      int32_t v = 0;
      if (ts.nint > 0 && rk[i] >= 0 && rk[i] < kStageMaxInt) {
        int32_t klo = 0, koff = 0;
#pragma unroll
        for (int k = 0; k < kStageMaxInt; ++k)
          if (k == rk[i]) {
            klo = ts.lo[k];
            koff = ts.off[k];
          }
        v = base + koff - klo;
      }
      reinterpret_cast<int32_t *>(lmeta)[4 * c + u] = v;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void pack_level(Level &L, Ctx &ctx) {
  L.pmeta.alloc(ctx, std::max<int64_t>(L.nchunks, 1));
  L.packed_slices = L.packed_nnz = 0;
  if (L.nchunks == 0) return;
  if (ctx.pack == 0) {
    k_meta_plain<<<grid_for(L.nchunks, kBlock), kBlock, 0, ctx.stream>>>(L.pmeta.get(), L.nchunks);
    RSB_LAUNCHED();
    return;
  }
  L.pk.alloc(ctx, std::max<int64_t>(packed_slice_word(L.words, L.nchunks), 1));
  L.crlo.alloc(ctx, L.nchunks);
  L.crhi.alloc(ctx, L.nchunks);
  DevBuf<unsigned long long> cnt(ctx, 2);
  RSB_HIP(hipMemsetAsync(cnt.get(), 0, 2 * sizeof(unsigned long long), ctx.stream));
  const int64_t per = kBlock / kWave;
  const unsigned grid = (unsigned)std::min<int64_t>((L.nchunks + per - 1) / per, 2048);
  k_pack_slices<<<grid, kBlock, 0, ctx.stream>>>(
      L.chunk_ptr.get(), L.cols.get(), L.nchunks, L.pk.get(), L.pmeta.get(), L.crlo.get(),
      L.crhi.get(), cnt.get());
  RSB_LAUNCHED();
  unsigned long long h[2] = {0, 0};
  RSB_HIP(hipMemcpyAsync(h, cnt.get(), sizeof(h), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  L.packed_nnz = (int64_t)h[0];
  L.packed_slices = (int64_t)h[1];
}

// The staging tables of the level's current tiles (levels with a packed
// copy only; other tiles are never staged).
void stage_tiles(Level &L, Ctx &ctx) {
  if (L.nchunks == 0 || L.crlo.get() == nullptr || L.blk.empty()) return;
  L.stage.alloc(ctx, L.nchunks);
  L.lmeta.alloc(ctx, L.nchunks);
  RSB_HIP(hipMemsetAsync(L.stage.get(), 0, L.nchunks * sizeof(TileStage), ctx.stream));
  L.staged_tiles = 0;
  if (ctx.pack < 2) return;
  DevBuf<unsigned> cnt(ctx, 1);
  RSB_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(unsigned), ctx.stream));
  const int per = kBlock / kWave;
  k_stage_tiles<<<(unsigned)((L.nblk + per - 1) / per), kBlock, 0, ctx.stream>>>(
      L.d_blk.get(), L.nblk, L.pmeta.get(), L.crlo.get(), L.crhi.get(), L.stage.get(),
      L.lmeta.get(), cnt.get());
  RSB_LAUNCHED();
  unsigned h = 0;
  RSB_HIP(hipMemcpyAsync(&h, cnt.get(), sizeof(unsigned), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  L.staged_tiles = (int64_t)h;
}

void level_tables(Level &L, int rpt, Ctx &ctx) {
  L.rpt = rpt;
  L.blk.clear();
  L.grp.clear();
  const int64_t tile = (int64_t)kBlock * rpt;
  for (int s = 0; s < L.nseg; ++s) {
    SegDev &sg = L.seg[s];
    sg.blk0 = (int32_t)L.blk.size();
    sg.grp0 = (int32_t)L.grp.size();
    int64_t nb = std::max<int64_t>(1, (sg.npad + tile - 1) / tile);
    // about sqrt(nb) blocks per group (at least kGroup): both reduction
    // stages then read about as many partials per segment
    int64_t gs = kGroup;
    while (gs * gs < nb) gs += 8;
    for (int64_t b = 0; b < nb; ++b) {
      BlkDev bd{};
      bd.row0 = sg.row0 + b * tile;
      bd.nrows = (int32_t)std::min<int64_t>(tile, sg.npad - b * tile);
      bd.seg = s;
      bd.grp = sg.grp0 + (int32_t)(b / gs);
      L.blk.push_back(bd);
    }
    sg.nblk = (int32_t)nb;
    int64_t ng = (nb + gs - 1) / gs;
    for (int64_t g = 0; g < ng; ++g) {
      GrpDev gd{};
      gd.seg = s;
      gd.blk0 = sg.blk0 + (int32_t)(g * gs);
      gd.nblk = (int32_t)std::min<int64_t>(gs, nb - g * gs);
      L.grp.push_back(gd);
    }
    sg.ngrp = (int32_t)ng;
  }
  L.nblk = (int32_t)L.blk.size();
  L.ngrp = (int32_t)L.grp.size();
  L.d_seg.alloc(ctx, L.seg.size());
  L.d_blk.alloc(ctx, L.blk.size());
  L.d_grp.alloc(ctx, L.grp.size());
  RSB_HIP(hipMemcpyAsync(L.d_seg.get(), L.seg.data(), L.seg.size() * sizeof(SegDev),
                         hipMemcpyHostToDevice, ctx.stream));
  RSB_HIP(hipMemcpyAsync(L.d_blk.get(), L.blk.data(), L.blk.size() * sizeof(BlkDev),
                         hipMemcpyHostToDevice, ctx.stream));
  RSB_HIP(hipMemcpyAsync(L.d_grp.get(), L.grp.data(), L.grp.size() * sizeof(GrpDev),
                         hipMemcpyHostToDevice, ctx.stream));
  stage_tiles(L, ctx);
  // the host vectors must stay alive until the copies ran
  RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void level0_from_csr(Level &L, const std::vector<const DevCsr *> &g,
                     const std::vector<int32_t> &nparts, int rpt, Ctx &ctx,
                     const std::vector<const int32_t *> *perm) {
  // segments for meshes that need splitting
  L.seg.clear();
  int64_t row = 0;
  std::vector<int64_t> orig_base(g.size(), 0);
  int64_t ob = 0;
  for (size_t b = 0; b < g.size(); ++b) {
    orig_base[b] = ob;
    ob += g[b]->n;
  }
  std::vector<int> mesh_seg;
  for (size_t b = 0; b < g.size(); ++b) {
    if (nparts[b] < 2) continue;
    SegDev sd{};
    sd.row0 = row;
    sd.n = (int32_t)g[b]->n;
    sd.npad = (int32_t)round_up(sd.n, kWave);
    sd.P = nparts[b];
    sd.p0 = 0;
    sd.nlow = (int32_t)((int64_t)sd.n * (sd.P / 2) / sd.P);
    sd.mesh = (int32_t)b;
    row += sd.npad;
    L.seg.push_back(sd);
    mesh_seg.push_back((int)b);
  }
  L.nseg = (int32_t)L.seg.size();
  L.nrows = row;
  L.nchunks = row / kWave;
  if (L.nrows >= kMaxRows) fail(RSB_EINVAL, "too many elements (limit 2^28 per call)");
  L.chunk_ptr.alloc(ctx, L.nchunks + 1);
  L.orig.alloc(ctx, std::max<int64_t>(L.nrows, 1));
  L.gid.alloc(ctx, std::max<int64_t>(L.nrows, 1));
  if (L.nseg == 0) {
    pack_level(L, ctx);
    level_tables(L, rpt, ctx);
    return;
  }
  DevBuf<int64_t> words(ctx, L.nchunks);
  for (int s = 0; s < L.nseg; ++s) {
    const DevCsr &c = *g[mesh_seg[s]];
    int64_t nch = L.seg[s].npad / kWave;
    k_chunk_words_csr<<<grid_for(L.seg[s].npad, kBlock), kBlock, 0, ctx.stream>>>(
        c.row_ptr.get(), c.n, L.seg[s].row0, L.seg[s].row0 / kWave, nch, words.get());
    RSB_LAUNCHED();
  }
  scan_exclusive(words.get(), L.nchunks, L.chunk_ptr.get(), L.chunk_ptr.get() + L.nchunks, ctx);
  RSB_HIP(hipMemcpyAsync(&L.words, L.chunk_ptr.get() + L.nchunks, sizeof(int64_t),
                         hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  L.cols.alloc(ctx, L.words + kColSlack);
  k_zero_u32<<<grid_for(kColSlack, kBlock), kBlock, 0, ctx.stream>>>(L.cols.get() + L.words,
                                                                     kColSlack);
  RSB_LAUNCHED();
  L.nnz = 0;
  for (int s = 0; s < L.nseg; ++s) L.nnz += g[mesh_seg[s]]->nnz;
  for (int s = 0; s < L.nseg; ++s) {
    const DevCsr &c = *g[mesh_seg[s]];
    int64_t nch = L.seg[s].npad / kWave;
    k_fill_sell_csr<<<grid_for(L.seg[s].npad, kBlock), kBlock, 0, ctx.stream>>>(
        c.row_ptr.get(), c.col.get(), c.wgt.get(), c.n, L.seg[s].row0, L.seg[s].row0 / kWave,
        nch, L.chunk_ptr.get(), L.cols.get(), L.orig.get(), L.gid.get(),
        orig_base[mesh_seg[s]], perm ? (*perm)[mesh_seg[s]] : nullptr);
    RSB_LAUNCHED();
  }
  pack_level(L, ctx);
  level_tables(L, rpt, ctx);
}

void components_and_targets(Level &L, CompDev &C, SolveDev &S, Ctx &ctx) {
  const int64_t n = L.nrows;
  C.root.alloc(ctx, std::max<int64_t>(n, 1));
  C.size.alloc(ctx, std::max<int64_t>(n, 1));
  C.pre.alloc(ctx, std::max<int64_t>(n, 1) + 1);
  k_seg_state_init<<<grid_for(L.nseg, 64), 64, 0, ctx.stream>>>(S.st.get(), L.d_seg.get(), L.nseg);
  RSB_LAUNCHED();
  if (n == 0) return;
  unsigned g = grid_for(n, kBlock);
  k_cc_init<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), C.size.get(), n);
  RSB_LAUNCHED();
  k_cc_init_link<<<g, kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(), L.orig.get(),
                                               C.root.get(), n);
  RSB_LAUNCHED();
  k_cc_flatten<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), L.orig.get(), n);
  RSB_LAUNCHED();
  k_cc_hook<true><<<g, kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(), L.orig.get(),
                                                L.d_seg.get(), L.nseg, C.root.get(), n);
  RSB_LAUNCHED();
  k_cc_flatten<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), L.orig.get(), n);
  RSB_LAUNCHED();
  k_cc_hook<false><<<g, kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(), L.orig.get(),
                                                 L.d_seg.get(), L.nseg, C.root.get(), n);
  RSB_LAUNCHED();
  k_cc_compress<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), C.size.get(), L.orig.get(), n);
  RSB_LAUNCHED();
  // components in order of their least global id within each segment (the
  // rows need not be in global-id order, see the locality order)
  {
    DevBuf<int32_t> mingid(ctx, n), flag(ctx, n);
    DevBuf<int64_t> pos(ctx, n + 1);
    fill_i32(mingid.get(), n, 0x7fffffff, ctx);
    k_cc_mingid<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), L.gid.get(), L.orig.get(), n,
                                              mingid.get());
    k_cc_root_flag<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), L.orig.get(), n, flag.get());
    RSB_LAUNCHED();
    scan_exclusive(flag.get(), n, pos.get(), pos.get() + n, ctx);
    int64_t nroots = 0;
    RSB_HIP(hipMemcpyAsync(&nroots, pos.get() + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                           ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    if (nroots > 0) {
      DevBuf<uint64_t> keys(ctx, nroots);
      DevBuf<uint32_t> vals(ctx, nroots);
      DevBuf<int64_t> sz(ctx, nroots), off(ctx, nroots + 1);
      k_cc_root_keys<<<g, kBlock, 0, ctx.stream>>>(flag.get(), pos.get(), mingid.get(),
                                                   L.d_seg.get(), L.nseg, n, keys.get(),
                                                   vals.get());
      RSB_LAUNCHED();
      int segbits = 0;
      while ((1ll << segbits) < (int64_t)L.nseg) ++segbits;
      sort_pairs(keys.get(), vals.get(), nroots, 32 + segbits, ctx);
      const unsigned gk = grid_for(nroots, kBlock);
      k_cc_root_sizes<<<gk, kBlock, 0, ctx.stream>>>(vals.get(), C.size.get(), nroots, sz.get());
      RSB_LAUNCHED();
      scan_exclusive(sz.get(), nroots, off.get(), off.get() + nroots, ctx);
      DevBuf<int64_t> base(ctx, std::max(L.nseg, 1));
      k_cc_seg_base<<<gk, kBlock, 0, ctx.stream>>>(keys.get(), off.get(), nroots, base.get());
      k_cc_root_pre<<<gk, kBlock, 0, ctx.stream>>>(keys.get(), vals.get(), off.get(), base.get(),
                                                   nroots, C.pre.get());
      RSB_LAUNCHED();
    }
    RSB_HIP(hipStreamSynchronize(ctx.stream));
  }
  k_cc_targets<<<g, kBlock, 0, ctx.stream>>>(C.root.get(), C.size.get(), C.pre.get(),
                                             L.orig.get(), L.d_seg.get(), L.nseg, S.st.get(), n);
  RSB_LAUNCHED();
}

void split_level(Level &L, CompDev &C, SolveDev &S, const double *y64, uint8_t *side, Ctx &ctx) {
  const int64_t n = L.nrows;
  if (n == 0) return;
  DevBuf<unsigned long long> ymax(ctx, L.nseg);
  DevBuf<uint64_t> pk(ctx, L.nseg);
  DevBuf<uint32_t> pg(ctx, L.nseg);
  DevBuf<int64_t> rank(ctx, L.nseg);
  DevBuf<unsigned> hist(ctx, (size_t)L.nseg * 256);
  RSB_HIP(hipMemsetAsync(ymax.get(), 0, ymax.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(hist.get(), 0, hist.bytes(), ctx.stream));
  unsigned g = grid_for(n, kBlock);
  DevBuf<unsigned long long> firstkey(ctx, L.nseg);
  RSB_HIP(hipMemsetAsync(firstkey.get(), 0xFF, firstkey.bytes(), ctx.stream));
  k_sign_max<<<g, kBlock, 0, ctx.stream>>>(y64, C.root.get(), L.d_seg.get(), L.nseg, S.st.get(),
                                           ymax.get(), n);
  RSB_LAUNCHED();
  k_sign_first<<<g, kBlock, 0, ctx.stream>>>(y64, C.root.get(), L.gid.get(), L.d_seg.get(),
                                             L.nseg, S.st.get(), ymax.get(), n, firstkey.get());
  RSB_LAUNCHED();
  k_sign_flip<<<grid_for(L.nseg, 64), 64, 0, ctx.stream>>>(y64, S.st.get(), L.nseg, pk.get(),
                                                           pg.get(), rank.get(), firstkey.get());
  RSB_LAUNCHED();
  for (int pass = 0; pass < 12; ++pass) {
    k_sel_hist<<<L.nblk, kBlock, 0, ctx.stream>>>(y64, L.gid.get(), C.root.get(), L.d_blk.get(),
                                                  S.st.get(), pk.get(), pg.get(), hist.get(),
                                                  pass);
    RSB_LAUNCHED();
    k_sel_pick<<<L.nseg, kWave, 0, ctx.stream>>>(hist.get(), S.st.get(), pk.get(), pg.get(),
                                                 rank.get(), L.nseg, pass);
    RSB_LAUNCHED();
  }
  k_side<<<g, kBlock, 0, ctx.stream>>>(y64, L.gid.get(), C.root.get(), C.size.get(), C.pre.get(),
                                       L.orig.get(), L.d_seg.get(), L.nseg, S.st.get(), pk.get(),
                                       pg.get(), side, n);
  RSB_LAUNCHED();
}

void canonical_sign_level(Level &L, CompDev &C, SolveDev &S, double *y, Ctx &ctx) {
  const int64_t n = L.nrows;
  if (n == 0) return;
  DevBuf<unsigned long long> ymax(ctx, L.nseg);
  DevBuf<uint64_t> pk(ctx, L.nseg);
  DevBuf<uint32_t> pg(ctx, L.nseg);
  DevBuf<int64_t> rank(ctx, L.nseg);
  RSB_HIP(hipMemsetAsync(ymax.get(), 0, ymax.bytes(), ctx.stream));
  const unsigned g = grid_for(n, kBlock);
  DevBuf<unsigned long long> firstkey(ctx, L.nseg);
  RSB_HIP(hipMemsetAsync(firstkey.get(), 0xFF, firstkey.bytes(), ctx.stream));
  k_sign_max<<<g, kBlock, 0, ctx.stream>>>(y, C.root.get(), L.d_seg.get(), L.nseg, S.st.get(),
                                           ymax.get(), n);
  k_sign_first<<<g, kBlock, 0, ctx.stream>>>(y, C.root.get(), L.gid.get(), L.d_seg.get(), L.nseg,
                                             S.st.get(), ymax.get(), n, firstkey.get());
  k_sign_flip<<<grid_for(L.nseg, 64), 64, 0, ctx.stream>>>(y, S.st.get(), L.nseg, pk.get(),
                                                           pg.get(), rank.get(), firstkey.get());
  k_sign_apply<<<g, kBlock, 0, ctx.stream>>>(y, C.root.get(), L.d_seg.get(), L.nseg, S.st.get(),
                                             n);
  RSB_LAUNCHED();
}

void split_vector(const double *d_y, const int64_t *d_gid, int64_t n, int64_t n_low,
                  uint8_t *d_side, Ctx &ctx) {
  // One segment holding all rows: a level with identity components.
  Level L;
  SegDev sd{};
  sd.row0 = 0;
  sd.n = (int32_t)n;
  sd.npad = (int32_t)round_up(n, kWave);
  sd.P = 2;
  sd.nlow = (int32_t)n_low;
  L.seg.push_back(sd);
  L.nseg = 1;
  L.nrows = sd.npad;
  level_tables(L, 16, ctx);
  DevBuf<double> y(ctx, L.nrows);
  DevBuf<int32_t> gid(ctx, L.nrows), root(ctx, L.nrows);
  DevBuf<SegState> st(ctx, 1);
  // copy y and gid into the padded arrays; all real rows share root 0
  RSB_HIP(hipMemsetAsync(y.get(), 0, y.bytes(), ctx.stream));
  RSB_HIP(hipMemcpyAsync(y.get(), d_y, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  std::vector<int32_t> hg(L.nrows, -1), hr(L.nrows, -1);
  std::vector<int64_t> gsrc(n);
  RSB_HIP(hipMemcpyAsync(gsrc.data(), d_gid, n * sizeof(int64_t), hipMemcpyDeviceToHost,
                         ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  for (int64_t i = 0; i < n; ++i) {
    if (gsrc[i] < 0 || gsrc[i] >= (int64_t)1 << 31) fail(RSB_EINVAL, "gid out of range");
    hg[i] = (int32_t)gsrc[i];
    hr[i] = 0;
  }
  RSB_HIP(hipMemcpyAsync(gid.get(), hg.data(), L.nrows * sizeof(int32_t), hipMemcpyHostToDevice,
                         ctx.stream));
  RSB_HIP(hipMemcpyAsync(root.get(), hr.data(), L.nrows * sizeof(int32_t), hipMemcpyHostToDevice,
                         ctx.stream));
  SegState hs = {};
  hs.strad = 0;
  hs.nlow2 = (int32_t)n_low;
  hs.first = 0x7fffffff;
  RSB_HIP(hipMemcpyAsync(st.get(), &hs, sizeof(hs), hipMemcpyHostToDevice, ctx.stream));
  DevBuf<uint64_t> pk(ctx, 1);
  DevBuf<uint32_t> pg(ctx, 1);
  DevBuf<int64_t> rank(ctx, 1);
  DevBuf<unsigned> hist(ctx, 256);
  RSB_HIP(hipMemsetAsync(hist.get(), 0, hist.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(pk.get(), 0, pk.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(pg.get(), 0, pg.bytes(), ctx.stream));
  int64_t r0 = n_low - 1;
  RSB_HIP(hipMemcpyAsync(rank.get(), &r0, sizeof(r0), hipMemcpyHostToDevice, ctx.stream));
  if (n_low > 0) {
    for (int pass = 0; pass < 12; ++pass) {
      k_sel_hist<<<L.nblk, kBlock, 0, ctx.stream>>>(y.get(), gid.get(), root.get(),
                                                    L.d_blk.get(), st.get(), pk.get(), pg.get(),
                                                    hist.get(), pass);
      RSB_LAUNCHED();
      k_sel_pick<<<1, kWave, 0, ctx.stream>>>(hist.get(), st.get(), pk.get(), pg.get(),
                                              rank.get(), 1, pass);
      RSB_LAUNCHED();
    }
  }
  // side: composite key <= threshold (none when n_low == 0)
  DevBuf<int32_t> orig(ctx, L.nrows), size(ctx, L.nrows);
  DevBuf<int64_t> pre(ctx, L.nrows);
  std::vector<int32_t> ho(L.nrows, -1);
  for (int64_t i = 0; i < n; ++i) ho[i] = (int32_t)i;
  RSB_HIP(hipMemcpyAsync(orig.get(), ho.data(), L.nrows * sizeof(int32_t), hipMemcpyHostToDevice,
                         ctx.stream));
  RSB_HIP(hipMemsetAsync(size.get(), 0, size.bytes(), ctx.stream));
  RSB_HIP(hipMemsetAsync(pre.get(), 0, pre.bytes(), ctx.stream));
  if (n_low == 0) {
    // no low element: a threshold below every key
    hs.strad = -1;
    RSB_HIP(hipMemcpyAsync(st.get(), &hs, sizeof(hs), hipMemcpyHostToDevice, ctx.stream));
    // component rule with one "component" of size n at root 0 (rel 0):
    // 0 + size <= 0 is false -> all high
    std::vector<int32_t> hsz(L.nrows, 0);
    hsz[0] = (int32_t)n;
    RSB_HIP(hipMemcpyAsync(size.get(), hsz.data(), L.nrows * sizeof(int32_t),
                           hipMemcpyHostToDevice, ctx.stream));
  }
  DevBuf<uint8_t> side(ctx, L.nrows);
  k_side<<<grid_for(L.nrows, kBlock), kBlock, 0, ctx.stream>>>(
      y.get(), gid.get(), root.get(), size.get(), pre.get(), orig.get(), L.d_seg.get(), 1,
      st.get(), pk.get(), pg.get(), side.get(), L.nrows);
  RSB_LAUNCHED();
  RSB_HIP(hipMemcpyAsync(d_side, side.get(), n, hipMemcpyDeviceToDevice, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void compact_level(Level &L, const uint8_t *side, int32_t *d_part_out, Level &next, int rpt,
                   Ctx &ctx) {
  // next level's segments, computed on the host from the balance rule
  next.seg.clear();
  std::vector<int64_t> child_row0(2 * (size_t)L.nseg, -1);
  std::vector<int32_t> child_part(2 * (size_t)L.nseg, 0);
  int64_t row = 0;
  for (int s = 0; s < L.nseg; ++s) {
    const SegDev &sg = L.seg[s];
    int32_t PL = sg.P / 2;
    int32_t nc[2] = {sg.nlow, sg.n - sg.nlow};
    int32_t Pc[2] = {PL, sg.P - PL};
    int32_t p0c[2] = {sg.p0, sg.p0 + PL};
    for (int d = 0; d < 2; ++d) {
      child_part[2 * s + d] = p0c[d];
      if (Pc[d] < 2) continue;
      SegDev c{};
      c.row0 = row;
      c.n = nc[d];
      c.npad = (int32_t)round_up(c.n, kWave);
      c.P = Pc[d];
      c.p0 = p0c[d];
      c.nlow = (int32_t)((int64_t)c.n * (c.P / 2) / c.P);
      c.mesh = sg.mesh;
      child_row0[2 * s + d] = row;
      row += c.npad;
      next.seg.push_back(c);
    }
  }
  next.nseg = (int32_t)next.seg.size();
  next.nrows = row;
  next.nchunks = row / kWave;
  DevBuf<int64_t> d_child_row0(ctx, child_row0.size());
  DevBuf<int32_t> d_child_part(ctx, child_part.size());
  RSB_HIP(hipMemcpyAsync(d_child_row0.get(), child_row0.data(),
                         child_row0.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
  RSB_HIP(hipMemcpyAsync(d_child_part.get(), child_part.data(),
                         child_part.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
  // element ranks within each segment
  DevBuf<int64_t> bcnt(ctx, L.nblk), bexcl(ctx, L.nblk + 1);
  k_block_low_count<<<L.nblk, kBlock, 0, ctx.stream>>>(side, L.d_blk.get(), bcnt.get());
  RSB_LAUNCHED();
  scan_exclusive(bcnt.get(), L.nblk, bexcl.get(), bexcl.get() + L.nblk, ctx);
  DevBuf<int32_t> newidx(ctx, std::max<int64_t>(L.nrows, 1));
  k_new_index<<<L.nblk, kBlock, 0, ctx.stream>>>(side, L.d_blk.get(), L.d_seg.get(), bexcl.get(),
                                                 d_child_row0.get(), d_child_part.get(),
                                                 L.orig.get(), newidx.get(), d_part_out);
  RSB_LAUNCHED();
  next.chunk_ptr.alloc(ctx, next.nchunks + 1);
  next.orig.alloc(ctx, std::max<int64_t>(next.nrows, 1));
  next.gid.alloc(ctx, std::max<int64_t>(next.nrows, 1));
  if (next.nseg == 0) {
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    pack_level(next, ctx);
    level_tables(next, rpt, ctx);
    return;
  }
  DevBuf<int32_t> newlen(ctx, next.nrows);
  k_fill_pad_rows<<<grid_for(next.nrows, kBlock), kBlock, 0, ctx.stream>>>(
      next.orig.get(), next.gid.get(), newlen.get(), next.nrows);
  RSB_LAUNCHED();
  const unsigned g = grid_for(L.nrows, kBlock);
  k_new_rowlen<<<g, kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(), side, newidx.get(),
                                             newlen.get(), L.nrows);
  RSB_LAUNCHED();
  {
    DevBuf<int64_t> lexcl(ctx, next.nrows + 1);
    scan_exclusive(newlen.get(), next.nrows, lexcl.get(), lexcl.get() + next.nrows, ctx);
    RSB_HIP(hipMemcpyAsync(&next.nnz, lexcl.get() + next.nrows, sizeof(int64_t),
                           hipMemcpyDeviceToHost, ctx.stream));
  }
  DevBuf<int64_t> words(ctx, next.nchunks);
  k_chunk_words<<<grid_for(next.nrows, kBlock), kBlock, 0, ctx.stream>>>(newlen.get(),
                                                                        next.nchunks, words.get());
  RSB_LAUNCHED();
  scan_exclusive(words.get(), next.nchunks, next.chunk_ptr.get(),
                 next.chunk_ptr.get() + next.nchunks, ctx);
  RSB_HIP(hipMemcpyAsync(&next.words, next.chunk_ptr.get() + next.nchunks, sizeof(int64_t),
                         hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  next.cols.alloc(ctx, next.words + kColSlack);
  k_zero_u32<<<grid_for(next.words + kColSlack, kBlock), kBlock, 0, ctx.stream>>>(
      next.cols.get(), next.words + kColSlack);
  RSB_LAUNCHED();
  k_new_fill<<<g, kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(), side, newidx.get(),
                                           L.orig.get(), L.gid.get(), next.chunk_ptr.get(),
                                           next.cols.get(), next.orig.get(), next.gid.get(),
                                           L.nrows);
  RSB_LAUNCHED();
  pack_level(next, ctx);
  level_tables(next, rpt, ctx);
}

void laplacian_apply_csr(const DevCsr &g, const double *d_x, double *d_y, Ctx &ctx) {
  Level L;
  std::vector<const DevCsr *> gs{&g};
  std::vector<int32_t> np{2};
  level0_from_csr(L, gs, np, 16, ctx);
  DevBuf<double> x(ctx, L.nrows), y(ctx, L.nrows);
  RSB_HIP(hipMemsetAsync(x.get(), 0, x.bytes(), ctx.stream));
  RSB_HIP(hipMemcpyAsync(x.get(), d_x, g.n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  k_spmv64<<<grid_for(L.nrows, kBlock), kBlock, 0, ctx.stream>>>(L.chunk_ptr.get(), L.cols.get(),
                                                                  x.get(), y.get(), L.nrows);
  RSB_LAUNCHED();
  RSB_HIP(hipMemcpyAsync(d_y, y.get(), g.n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
}

void partition_metrics(Level &L0, const int32_t *d_part, int32_t nparts_total,
                       const std::vector<int32_t> &part_offset, rsb_stats *st, Ctx &ctx) {
  if (!st || L0.nrows == 0) return;
  DevBuf<unsigned long long> acc(ctx, 5);
  RSB_HIP(hipMemsetAsync(acc.get(), 0, acc.bytes(), ctx.stream));
  DevBuf<int32_t> moff(ctx, part_offset.size()), poff(ctx, L0.nrows);
  RSB_HIP(hipMemcpyAsync(moff.get(), part_offset.data(), part_offset.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, ctx.stream));
  unsigned g = grid_for(L0.nrows, kBlock);
  k_row_part_offset<<<g, kBlock, 0, ctx.stream>>>(L0.orig.get(), L0.d_seg.get(), L0.nseg,
                                                  moff.get(), poff.get(), L0.nrows);
  RSB_LAUNCHED();
  const bool nb = nparts_total <= 16384;
  DevBuf<unsigned> bits;
  if (nb) {
    int64_t words = ((int64_t)nparts_total * nparts_total + 31) / 32;
    bits.alloc(ctx, words);
    RSB_HIP(hipMemsetAsync(bits.get(), 0, bits.bytes(), ctx.stream));
  }
  k_metrics<<<g, kBlock, 0, ctx.stream>>>(L0.chunk_ptr.get(), L0.cols.get(), L0.orig.get(), d_part,
                                          poff.get(), acc.get(), nb ? bits.get() : nullptr,
                                          nparts_total, L0.nrows);
  RSB_LAUNCHED();
  if (nb) {
    k_neighbor_counts<<<grid_for(nparts_total, 256), 256, 0, ctx.stream>>>(bits.get(), nparts_total,
                                                                           acc.get());
    RSB_LAUNCHED();
  }
  unsigned long long h[5];
  RSB_HIP(hipMemcpyAsync(h, acc.get(), sizeof(h), hipMemcpyDeviceToHost, ctx.stream));
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  if (h[4]) fail(RSB_EINTERNAL, std::to_string(h[4]) + " elements left without a part");
  st->edge_cut = (double)h[0];
  st->cut_pairs = (int64_t)h[1];
  st->max_neighbors = nb ? (int32_t)h[2] : -1;
  st->avg_neighbors = nb ? (double)h[3] / nparts_total : -1.0;
}

}  // namespace rsb
