// scan.hip -- exclusive prefix sums on the device (int32/int64 in, int64 out).
//
// Three phases: per-tile sums, a scan of the tile sums (recursive), and a
// per-tile scan that adds the tile offset.  Tiles are 256 threads x 16 items.
#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

constexpr int kScanIpt = 16;
constexpr int kScanTile = kBlock * kScanIpt;

template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const Tin *__restrict__ in, int64_t n,
                                                      int64_t *__restrict__ sums) {
  __shared__ int64_t lds[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanIpt; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += lds[w];
    sums[blockIdx.x] = t;
  }
}

// Exclusive scan of one tile (blocked: thread t owns items t*16 .. t*16+15),
// plus the tile's offset.  Writes n outputs; if total != nullptr the last
// tile also writes the grand total there.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const Tin *__restrict__ in, int64_t n,
                                                      const int64_t *__restrict__ offsets,
                                                      int64_t *__restrict__ out,
                                                      int64_t *__restrict__ total) {
  __shared__ int64_t lds[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  int64_t v[kScanIpt];
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanIpt; ++r) {
    int64_t i = base + r;
    v[r] = (i < n) ? (int64_t)in[i] : 0;
    s += v[r];
  }
  // inclusive scan of the per-thread sums across the block
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int64_t add = (threadIdx.x >= (unsigned)off) ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = lds[threadIdx.x] - s + (offsets ? offsets[blockIdx.x] : 0);
#pragma unroll
  for (int r = 0; r < kScanIpt; ++r) {
    int64_t i = base + r;
    if (i < n) out[i] = run;
    run += v[r];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) *total = run;
}

template <typename Tin>
void scan_impl(const Tin *in, int64_t n, int64_t *out, int64_t *total, Ctx &ctx) {
  if (n <= 0) {
    if (total) RSB_HIP(hipMemsetAsync(total, 0, sizeof(int64_t), ctx.stream));
    return;
  }
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    k_tile_scan<Tin><<<1, kBlock, 0, ctx.stream>>>(in, n, nullptr, out, total);
    RSB_LAUNCHED();
    return;
  }
  DevBuf<int64_t> sums(ctx, tiles), offs(ctx, tiles);
  k_tile_sums<Tin><<<(unsigned)tiles, kBlock, 0, ctx.stream>>>(in, n, sums.get());
  RSB_LAUNCHED();
  scan_impl<int64_t>(sums.get(), tiles, offs.get(), nullptr, ctx);
  k_tile_scan<Tin><<<(unsigned)tiles, kBlock, 0, ctx.stream>>>(in, n, offs.get(), out, total);
  RSB_LAUNCHED();
}

}  // namespace

void scan_exclusive(const int64_t *in, int64_t n, int64_t *out, int64_t *total, Ctx &ctx) {
  scan_impl<int64_t>(in, n, out, total, ctx);
}
void scan_exclusive(const int32_t *in, int64_t n, int64_t *out, int64_t *total, Ctx &ctx) {
  scan_impl<int32_t>(in, n, out, total, ctx);
}

}  // namespace rsb
