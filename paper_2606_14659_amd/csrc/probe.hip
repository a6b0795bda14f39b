// probe.hip -- reference measurements for the roofline of the streaming
// kernels: what plain HBM streams reach on this GPU (read, copy, write), and
// the Laplacian SpMV of a level on its own (the Lanczos step fuses it with
// the projection, so it has no launch of its own there).
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "solver_dev.h"

namespace rsb {

namespace {

constexpr int kProbeBlock = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kProbeUnroll = 4;  // 16-byte loads in flight per thread

// Read stream: each thread sums 16-byte vectors (non-temporal loads) and the
// block writes one value, so the loads cannot be dropped.
__global__ __launch_bounds__(kProbeBlock) void k_hbm_read(const f32x4 *__restrict__ src,
                                                          int64_t n4, float *__restrict__ out) {
  __shared__ float red[kProbeBlock / kWave];
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  float acc = 0.f;
  for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
    f32x4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n4; i += stride) {
    const f32x4 v = __builtin_nontemporal_load(src + i);
    acc += (v.x + v.y) + (v.z + v.w);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < kProbeBlock / kWave; ++w) s += red[w];
    out[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kProbeBlock) void k_hbm_copy(const f32x4 *__restrict__ src,
                                                          f32x4 *__restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
    f32x4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(kProbeBlock) void k_hbm_write(f32x4 *__restrict__ dst, int64_t n4,
                                                           float v) {
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  const f32x4 w = {v, v, v, v};
  for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(w, dst + i);
}

__global__ void k_fill_f32(float *p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// y = L x on the level's sliced ELL (difference form; packed slices and
// their tiles' staged gathers where the level has them), one row per thread
// slot, tiles and block order as the Lanczos kernels use them.
template <typename T, int RPT>
__global__ __launch_bounds__(kBlock) void k_spmv_alone(const BlkDev *__restrict__ blk, SellRef m,
                                                       const T *__restrict__ x,
                                                       T *__restrict__ y) {
  __shared__ T xs[kStageCap];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const BlkDev b = blk[lb];
  const bool staged = tile_staged(m, b.row0);
  if (staged) {
    stage_copy(m, b.row0, x, xs, (int)threadIdx.x, kBlock);
    __syncthreads();
  }
  const TileRows<RPT> tr(b);
  T v[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    v[r] = staged ? lap_row<T, true>(m, x, xs, tr.row[r], x[tr.row[r]])
                  : lap_row<T, false>(m, x, nullptr, tr.row[r], x[tr.row[r]]);
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (tr.ok[r]) y[tr.row[r]] = v[r];
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    RSB_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      fail(RSB_EDEVICE, "hipEventCreate");
    }
  }
  ~EventPair() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  float ms(hipStream_t s) {
    RSB_HIP(hipEventRecord(b, s));
    RSB_HIP(hipEventSynchronize(b));
    float t = 0.f;
    RSB_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
};

template <typename T>
double spmv_alone_typed(const LevelView &L, int reps, Ctx &ctx) {
  DevBuf<T> x(ctx, (size_t)L.nrows), y(ctx, (size_t)L.nrows);
  if constexpr (sizeof(T) == 4) {
    k_fill_f32<<<1024, 256, 0, ctx.stream>>>((float *)x.get(), L.nrows, 1.0f);
  } else {
    fill_f64((double *)x.get(), L.nrows, 1.0, ctx);
  }
  RSB_LAUNCHED();
  double total = 0.0;
  auto launch = [&](auto rpt_tag) {
    constexpr int RPT = decltype(rpt_tag)::value;
    k_spmv_alone<T, RPT><<<L.nblk, kBlock, 0, ctx.stream>>>(
        L.blk, SellRef{L.chunk_ptr, L.cols, L.pk, L.pmeta, L.stage, L.lmeta}, x.get(), y.get());
  };
  auto run = [&]() {
    switch (L.rpt) {
      case 2: launch(std::integral_constant<int, 2>()); break;
      case 4: launch(std::integral_constant<int, 4>()); break;
      case 8: launch(std::integral_constant<int, 8>()); break;
      default: fail(RSB_EINTERNAL, "unsupported rows-per-thread");
    }
  };
  run();  // warm-up
  RSB_LAUNCHED();
  EventPair ev;
  RSB_HIP(hipEventRecord(ev.a, ctx.stream));
  for (int r = 0; r < reps; ++r) run();
  RSB_LAUNCHED();
  total = ev.ms(ctx.stream);
  return total * 1e3 / reps;
}

}  // namespace

double spmv_alone_us(const LevelView &L, bool fp32, int reps, Ctx &ctx) {
  if (L.nrows == 0 || L.nblk == 0 || L.gs.nv > 0) return 0.0;
  return fp32 ? spmv_alone_typed<float>(L, reps, ctx) : spmv_alone_typed<double>(L, reps, ctx);
}

__global__ void k_meta_words(int4 *meta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) meta[i] = make_int4(kPlainSlice, 0, 0, 0);
}

double spmv_words_us(const LevelView &L, bool fp32, int reps, Ctx &ctx) {
  if (L.nrows == 0 || L.nblk == 0 || L.gs.nv > 0 || L.nchunks == 0) return 0.0;
  // every slice marked as kept in words, no staging
  DevBuf<int4> meta(ctx, (size_t)L.nchunks);
  k_meta_words<<<(unsigned)((L.nchunks + 255) / 256), 256, 0, ctx.stream>>>(meta.get(), L.nchunks);
  RSB_LAUNCHED();
  LevelView w = L;
  w.pmeta = meta.get();
  w.stage = nullptr;
  w.lmeta = nullptr;
  return spmv_alone_us(w, fp32, reps, ctx);
}

double hbm_probe_gbs(int kind, int64_t bytes, int reps, int device, Ctx &ctx) {
  const int64_t n4 = bytes / 16;
  DevBuf<f32x4> src(ctx, (size_t)n4);
  DevBuf<f32x4> dst;
  if (kind == 1) dst.alloc(ctx, (size_t)n4);
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  const int grid = cus * 16;  // 16 workgroups of 256 threads per compute unit
  DevBuf<float> out(ctx, (size_t)grid);
  k_fill_f32<<<1024, 256, 0, ctx.stream>>>((float *)src.get(), n4 * 4, 1.0f);
  RSB_LAUNCHED();
  auto once = [&]() {
    if (kind == 0) k_hbm_read<<<grid, kProbeBlock, 0, ctx.stream>>>(src.get(), n4, out.get());
    else if (kind == 1) k_hbm_copy<<<grid, kProbeBlock, 0, ctx.stream>>>(src.get(), dst.get(), n4);
    else k_hbm_write<<<grid, kProbeBlock, 0, ctx.stream>>>(src.get(), n4, 2.0f);
  };
  once();  // warm-up
  RSB_LAUNCHED();
  EventPair ev;
  RSB_HIP(hipEventRecord(ev.a, ctx.stream));
  for (int r = 0; r < reps; ++r) once();
  RSB_LAUNCHED();
  const double ms = ev.ms(ctx.stream);
  const double moved = (double)n4 * 16.0 * (kind == 1 ? 2.0 : 1.0) * reps;
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  return moved / (ms * 1e-3) / 1e9;
}

}  // namespace rsb
