// common.h -- shared host/device helpers of the gfx950 RSB library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rsb.h"

namespace rsb {

constexpr int kWave = 64;    // CDNA wavefront width
constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels
constexpr int kMaxM = 250;   // largest Lanczos cycle length
constexpr int kMaxKeep = 16; // most Ritz pairs kept by a thick restart
constexpr int kMaxFullProj = 32;  // most CG directions kept by full projection
constexpr int kGroup = 32;   // least blocks per first-level reduction group
constexpr int kSlotGroup = 16;  // ELL slots a row reads at once (unconditional loads)
// zero words after the last slice so that a row may read a whole slot group
constexpr int64_t kColSlack = (int64_t)kSlotGroup * 64;

// ---------------------------------------------------------------------------
// Errors: internal code throws, the C entry points convert to return codes.
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Error{code, msg}; }

#define RSB_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      ::rsb::fail(e_ == hipErrorOutOfMemory ? RSB_ENOMEM : RSB_EDEVICE,                      \
                  std::string(#call) + ": " + hipGetErrorString(e_));                        \
  } while (0)

#define RSB_LAUNCHED()                                                                       \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess)                                                                    \
      ::rsb::fail(RSB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_));      \
    ::rsb::fault_point(false);                                                               \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory from the stream-ordered pool, freed when the owner dies.
// ---------------------------------------------------------------------------
// Failure injection for tests of the error paths: the environment variable
// RSB_FAULT_INJECT = "alloc:N" or "launch:N" makes the N-th device allocation,
// or the N-th launch check made outside graph capture, of a call fail with
// RSB_EDEVICE.  Read when a call sets up its context.
struct FaultPlan {
  int64_t alloc_at = 0, launch_at = 0;
  int64_t allocs = 0, launches = 0;
  hipStream_t stream = nullptr;
};
inline FaultPlan *&fault_plan() {
  static thread_local FaultPlan *plan = nullptr;
  return plan;
}
inline void fault_point(bool alloc) {
  FaultPlan *f = fault_plan();
  if (!f || (alloc ? f->alloc_at : f->launch_at) <= 0) return;
  // never inside a stream capture: the capture must be ended by its owner
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (f->stream && hipStreamIsCapturing(f->stream, &cs) == hipSuccess &&
      cs != hipStreamCaptureStatusNone)
    return;
  if (alloc && ++f->allocs == f->alloc_at)
    fail(RSB_EDEVICE, "injected allocation failure (RSB_FAULT_INJECT)");
  if (!alloc && ++f->launches == f->launch_at)
    fail(RSB_EDEVICE, "injected launch failure (RSB_FAULT_INJECT)");
}

// Device scratch carved from one fixed region instead of the allocator (the
// entry point for callers that cannot allocate).  First fit over a free list
// with coalescing; offsets are aligned to 256 bytes.  Every buffer of a call
// lives on the call's one stream, so a region freed by the host may be handed
// out again at once: later work on the stream runs after the earlier work.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t in_use = 0, peak = 0;
  std::map<size_t, size_t> free_list;  // offset -> bytes
  void reset(void *b, size_t bytes) {
    base = (char *)b;
    cap = bytes;
    in_use = peak = 0;
    free_list.clear();
    free_list[0] = bytes;
  }
  static size_t rounded(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~size_t(255); }
  void *take(size_t bytes) {
    const size_t need = rounded(bytes);
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_list.erase(it);
      if (len > need) free_list[off + need] = len - need;
      in_use += need;
      peak = std::max(peak, in_use);
      return base + off;
    }
    return nullptr;
  }
  void give(void *p, size_t bytes) {
    const size_t len = rounded(bytes);
    size_t off = (size_t)((char *)p - base);
    size_t end = off + len;
    in_use -= len;
    auto next = free_list.lower_bound(off);
    if (next != free_list.end() && next->first == end) {
      end += next->second;
      next = free_list.erase(next);
    }
    if (next != free_list.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        free_list.erase(prev);
      }
    }
    free_list[off] = end - off;
  }
};

// Idle device blocks of calls that have ended, per device.  A call takes
// from here before it asks the pool: each hipMallocAsync and hipFreeAsync
// holds the host for about 0.1 ms, and a partition makes hundreds of them.
// Blocks only enter after their call has synchronised its stream, so any
// later call, on any stream, may use them.  Beyond kBlockCacheMax bytes the
// largest go back to the pool.
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void *> blocks;
  size_t bytes = 0;
};
constexpr size_t kBlockCacheMax = size_t(32) << 30;
inline BlockCache &block_cache(int device) {
  static BlockCache caches[64];
  return caches[(unsigned)device % 64u];
}

// Takes a block of at least `bytes` and at most twice that from `m`, or
// returns null; *cap receives its size.
inline void *take_block(std::multimap<size_t, void *> &m, size_t bytes, size_t *cap) {
  auto it = m.lower_bound(bytes);
  if (it == m.end() || it->first > 2 * bytes) return nullptr;
  void *q = it->second;
  *cap = it->first;
  m.erase(it);
  return q;
}

struct Ctx {
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created for a call that passed the null stream
  int device = 0;
  int64_t limit = 0;  // 0 = unlimited
  int64_t in_use = 0;
  int64_t peak = 0;
  int verbose = 0;
  std::vector<std::string> tuned;  // tile classes timed during this call
  int64_t fp64_level_steps = 0;    // mixed precision: level steps continued with FP64 directions
  int pack = 1;  // 0: 32-bit words only; 1: packed copy of the slices that fit; 2: and
                 // their tiles' gathers staged in LDS
  Arena *arena = nullptr;          // non-null: device scratch comes from this region only
  FaultPlan fault;
  // device blocks released during the call, by size: a later allocation on
  // the same stream takes one (stream order makes that safe); at the end of
  // the call, with its work done, they join the device's block cache
  // (returning memory that captured graphs used can hold the host while the
  // queue runs dry)
  std::multimap<size_t, void *> spare;
  Ctx() = default;
  Ctx(const Ctx &) = delete;
  Ctx &operator=(const Ctx &) = delete;
  ~Ctx() {
    if (fault_plan() == &fault) fault_plan() = nullptr;
    if (!spare.empty()) {
      (void)hipStreamSynchronize(stream);
      BlockCache &bc = block_cache(device);
      std::lock_guard<std::mutex> lock(bc.mu);
      for (auto &kv : spare) {
        bc.blocks.emplace(kv.first, kv.second);
        bc.bytes += kv.first;
      }
      spare.clear();
      while (bc.bytes > kBlockCacheMax && !bc.blocks.empty()) {
        auto it = std::prev(bc.blocks.end());
        (void)hipFreeAsync(it->second, stream);
        bc.bytes -= it->first;
        bc.blocks.erase(it);
      }
      (void)hipStreamSynchronize(stream);
    }
    if (own_stream && stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
  }
};

template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  size_t cap = 0;  // bytes of the block held
  Ctx *ctx = nullptr;
  DevBuf() = default;
  DevBuf(Ctx &c, size_t count) { alloc(c, count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), cap(o.cap), ctx(o.ctx) {
    o.p = nullptr; o.n = 0; o.cap = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; cap = o.cap; ctx = o.ctx;
      o.p = nullptr; o.n = 0; o.cap = 0;
    }
    return *this;
  }
  void alloc(Ctx &c, size_t count) {
    release();
    ctx = &c;
    n = count;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    fault_point(true);
    if (c.limit > 0 && c.in_use + (int64_t)bytes > c.limit)
      fail(RSB_ENOMEM, "device_mem_limit exceeded: need " + std::to_string(c.in_use + bytes) +
                           " bytes, limit " + std::to_string(c.limit));
    if (c.arena) {
      cap = bytes;
      p = (T *)c.arena->take(bytes);
      if (!p)
        fail(RSB_ENOMEM, "the problem needs more device scratch than the fixed region of " +
                             std::to_string(c.arena->cap) + " bytes (" +
                             std::to_string(c.arena->in_use) + " in use, " +
                             std::to_string(bytes) + " more asked for)");
      c.in_use += bytes;
      c.peak = std::max(c.peak, c.in_use);
      return;
    }
    // a block released earlier in the call, or by a call that has ended, at
    // least this size and at most twice it
    p = (T *)take_block(c.spare, bytes, &cap);
    if (!p) {
      BlockCache &bc = block_cache(c.device);
      std::lock_guard<std::mutex> lock(bc.mu);
      p = (T *)take_block(bc.blocks, bytes, &cap);
      if (p) bc.bytes -= cap;
    }
    if (p) {
      c.in_use += bytes;
      c.peak = std::max(c.peak, c.in_use);
      return;
    }
    cap = bytes;
    hipError_t e = hipMallocAsync((void **)&p, bytes, c.stream);
    if (e == hipErrorOutOfMemory) {
      // the kept blocks go back to the pool and the allocation is tried again
      (void)hipGetLastError();
      (void)hipStreamSynchronize(c.stream);
      for (auto &kv : c.spare) (void)hipFreeAsync(kv.second, c.stream);
      c.spare.clear();
      {
        BlockCache &bc = block_cache(c.device);
        std::lock_guard<std::mutex> lock(bc.mu);
        for (auto &kv : bc.blocks) (void)hipFreeAsync(kv.second, c.stream);
        bc.blocks.clear();
        bc.bytes = 0;
      }
      (void)hipStreamSynchronize(c.stream);
      e = hipMallocAsync((void **)&p, bytes, c.stream);
    }
    if (e != hipSuccess) {
      p = nullptr;
      fail(e == hipErrorOutOfMemory ? RSB_ENOMEM : RSB_EDEVICE,
           std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    c.in_use += bytes;
    c.peak = std::max(c.peak, c.in_use);
  }
  void release() {
    if (p) {
      if (ctx->arena) ctx->arena->give(p, cap);
      else ctx->spare.emplace(cap, p);
      ctx->in_use -= std::max<size_t>(n, 1) * sizeof(T);
      p = nullptr;
    }
    n = 0;
    cap = 0;
  }
  ~DevBuf() { release(); }
  T *get() const { return p; }
  size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// Packed column word of the sliced-ELL Laplacian: (column << 4) | weight.
// Weight 0 marks a padding slot; padding words are 0 (column 0, weight 0).
// ---------------------------------------------------------------------------
constexpr int kColShift = 4;
constexpr uint32_t kWeightMask = 15u;
constexpr int64_t kMaxRows = int64_t(1) << 28;

__host__ __device__ inline uint32_t pack_colw(uint32_t col, uint32_t w) {
  return (col << kColShift) | w;
}
__host__ __device__ inline uint32_t colw_col(uint32_t word) { return word >> kColShift; }
__host__ __device__ inline uint32_t colw_wt(uint32_t word) { return word & kWeightMask; }

// ---------------------------------------------------------------------------
// Packed copy of a slice (16-bit slot entries, two per word: slot 2p in the
// low half of word p, slot 2p + 1 in the high half).  A slice's deltas
// (column - row) are covered by at most kPackClusters windows of
// 2^kPackOffBits, window b starting at base b (ascending); an entry holds
// (weight << 12) | (b << 10) | (delta - base b), 0 for a padding slot.  Slice
// c starts at word (chunk_ptr[c] + 64 c) / 2 (room for ceil(width / 2) words
// per row).  A slice whose deltas need more windows keeps only its 32-bit
// words; its meta.x is kPlainSlice.
// ---------------------------------------------------------------------------
constexpr int kPackOffBits = 10;
constexpr int kPackClusters = 4;
constexpr int32_t kPlainSlice = INT32_MIN;

__host__ __device__ inline int64_t packed_slice_word(int64_t chunk_word, int64_t chunk) {
  return (chunk_word + 64 * chunk) >> 1;
}

// Gathers staged in LDS: a tile's launch first copies the intervals of the
// gathered vector that its packed slices reach (at most kStageMaxInt of them,
// kStageCap values together) into LDS; the rows then read their neighbours
// there.  Filled per tile layout (rows per thread) at its first slice.
constexpr int kStageMaxInt = 6;
constexpr int kStageCap = 4864;
constexpr int kStageGap = 64;  // ranges closer than this share an interval

struct TileStage {
  int32_t nint;   // intervals; 0 = the tile reads its neighbours from global memory
  int32_t total;  // values staged
  int32_t lo[kStageMaxInt], len[kStageMaxInt], off[kStageMaxInt];
};

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Workgroup ids are dispatched round-robin over the 8 XCDs of the chip.
// Map them so that each XCD works on one contiguous range of logical blocks
// (its L2 then sees one contiguous slice of rows and their neighbours).
__device__ inline int xcd_block(int b, int nb) {
  int x = b & 7, i = b >> 3;
  int q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum of NV values over a 256-thread block; result valid in thread t < NV
// for value t (returned), fixed summation order.
template <int NV>
__device__ inline void block_sum_multi(double (&v)[NV], double *lds /* [4*NV] */) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
  }
  __syncthreads();
}

}  // namespace rsb
