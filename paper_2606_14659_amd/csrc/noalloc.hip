// noalloc.hip -- the fixed device region behind rsb_partition_noalloc, the
// partition entry point for callers that cannot allocate device memory.
//
// The region is one file-scope device array; every GPU the library runs on
// holds its own copy at its own address for the life of the process.  In
// host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device, with that device current, and that
// address is what the library hands to kernels and copies.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rsb {

namespace {

constexpr size_t kScratchBytes = (size_t)RSB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

NoallocRegion g_regions[kMaxDevices];
std::once_flag g_once[kMaxDevices];

}  // namespace

NoallocRegion &noalloc_region(int device) {
  if (device < 0 || device >= kMaxDevices) fail(RSB_EINVAL, "device ordinal out of range");
  NoallocRegion &r = g_regions[device];
  RSB_HIP(hipSetDevice(device));
  std::call_once(g_once[device], [&] {
    void *ptr = nullptr;
    r.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (r.err == hipSuccess) {
      r.ptr = ptr;
      r.bytes = kScratchBytes;
    }
  });
  if (r.err != hipSuccess)
    fail(RSB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(r.err));
  return r;
}

}  // namespace rsb
