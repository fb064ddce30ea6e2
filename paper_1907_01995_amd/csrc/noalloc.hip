// noalloc.hip -- the partition draw for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): rac_permutation_noalloc runs the same bucket-sort kernels
// as rac_permutation, with their scratch in a fixed device array of this
// library instead of per-call allocations.
//
// The array `scratch` exists once per GPU for the life of the process.  Host
// code never uses its name as an address: on the first call on a device, with
// that device current, hipGetSymbolAddress gives the device address of that
// GPU's copy, which is kept per device and passed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rac_internal.h"
#include "racmb.h"

namespace rac {
namespace {

constexpr int64_t kNoAllocMaxN = RAC_NOALLOC_MAX_N;   // largest n (a power of two: buckets = n)
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// Scratch of one sort of up to kNoAllocMaxN keys: keys (8 B each), bucket counts,
// bucket offsets (one more), bucket fill counters, bucket members.
constexpr size_t kKeysOff = 0;
constexpr size_t kCountOff = align_up(kKeysOff + 8 * (size_t)kNoAllocMaxN);
constexpr size_t kOffsetOff = align_up(kCountOff + 4 * (size_t)kNoAllocMaxN);
constexpr size_t kFillOff = align_up(kOffsetOff + 4 * ((size_t)kNoAllocMaxN + 1));
constexpr size_t kMembersOff = align_up(kFillOff + 4 * (size_t)kNoAllocMaxN);
constexpr size_t kScratchBytes = align_up(kMembersOff + 4 * (size_t)kNoAllocMaxN);
static_assert(kScratchBytes == RAC_NOALLOC_SCRATCH_BYTES, "header states the scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device).
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

__global__ void __launch_bounds__(256) k_zero_u32(uint32_t* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0u;
}

}  // namespace
}  // namespace rac

extern "C" rac_status rac_permutation_noalloc(uint64_t seed, uint64_t instance, int64_t iter, int64_t n,
                                              int32_t* perm, void* stream) {
  using namespace rac;
  if (n < 1 || n > kNoAllocMaxN || !perm || iter < 0) return RAC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RAC_ERR_DEVICE;
  void* base = nullptr;
  if (scratch_address(dev, &base) != hipSuccess) return RAC_ERR_DEVICE;
  unsigned char* b = (unsigned char*)base;
  PermWork w{};
  int64_t nb = 1;
  int lg = 0;
  while (nb < n) { nb <<= 1; ++lg; }
  w.nb = nb;
  w.log2nb = lg;
  w.keys = (uint64_t*)(b + kKeysOff);
  w.count = (uint32_t*)(b + kCountOff);
  w.offset = (uint32_t*)(b + kOffsetOff);
  w.fill = (uint32_t*)(b + kFillOff);
  w.members = (int32_t*)(b + kMembersOff);
  hipStream_t st = (hipStream_t)stream;
  // the bucket counters start at zero (a fill kernel, so that the call can be captured)
  const unsigned grid = (unsigned)((nb + 255) / 256);
  k_zero_u32<<<grid, 256, 0, st>>>(w.count, nb);
  k_zero_u32<<<grid, 256, 0, st>>>(w.fill, nb);
  if (hipGetLastError() != hipSuccess) return RAC_ERR_DEVICE;
  return launch_permutations(seed, instance, iter, 1, n, w, perm, st) == hipSuccess ? RAC_OK : RAC_ERR_DEVICE;
}
