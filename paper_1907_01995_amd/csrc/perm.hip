// perm.hip -- the random partition of Eq.(3) ("randomly, without replacement,
// assemble the variables into p blocks") on the GPU.
//
// Variable j of iteration k gets the 64-bit key
//   key_j = mix(mix(mix(seed + G(inst+1)) + G(k+1)) + G(j+1))      (SplitMix64 chain)
// and the permutation lists the variables in ascending (key, j) order; block i
// is positions [floor(i n/p), floor((i+1) n/p)).  Keys are uniform, so a
// distribution sort is used instead of a comparison sort: the top log2(nb) bits
// of the key pick one of nb >= n buckets (about one key per bucket), a scan
// gives each bucket its output range, and each variable's position inside its
// bucket is its rank among the bucket's members under (key, j).  The result is
// the exact lexicographic order, independent of the atomic arrival order.
// All iterations of a chunk are sorted by the same four launches.
#include "rac_internal.h"

namespace rac {
namespace {

__device__ __forceinline__ uint32_t bucket_of(uint64_t key, int log2nb) {
  return log2nb == 0 ? 0u : (uint32_t)(key >> (64 - log2nb));
}

__global__ void __launch_bounds__(256) k_perm_keys(uint64_t seed, uint64_t inst, int64_t iter0,
                                                   int64_t n, int64_t nb, int log2nb,
                                                   uint64_t* keys, uint32_t* count) {
  const int64_t t = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint64_t key = perm_key(seed, inst, (uint64_t)(iter0 + t), (uint64_t)j);
  keys[t * n + j] = key;
  atomicAdd(&count[t * nb + bucket_of(key, log2nb)], 1u);
}

// Exclusive scan of the bucket counts of one iteration (one workgroup of 1024
// threads per iteration); re-zeroes the counts for the next chunk.
__global__ void __launch_bounds__(1024) k_perm_scan(int64_t nb, uint32_t* count, uint32_t* offset) {
  const int64_t t = blockIdx.x;
  uint32_t* cnt = count + t * nb;
  uint32_t* off = offset + t * (nb + 1);
  __shared__ uint32_t part[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += cnt[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {   // Hillis-Steele inclusive scan
    uint32_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x == 0 ? 0u : part[threadIdx.x - 1];
  for (int64_t i = lo; i < hi; ++i) {
    off[i] = run;
    run += cnt[i];
    cnt[i] = 0u;
  }
  if (threadIdx.x == 1023) off[nb] = part[1023];
}

__global__ void __launch_bounds__(256) k_perm_scatter(int64_t n, int64_t nb, int log2nb,
                                                      const uint64_t* keys, const uint32_t* offset,
                                                      uint32_t* fill, int32_t* members) {
  const int64_t t = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t b = bucket_of(keys[t * n + j], log2nb);
  uint32_t slot = atomicAdd(&fill[t * nb + b], 1u);
  members[t * n + offset[t * (nb + 1) + b] + slot] = (int32_t)j;
}

__global__ void __launch_bounds__(256) k_perm_rank(int64_t n, int64_t nb, int log2nb,
                                                   const uint64_t* keys, const uint32_t* offset,
                                                   uint32_t* fill, const int32_t* members,
                                                   int32_t* perm) {
  const int64_t t = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t* kt = keys + t * n;
  const uint64_t kj = kt[j];
  const uint32_t b = bucket_of(kj, log2nb);
  const uint32_t lo = offset[t * (nb + 1) + b], hi = offset[t * (nb + 1) + b + 1];
  uint32_t rank = 0;
  for (uint32_t q = lo; q < hi; ++q) {
    int32_t i = members[t * n + q];
    uint64_t ki = kt[i];
    rank += (ki < kj || (ki == kj && i < (int32_t)j)) ? 1u : 0u;
  }
  perm[t * n + lo + rank] = (int32_t)j;
  fill[t * nb + b] = 0u;   // every member writes the same zero: ready for the next chunk
}

}  // namespace

hipError_t launch_permutations(uint64_t seed, uint64_t inst, int64_t iter0, int64_t T, int64_t n,
                               const PermWork& w, int32_t* perm, hipStream_t st) {
  if (T <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)T);
  k_perm_keys<<<grid, 256, 0, st>>>(seed, inst, iter0, n, w.nb, w.log2nb, w.keys, w.count);
  k_perm_scan<<<(unsigned)T, 1024, 0, st>>>(w.nb, w.count, w.offset);
  k_perm_scatter<<<grid, 256, 0, st>>>(n, w.nb, w.log2nb, w.keys, w.offset, w.fill, w.members);
  k_perm_rank<<<grid, 256, 0, st>>>(n, w.nb, w.log2nb, w.keys, w.offset, w.fill, w.members, perm);
  return hipGetLastError();
}

}  // namespace rac
