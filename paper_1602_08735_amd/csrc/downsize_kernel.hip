// Downsizing pass over packed outputs: a bin costs its capacity, so once a
// packing is fixed every bin can take the smallest type whose capacity holds
// its load (with the LARGEST type rule every bin opens at B_1 whatever it
// ends up holding).  Bins, ids and the item assignment stay; the bin types
// and the cost are rewritten.
//
// One workgroup per instance (a static stride over the batch) owns that
// instance's bins.  The bin loads are summed with atomics, in LDS when the
// batch's largest instance fits (max_items loads), else in the instance's
// bin-type entries in global memory.  Only the owning workgroup touches
// them, so workgroup-scope atomics suffice; the global entries are read back
// with atomic loads after a workgroup fence and barrier.  (Device-scope
// atomics would be performed beyond the per-XCD L2 and cost a memory round
// trip each.)  A load never exceeds B_1 <= 2^31 - 1.
#include "device_common.h"
#include "host_internal.h"
#include "kernels.h"

namespace vsbpp {
namespace {

constexpr int kBlock = 256;

template <bool LDS>
__global__ void __launch_bounds__(kBlock) k_downsize(BatchArgs a) {
  extern __shared__ int32_t s_load[];
  __shared__ int32_t s_caps[kMaxTypes];
  __shared__ int64_t s_part[kBlock / kWave];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int inst = blockIdx.x; inst < a.num; inst += gridDim.x) {
    const int nb = a.nbins[inst];
    if (nb < 1) continue;  // an instance that failed its checks: left as it is
    const int64_t off = a.item_off[inst], m = a.item_off[inst + 1] - off;
    const int c0 = a.cap_off[inst], n = a.cap_off[inst + 1] - c0;
    if (tid < kMaxTypes) s_caps[tid] = tid < n ? a.caps[c0 + tid] : 0;
    int32_t* load = LDS ? s_load : a.types + off;
    for (int b = tid; b < nb; b += nt) {
      if constexpr (LDS) load[b] = 0;
      else __hip_atomic_store(load + b, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if constexpr (!LDS) __threadfence_block();
    __syncthreads();
    for (int64_t j = tid; j < m; j += nt)
      __hip_atomic_fetch_add(load + a.assign[off + j], a.w[off + j], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    if constexpr (!LDS) __threadfence_block();
    __syncthreads();
    int64_t c = 0;
    for (int b = tid; b < nb; b += nt) {
      const int32_t l =
          __hip_atomic_load(load + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      int t = 0;
      for (int k = 1; k < n; ++k)
        if (s_caps[k] >= l) t = k;
      a.types[off + b] = t;
      c += s_caps[t];
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) c += __shfl_xor(c, d, kWave);
    if ((tid & (kWave - 1)) == 0) s_part[tid >> 6] = c;
    __syncthreads();
    if (tid == 0) {
      int64_t total = 0;
      for (int w = 0; w < nt / kWave; ++w) total += s_part[w];
      a.cost[inst] = total;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_downsize(const BatchArgs& a, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  const size_t lds = sizeof(int32_t) * (size_t)a.max_items;
  const int cap = 8 * device_info().cus;
  const int grid = a.num < cap ? a.num : cap;
  if (lds <= 32768) {
    hipLaunchKernelGGL(k_downsize<true>, dim3(grid), dim3(kBlock), lds, s, a);
  } else {
    hipLaunchKernelGGL(k_downsize<false>, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace vsbpp
