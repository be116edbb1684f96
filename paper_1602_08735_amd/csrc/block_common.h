// Workgroup-level helpers shared by kernels that give one instance to a
// whole workgroup: instance validation and the next instance of a
// workgroup.
#pragma once
#include "device_common.h"
#include "kernels.h"

namespace vsbpp {
namespace {

// Block-level validation of instance `inst`.  Returns 0 or an error code
// (uniform across the block) and loads the capacities into s_caps.
__device__ int validate_block(const BatchArgs& a, int inst, int64_t off, int m, int c0, int n,
                              int32_t* s_caps, int* s_flag) {
  if ((int64_t)m < 1 || m > a.max_items || n < 1 || n > kMaxTypes || n > a.max_types)
    return kErrSize;
  const int tid = threadIdx.x;
  if (tid < kMaxTypes) s_caps[tid] = tid < n ? a.caps[c0 + tid] : 0;
  __syncthreads();
  int bad = 0;
  if (tid < n) {
    const int32_t c = s_caps[tid];
    if (c <= 0 || (tid > 0 && c >= s_caps[tid - 1])) bad = 1;
  }
  if (__syncthreads_or(bad)) return kErrCaps;
  const int32_t B1 = s_caps[0];
  if (B1 > a.max_cap) return kErrSize;
  int badw = 0, bado = 0;
  for (int q = tid; q < m; q += blockDim.x) {
    const int32_t w = a.w[off + q];
    badw |= (w < 1 || w > B1);
    if (a.order) {
      const int32_t it = a.order[off + q];
      bado |= ((unsigned)it >= (unsigned)m);
    }
  }
  if (__syncthreads_or(badw)) return kErrWeight;
  if (__syncthreads_or(bado)) return kErrOption;
  (void)inst;
  (void)s_flag;
  return 0;
}

// next instance slot of this workgroup: static stride, or the global work
// counter in persistent mode (thread 0 takes it and broadcasts through LDS)
__device__ __forceinline__ int next_slot(const BatchArgs& a, int* cursor, int* s_slot) {
  if (a.queue) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(a.queue, 1);
    __syncthreads();
    const int v = *s_slot;
    __syncthreads();
    return v;
  }
  const int v = *cursor;
  *cursor += gridDim.x;
  return v;
}

}  // namespace
}  // namespace vsbpp
