// Lower bounds of the optimum cost of every instance of a batch, for the
// cost/LB quality metric:
//   sum    = total weight (the continuous bound when cost = capacity);
//   LB_cap = the least total >= sum that is a non-negative integer combination
//            of the capacities (the used bins' capacities must cover the
//            weight and are such a combination);
//   LB_big = items heavier than B_1/2 pairwise cannot share a bin, so each
//            needs its own bin of capacity >= its weight.
// LB_cap: with M = B_n, the representable totals congruent to r mod M are
// exactly dist[r] + t*M (t >= 0), where dist[r] is the least representable
// total in that class -- a shortest path over the M residues with one edge
// per capacity, relaxed in parallel until stable (LDS atomics on int64).
#include "device_common.h"
#include "kernels.h"

namespace vsbpp {
namespace {

constexpr int kMaxResidues = 8192;

__global__ void __launch_bounds__(256) k_bounds(int32_t num, const int32_t* w,
                                                const int64_t* item_off, const int32_t* caps,
                                                const int32_t* cap_off, int64_t* out) {
  __shared__ unsigned long long dist[kMaxResidues];
  __shared__ int64_t s_part[8];
  __shared__ int s_changed;
  const int inst = blockIdx.x;
  if (inst >= num) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t off = item_off[inst], m = item_off[inst + 1] - off;
  const int c0 = cap_off[inst], n = cap_off[inst + 1] - c0;
  if (m < 1 || n < 1 || n > kMaxTypes) {
    if (tid == 0) out[3 * (int64_t)inst] = out[3 * (int64_t)inst + 1] = out[3 * (int64_t)inst + 2] = -1;
    return;
  }
  int32_t cp[kMaxTypes];
#pragma unroll
  for (int k = 0; k < kMaxTypes; ++k) cp[k] = k < n ? caps[c0 + k] : 0;
  const int32_t b1 = cp[0];
  int64_t sum = 0, big = 0;
  for (int64_t j = tid; j < m; j += nt) {
    const int32_t x = w[off + j];
    sum += x;
    if (2 * (int64_t)x > b1) {
      int32_t c = b1;
#pragma unroll
      for (int k = 0; k < kMaxTypes; ++k)
        if (k < n && cp[k] >= x) c = cp[k];
      big += c;
    }
  }
  // block sums (fixed order)
  const int lane = lane_id(), wave = tid >> 6;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    sum += __shfl_xor(sum, d, kWave);
    big += __shfl_xor(big, d, kWave);
  }
  if (lane == 0) {
    s_part[wave] = sum;
    s_part[4 + wave] = big;
  }
  __syncthreads();
  sum = s_part[0] + s_part[1] + s_part[2] + s_part[3];
  big = s_part[4] + s_part[5] + s_part[6] + s_part[7];
  __syncthreads();
  const int32_t M = cp[n - 1];
  int64_t lbcap = sum;
  if (M <= kMaxResidues) {
    const unsigned long long INF = ~0ull;
    for (int r = tid; r < M; r += nt) dist[r] = r == 0 ? 0ull : INF;
    __syncthreads();
    for (;;) {
      if (tid == 0) s_changed = 0;
      __syncthreads();
      int changed = 0;
      for (int r = tid; r < M; r += nt) {
        const unsigned long long dr =
            __hip_atomic_load(&dist[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (dr == INF) continue;
        for (int k = 0; k < n - 1; ++k) {
          const int r2 = (int)((r + (int64_t)cp[k]) % M);
          const unsigned long long nv = dr + (unsigned long long)cp[k];
          if (nv < __hip_atomic_load(&dist[r2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            atomicMin(&dist[r2], nv);
            changed = 1;
          }
        }
      }
      if (changed) s_changed = 1;
      __syncthreads();
      const int any = s_changed;
      __syncthreads();
      if (!any) break;
    }
    int64_t best = INT64_MAX;
    for (int r = tid; r < M; r += nt) {
      const unsigned long long dr = dist[r];
      if (dr == INF) continue;
      int64_t v = (int64_t)dr;
      if (v < sum) v += ((sum - v + M - 1) / M) * (int64_t)M;
      best = v < best ? v : best;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t o = __shfl_xor(best, d, kWave);
      best = o < best ? o : best;
    }
    if (lane == 0) s_part[wave] = best;
    __syncthreads();
    lbcap = s_part[0];
    for (int i = 1; i < (nt >> 6); ++i) lbcap = s_part[i] < lbcap ? s_part[i] : lbcap;
  }
  if (tid == 0) {
    out[3 * (int64_t)inst] = sum;
    out[3 * (int64_t)inst + 1] = lbcap;
    out[3 * (int64_t)inst + 2] = big;
  }
}

}  // namespace

hipError_t launch_bounds(int32_t num, const int32_t* w, const int64_t* item_off,
                         const int32_t* caps, const int32_t* cap_off, int64_t* out,
                         hipStream_t s) {
  if (num <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bounds, dim3(num), dim3(256), 0, s, num, w, item_off, caps, cap_off, out);
  return hipGetLastError();
}

}  // namespace vsbpp
