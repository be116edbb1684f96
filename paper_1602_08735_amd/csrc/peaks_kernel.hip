// Achievable on-chip peaks of the device, measured by two stream kernels:
// LDS read bandwidth (16-byte reads at unit lane stride, conflict-free) and
// 32-bit integer VALU throughput (independent add/xor/min chains).  The
// roofline fractions of the packing kernels are taken against these, next
// to the published peaks.
#include <hip/hip_runtime.h>

#include "../../include/vsbpp.h"
#include "host_internal.h"
#include "kernels.h"

namespace vsbpp {
namespace {

constexpr int kLdsWords = 2048;  // uint4 words: 32 KB per workgroup
constexpr int kLdsUnroll = 8;

__global__ void __launch_bounds__(256) k_lds_stream(uint32_t* out, int iters) {
  __shared__ uint4 buf[kLdsWords];
  const int tid = threadIdx.x;
  for (int i = tid; i < kLdsWords; i += 256)
    buf[i] = make_uint4(i * 4u, i * 4u + 1u, i * 4u + 2u, i * 4u + 3u);
  __syncthreads();
  uint32_t acc = 0;
  int idx = tid;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kLdsUnroll; ++j) {
      const uint4 v = buf[(idx + j * 256) & (kLdsWords - 1)];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    idx = (idx + kLdsUnroll * 256 + (int)(acc & 1u)) & (kLdsWords - 1);
  }
  if (acc == 0x9e3779b9u) out[blockIdx.x] = acc;  // keeps the reads live
}

constexpr int kValuChains = 8;
constexpr int kValuUnroll = 16;

// per iteration and lane: kValuChains x kValuUnroll x 3 ops (add, xor, min)
__global__ void __launch_bounds__(256) k_valu_int(uint32_t* out, int iters, uint32_t seed) {
  uint32_t c[kValuChains];
#pragma unroll
  for (int i = 0; i < kValuChains; ++i) c[i] = seed * (threadIdx.x + 1u) + i;
  const uint32_t k = seed | 1u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kValuUnroll; ++u) {
#pragma unroll
      for (int i = 0; i < kValuChains; ++i) c[i] = min(c[i] + k, c[i] ^ 0x5bd1e995u);
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kValuChains; ++i) r ^= c[i];
  if (r == 0x9e3779b9u) out[blockIdx.x] = r;
}

template <typename F>
hipError_t time_launch(F launch, hipStream_t s, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e == hipSuccess) *ms /= 5.0f;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

}  // namespace
}  // namespace vsbpp

extern "C" int32_t vsbpp_measure_peaks(double* out) {
  using namespace vsbpp;
  if (!out) return VSBPP_E_NULL;
  if (!device_info().ok) return VSBPP_E_DEVICE;
  const int cus = device_info().cus;
  uint32_t* sink = nullptr;
  if (hipMalloc(&sink, sizeof(uint32_t) * 65536) != hipSuccess) {
    (void)hipGetLastError();
    return VSBPP_E_NOMEM;
  }
  hipStream_t s = nullptr;
  const int lds_blocks = cus * 16, lds_iters = 4096;
  const int valu_blocks = cus * 16, valu_iters = 2048;
  float t_lds = 0.0f, t_valu = 0.0f;
  hipError_t e = time_launch(
      [&]() {
        hipLaunchKernelGGL(k_lds_stream, dim3(lds_blocks), dim3(256), 0, s, sink, lds_iters);
        return hipGetLastError();
      },
      s, &t_lds);
  if (e == hipSuccess)
    e = time_launch(
        [&]() {
          hipLaunchKernelGGL(k_valu_int, dim3(valu_blocks), dim3(256), 0, s, sink, valu_iters,
                             0x2545F491u);
          return hipGetLastError();
        },
        s, &t_valu);
  (void)hipFree(sink);
  if (e != hipSuccess) {
    set_last_error("vsbpp_measure_peaks", e);
    (void)hipGetLastError();
    return VSBPP_E_DEVICE;
  }
  const double lds_bytes = (double)lds_blocks * 256.0 * lds_iters * kLdsUnroll * 16.0;
  const double valu_ops =
      (double)valu_blocks * 256.0 * valu_iters * kValuUnroll * kValuChains * 3.0;
  out[0] = lds_bytes / (t_lds * 1e-3);
  out[1] = valu_ops / (t_valu * 1e-3);
  return VSBPP_OK;
}
