// Learned scorer: kernels shared by the C-ABI host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace vsbpp {

// parameters in the flat order w1 b1 w2 b2 w3 b3 for n_out outputs
__host__ __device__ inline int param_count(int nout) { return 1024 + 64 + 4096 + 64 + 65 * nout; }

__device__ void write_param(vsbpp_model* mdl, int p, float w);

hipError_t launch_labels(const int64_t* cost, const int32_t* info, int32_t num, int32_t n,
                         int32_t* labels, int64_t* values, hipStream_t s);
size_t train_lds_bytes();
// forward + backward of the minibatch into grad[param_count(nout)];
// waves: a multiple of 4
hipError_t launch_train(const vsbpp_model* mdl, const float* X, const int32_t* mask,
                        const int32_t* label, const int32_t* idx, int32_t batch, int32_t waves,
                        int32_t nout, float* partial, float* loss_part, float* grad,
                        hipStream_t s);
hipError_t launch_adam(float* master, float* m1, float* m2, const float* grad, int32_t np,
                       float lr, float beta1, float beta2, float eps, int step, vsbpp_model* mdl,
                       hipStream_t s);
hipError_t launch_publish(const float* master, int32_t np, vsbpp_model* mdl, hipStream_t s);

}  // namespace vsbpp
