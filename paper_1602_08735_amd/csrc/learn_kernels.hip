// Learned bin-type scorer: depth-2 lookahead labels from rollout costs, and
// training of the MLP 16 -> 64 -> 64 -> n (bf16 working weights, fp32 master
// weights and accumulation, masked softmax cross-entropy, Adam).
//
// Training layout: a wavefront streams minibatch samples; lane l owns hidden
// unit l of both layers (and output l < n).  Forward values are fp32
// fused-multiply-add chains in index order.  Every wavefront accumulates its
// gradient in registers and writes one partial vector; a second kernel sums
// the partials in wavefront order, so a step is deterministic.
#include "device_common.h"
#include "learn.h"

namespace vsbpp {
namespace {

__device__ __forceinline__ float bf16f(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// fp32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void k_labels(const int64_t* cost, const int32_t* info, int32_t num, int32_t n,
                         int32_t* labels, int64_t* values) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= num) return;
  const uint32_t feas = (uint32_t)info[2 * (int64_t)i];
  const int base = info[2 * (int64_t)i + 1];
  int64_t best = -1;
  int64_t v[kMaxTypes];
  for (int k1 = 0; k1 < n; ++k1) {
    v[k1] = -1;
    if (!((feas >> k1) & 1u)) continue;
    int64_t mn = -1;
    for (int k2 = 0; k2 < n; ++k2) {
      const int64_t c = cost[((int64_t)i * n + k1) * n + k2];
      if (mn < 0 || c < mn) mn = c;
    }
    v[k1] = mn;
    if (best < 0 || mn < best) best = mn;
  }
  int lab = -1;
  if (base >= 0 && base < n && v[base] == best) lab = base;
  for (int k1 = 0; k1 < n && lab < 0; ++k1)
    if (v[k1] == best && v[k1] >= 0) lab = k1;
  labels[i] = lab;
  if (values)
    for (int k1 = 0; k1 < n; ++k1) values[(int64_t)i * n + k1] = v[k1];
}

// Forward + backward over a slice of the minibatch; one partial gradient per
// wavefront.  Weights: bf16 working copy in LDS (row blocks for the forward
// pass, column blocks of W2 for the backward pass).
struct TrainLds {
  float w1[64 * 16];       // W1[l][i]
  float w2r[64 * 64];      // W2[l][j] at [j][l]  (lane l reads unit-stride for fixed j)
  float w2c[64 * 64];      // W2[l][j] at [l][j]  (lane j reads unit-stride for fixed l)
  float w3[16 * 64];       // W3[k][j] at [j][k]
  float b1[64], b2[64], b3[16];
};

__global__ void __launch_bounds__(256) k_train(const vsbpp_model* mdl, const float* X,
                                               const int32_t* mask, const int32_t* label,
                                               const int32_t* idx, int32_t batch,
                                               int32_t per_wave, float inv_batch,
                                               float* partial, float* loss_part) {
  extern __shared__ __align__(16) unsigned char smem[];
  TrainLds* L = reinterpret_cast<TrainLds*>(smem);
  float* hb = reinterpret_cast<float*>(smem + sizeof(TrainLds));  // per wave: h1[64], h2[64], d[64]
  const int nout = mdl->n_out;
  for (int e = threadIdx.x; e < 64 * 16; e += blockDim.x) L->w1[e] = bf16f(mdl->w1[e]);
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int l = e >> 6, j = e & 63;
    const float v = bf16f(mdl->w2[e]);
    L->w2r[j * 64 + l] = v;
    L->w2c[e] = v;
  }
  for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
    const int k = e >> 6, j = e & 63;
    L->w3[j * 16 + k] = k < nout ? bf16f(mdl->w3[e]) : 0.0f;
  }
  for (int e = threadIdx.x; e < 64; e += blockDim.x) {
    L->b1[e] = mdl->b1[e];
    L->b2[e] = mdl->b2[e];
    if (e < 16) L->b3[e] = e < nout ? mdl->b3[e] : 0.0f;
  }
  __syncthreads();
  const int lane = lane_id();
  const int wave = uniform((int)(threadIdx.x >> 6));
  const int gw = blockIdx.x * (blockDim.x >> 6) + wave;
  float* h1s = hb + wave * 192;
  float* h2s = h1s + 64;
  float* ds = h1s + 128;

  float g1[16], g2[64], g3[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) g1[i] = 0.0f;
#pragma unroll
  for (int j = 0; j < 64; ++j) g2[j] = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) g3[k] = 0.0f;
  float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f, lsum = 0.0f;

  const int s0 = gw * per_wave;
  const int s1 = min(batch, s0 + per_wave);
  for (int sidx = s0; sidx < s1; ++sidx) {
    const int sm = uniform(idx[sidx]);
    float x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = X[16 * (int64_t)sm + i];
    const uint32_t feas = (uint32_t)uniform(mask[sm]);
    const int lab = uniform(label[sm]) & 15;
    // forward
    float acc = L->b1[lane];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc = __builtin_fmaf(L->w1[lane * 16 + i], x[i], acc);
    const bool on1 = acc > 0.0f;
    const float h1 = on1 ? acc : 0.0f;
    h1s[lane] = h1;
    acc = L->b2[lane];
    for (int j = 0; j < 64; ++j) acc = __builtin_fmaf(L->w2r[j * 64 + lane], h1s[j], acc);
    const bool on2 = acc > 0.0f;
    const float h2 = on2 ? acc : 0.0f;
    h2s[lane] = h2;
    const int k = lane & 15;
    acc = L->b3[k];
    for (int j = 0; j < 64; ++j) acc = __builtin_fmaf(L->w3[j * 16 + k], h2s[j], acc);
    const float z = acc;
    // masked softmax over the feasible types (fixed order over k)
    float zmax = -INFINITY;
    for (int kk = 0; kk < nout; ++kk)
      if ((feas >> kk) & 1u) zmax = fmaxf(zmax, __uint_as_float(readlane(__float_as_uint(z), kk)));
    const bool feasible = lane < nout && ((feas >> lane) & 1u);
    const float ez = feasible ? expf(z - zmax) : 0.0f;
    float ssum = 0.0f;
    for (int kk = 0; kk < nout; ++kk) ssum += __uint_as_float(readlane(__float_as_uint(ez), kk));
    const float zl = __uint_as_float(readlane(__float_as_uint(z), lab));
    lsum += -(zl - zmax - logf(ssum));
    // dz (mean over the minibatch)
    const float dz = feasible ? (ez / ssum - (lane == lab ? 1.0f : 0.0f)) * inv_batch : 0.0f;
    gb3 += lane < 16 ? dz : 0.0f;
    // dW3[k][j] += dz_k h2_j : lane j accumulates column j
    float dh2 = 0.0f;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      if (kk < nout) {
        const float dzk = __uint_as_float(readlane(__float_as_uint(dz), kk));
        g3[kk] = __builtin_fmaf(dzk, h2, g3[kk]);
        dh2 = __builtin_fmaf(L->w3[lane * 16 + kk], dzk, dh2);
      }
    }
    dh2 = on2 ? dh2 : 0.0f;
    gb2 += dh2;
    ds[lane] = dh2;
    // dW2[l][j] += dh2_l h1_j : lane l accumulates row l
#pragma unroll
    for (int j = 0; j < 64; ++j) g2[j] = __builtin_fmaf(dh2, h1s[j], g2[j]);
    // dh1_j = sum_l W2[l][j] dh2_l : lane j
    float dh1 = 0.0f;
    for (int l = 0; l < 64; ++l) dh1 = __builtin_fmaf(L->w2c[l * 64 + lane], ds[l], dh1);
    dh1 = on1 ? dh1 : 0.0f;
    gb1 += dh1;
#pragma unroll
    for (int i = 0; i < 16; ++i) g1[i] = __builtin_fmaf(dh1, x[i], g1[i]);
  }
  // partial gradient of this wavefront, parameter order w1 b1 w2 b2 w3 b3
  float* out = partial + (int64_t)gw * param_count(nout);
#pragma unroll
  for (int i = 0; i < 16; ++i) out[lane * 16 + i] = g1[i];
  out[1024 + lane] = gb1;
#pragma unroll
  for (int j = 0; j < 64; ++j) out[1088 + lane * 64 + j] = g2[j];
  out[1088 + 4096 + lane] = gb2;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk)
    if (kk < nout) out[5248 + kk * 64 + lane] = g3[kk];
  if (lane < nout) out[5248 + nout * 64 + lane] = gb3;
  if (lane == 0) loss_part[gw] = lsum;
}

__global__ void k_reduce(const float* partial, int32_t waves, int32_t np, float* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  float s = 0.0f;
  for (int w = 0; w < waves; ++w) s += partial[(int64_t)w * np + p];
  grad[p] = s;
}

__global__ void k_adam(float* master, float* m1, float* m2, const float* grad, int32_t np,
                       float lr, float beta1, float beta2, float eps, float c1, float c2,
                       vsbpp_model* mdl) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float g = grad[p];
  const float a = beta1 * m1[p] + (1.0f - beta1) * g;
  const float b = beta2 * m2[p] + (1.0f - beta2) * g * g;
  m1[p] = a;
  m2[p] = b;
  const float w = master[p] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  master[p] = w;
  write_param(mdl, p, w);
}

__global__ void k_publish(const float* master, int32_t np, vsbpp_model* mdl) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) write_param(mdl, p, master[p]);
}

}  // namespace

// parameter p of the flat vector (w1 b1 w2 b2 w3 b3) into the bf16 model
__device__ void write_param(vsbpp_model* mdl, int p, float w) {
  const int nout = mdl->n_out;
  if (p < 1024) {
    mdl->w1[p] = to_bf16(w);
  } else if (p < 1088) {
    mdl->b1[p - 1024] = w;
  } else if (p < 5184) {
    mdl->w2[p - 1088] = to_bf16(w);
  } else if (p < 5248) {
    mdl->b2[p - 5184] = w;
  } else if (p < 5248 + 64 * nout) {
    mdl->w3[p - 5248] = to_bf16(w);
  } else {
    mdl->b3[p - 5248 - 64 * nout] = w;
  }
}

hipError_t launch_labels(const int64_t* cost, const int32_t* info, int32_t num, int32_t n,
                         int32_t* labels, int64_t* values, hipStream_t s) {
  if (num <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_labels, dim3((num + 255) / 256), dim3(256), 0, s, cost, info, num, n,
                     labels, values);
  return hipGetLastError();
}

size_t train_lds_bytes() { return sizeof(TrainLds) + 4 * 192 * sizeof(float); }

hipError_t launch_train(const vsbpp_model* mdl, const float* X, const int32_t* mask,
                        const int32_t* label, const int32_t* idx, int32_t batch, int32_t waves,
                        int32_t nout, float* partial, float* loss_part, float* grad,
                        hipStream_t s) {
  const int per_wave = (batch + waves - 1) / waves;
  const size_t lds = train_lds_bytes();
  static bool raised = false;
  if (!raised) {
    const hipError_t e = allow_max_dynamic_lds(k_train);
    if (e != hipSuccess) return e;
    raised = true;
  }
  hipLaunchKernelGGL(k_train, dim3(waves / 4), dim3(256), lds, s, mdl, X, mask, label, idx,
                     batch, per_wave, 1.0f / (float)batch, partial, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = param_count(nout);
  hipLaunchKernelGGL(k_reduce, dim3((np + 255) / 256), dim3(256), 0, s, partial, waves, np, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* master, float* m1, float* m2, const float* grad, int32_t np,
                       float lr, float beta1, float beta2, float eps, int step, vsbpp_model* mdl,
                       hipStream_t s) {
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, master, m1, m2, grad, np,
                     lr, beta1, beta2, eps, c1, c2, mdl);
  return hipGetLastError();
}

hipError_t launch_publish(const float* master, int32_t np, vsbpp_model* mdl, hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3((np + 255) / 256), dim3(256), 0, s, master, np, mdl);
  return hipGetLastError();
}

}  // namespace vsbpp
