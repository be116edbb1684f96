// Host-side entry points of the formal problem: the cost of a packing and a
// lower bound on the optimum (Section 1 "Formal Definition of VSBPP",
// Section 6.1), and loading a trained scorer into device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/vsbpp.h"
#include "kernels.h"

namespace {

// capacities positive and strictly decreasing (B_1 > ... > B_n > 0)
int32_t check_caps(const int32_t* caps, int32_t n) {
  if (n < 1 || n > vsbpp::kMaxTypes) return VSBPP_E_SIZE;
  for (int32_t k = 0; k < n; ++k) {
    if (caps[k] <= 0) return VSBPP_E_CAPS;
    if (k > 0 && caps[k] >= caps[k - 1]) return VSBPP_E_CAPS;
  }
  return VSBPP_OK;
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Least total >= `total` that is a sum of capacities with repetition.
// Every such sum is (a sum of the larger capacities) + j * B_n, so it is
// enough to know, per residue r modulo B_n, the least sum of the larger
// capacities congruent to r: the round-robin algorithm (Boecker & Liptak,
// 2007) relaxes the residue classes one capacity at a time, walking each
// cycle of r -> r + B_k (mod B_n) from its least entry.
int64_t least_capacity_sum(int64_t total, const int32_t* caps, int32_t n) {
  const int64_t base = caps[n - 1];
  constexpr int64_t kInf = INT64_MAX / 4;
  std::vector<int64_t> d((size_t)base, kInf);
  d[0] = 0;
  for (int32_t k = 0; k + 1 < n; ++k) {
    const int64_t a = caps[k];
    const int64_t g = gcd64(a, base);
    const int64_t steps = base / g;
    for (int64_t p = 0; p < g; ++p) {
      // least entry of the cycle through p
      int64_t start = p, best = d[(size_t)p];
      for (int64_t s = 1, r = (p + a) % base; s < steps; ++s, r = (r + a) % base)
        if (d[(size_t)r] < best) {
          best = d[(size_t)r];
          start = r;
        }
      if (best >= kInf) continue;
      int64_t r = start;
      for (int64_t s = 0; s < steps; ++s) {
        const int64_t nx = (r + a) % base;
        if (d[(size_t)r] + a < d[(size_t)nx]) d[(size_t)nx] = d[(size_t)r] + a;
        r = nx;
      }
    }
  }
  int64_t lb = INT64_MAX;
  for (int64_t r = 0; r < base; ++r) {
    const int64_t v = d[(size_t)r];
    if (v >= kInf) continue;
    const int64_t c = v >= total ? v : v + (total - v + base - 1) / base * base;
    if (c < lb) lb = c;
  }
  return lb;
}

// residue tables above this many entries are not built (the bound is then
// the total weight)
constexpr int32_t kResidueLimit = 1 << 20;

bool finite_bf16(uint16_t h) { return (h & 0x7F80u) != 0x7F80u; }

}  // namespace

extern "C" {

int64_t vsbpp_cost(const int32_t* bin_types, int32_t nbins, const int32_t* caps, int32_t n) {
  if (!caps || (nbins > 0 && !bin_types)) return VSBPP_E_NULL;
  if (nbins < 0) return VSBPP_E_SIZE;
  const int32_t rc = check_caps(caps, n);
  if (rc != VSBPP_OK) return rc;
  int64_t cost = 0;
  for (int32_t b = 0; b < nbins; ++b) {
    const int32_t t = bin_types[b];
    if (t < 0 || t >= n) return VSBPP_E_SIZE;
    cost += caps[t];
  }
  return cost;
}

int64_t vsbpp_lower_bound(const int32_t* weights, int32_t m, const int32_t* caps, int32_t n) {
  if (!weights || !caps) return VSBPP_E_NULL;
  if (m < 1) return VSBPP_E_SIZE;
  int32_t rc = check_caps(caps, n);
  if (rc != VSBPP_OK) return rc;
  int64_t total = 0, big = 0;
  for (int32_t j = 0; j < m; ++j) {
    const int32_t w = weights[j];
    if (w < 1 || w > caps[0]) return VSBPP_E_WEIGHT;
    total += w;
    // two items heavier than B_1 / 2 never share a bin: each needs its own,
    // at least the smallest capacity holding it
    if (2 * (int64_t)w > caps[0]) {
      int32_t k = n - 1;
      while (caps[k] < w) --k;
      big += caps[k];
    }
  }
  const int64_t cap_lb = caps[n - 1] <= kResidueLimit ? least_capacity_sum(total, caps, n) : total;
  return cap_lb > big ? cap_lb : big;
}

int32_t vsbpp_model_load(const char* path, vsbpp_model** out) {
  if (!out) return VSBPP_E_NULL;
  *out = nullptr;
  if (!path) return VSBPP_E_NULL;
  vsbpp_model m;
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return VSBPP_E_MODEL;
  const size_t got = std::fread(&m, 1, sizeof m, f);
  const bool longer = std::fgetc(f) != EOF;
  std::fclose(f);
  if (got != sizeof m || longer) return VSBPP_E_MODEL;
  if (m.n_out < 1 || m.n_out > VSBPP_MAX_OUT) return VSBPP_E_MODEL;
  for (uint16_t h : m.w1)
    if (!finite_bf16(h)) return VSBPP_E_MODEL;
  for (uint16_t h : m.w2)
    if (!finite_bf16(h)) return VSBPP_E_MODEL;
  for (int i = 0; i < VSBPP_HIDDEN * m.n_out; ++i)
    if (!finite_bf16(m.w3[i])) return VSBPP_E_MODEL;
  for (float b : m.b1)
    if (!std::isfinite(b)) return VSBPP_E_MODEL;
  for (float b : m.b2)
    if (!std::isfinite(b)) return VSBPP_E_MODEL;
  for (int i = 0; i < m.n_out; ++i)
    if (!std::isfinite(m.b3[i])) return VSBPP_E_MODEL;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
    (void)hipGetLastError();
    return VSBPP_E_DEVICE;
  }
  vsbpp_model* d = nullptr;
  if (hipMalloc(&d, sizeof m) != hipSuccess) {
    (void)hipGetLastError();
    return VSBPP_E_NOMEM;
  }
  if (hipMemcpy(d, &m, sizeof m, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d);
    return VSBPP_E_DEVICE;
  }
  *out = d;
  return VSBPP_OK;
}

void vsbpp_model_free(vsbpp_model* d_model) {
  if (d_model) (void)hipFree(d_model);
}

}  // extern "C"
