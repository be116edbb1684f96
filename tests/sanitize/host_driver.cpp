// Drives the host-side entry points that need no device -- the cost of a
// packing, the host lower bound, and the checks of model loading -- over
// random and edge inputs, so that an AddressSanitizer /
// UndefinedBehaviorSanitizer build can check their memory and integer use.
// Argument: a scratch directory for model files.  Exits 0 when every call
// returns the documented code.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vsbpp.h"

static uint64_t g_state = 99;
static uint32_t next_u32() {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(g_state >> 33);
}
static int32_t uni(int32_t lo, int32_t hi) {
  return lo + (int32_t)(next_u32() % (uint32_t)((int64_t)hi - lo + 1));
}

int main(int argc, char** argv) {
  int bad = 0;
  const std::string dir = argc > 1 ? argv[1] : ".";
  for (int it = 0; it < 3000; ++it) {
    const int32_t n = uni(1, 16);
    std::vector<int32_t> caps((size_t)n);
    caps[0] = uni(n, it % 5 == 0 ? 2000000000 : 5000);
    bool ok = true;
    for (int32_t k = 1; k < n; ++k) {
      caps[(size_t)k] = caps[(size_t)k - 1] - uni(1, 50);
      if (caps[(size_t)k] <= 0) ok = false;
    }
    const int32_t m = uni(1, 400);
    std::vector<int32_t> w((size_t)m);
    for (auto& x : w) x = uni(1, caps[0]);
    const int64_t lb = vsbpp_lower_bound(w.data(), m, caps.data(), n);
    if (ok && lb < 1) bad++;
    if (!ok && lb != VSBPP_E_CAPS) bad++;
    std::vector<int32_t> types((size_t)m);
    for (auto& t : types) t = uni(0, n - 1);
    const int64_t c = vsbpp_cost(types.data(), m, caps.data(), n);
    if (ok && c < 1) bad++;
    types[0] = n;  // out of range
    if (ok && vsbpp_cost(types.data(), m, caps.data(), n) != VSBPP_E_SIZE) bad++;
  }
  int32_t caps[2] = {10, 6}, w[3] = {4, 11, 2};
  if (vsbpp_lower_bound(w, 3, caps, 2) != VSBPP_E_WEIGHT) bad++;
  if (vsbpp_lower_bound(nullptr, 3, caps, 2) != VSBPP_E_NULL) bad++;
  if (vsbpp_lower_bound(w, 0, caps, 2) != VSBPP_E_SIZE) bad++;
  if (vsbpp_cost(nullptr, 0, caps, 2) != 0) bad++;
  if (vsbpp_cost(nullptr, 1, caps, 2) != VSBPP_E_NULL) bad++;
  if (vsbpp_cost(w, -1, caps, 2) != VSBPP_E_SIZE) bad++;
  // model files: missing, short, long, bad n_out, non-finite, valid
  vsbpp_model* d = nullptr;
  if (vsbpp_model_load((dir + "/missing.bin").c_str(), &d) != VSBPP_E_MODEL || d) bad++;
  vsbpp_model mdl;
  std::memset(&mdl, 0, sizeof mdl);
  mdl.n_out = 5;
  auto write = [&](const char* name, const void* p, size_t sz) {
    const std::string path = dir + "/" + name;
    std::FILE* f = std::fopen(path.c_str(), "wb");
    std::fwrite(p, 1, sz, f);
    std::fclose(f);
    return path;
  };
  std::vector<unsigned char> big(sizeof mdl + 1, 0);
  std::memcpy(big.data(), &mdl, sizeof mdl);
  if (vsbpp_model_load(write("short.bin", &mdl, sizeof mdl - 4).c_str(), &d) != VSBPP_E_MODEL) bad++;
  if (vsbpp_model_load(write("long.bin", big.data(), big.size()).c_str(), &d) != VSBPP_E_MODEL) bad++;
  mdl.n_out = 17;
  if (vsbpp_model_load(write("nout.bin", &mdl, sizeof mdl).c_str(), &d) != VSBPP_E_MODEL) bad++;
  mdl.n_out = 3;
  mdl.b2[7] = NAN;
  if (vsbpp_model_load(write("nan.bin", &mdl, sizeof mdl).c_str(), &d) != VSBPP_E_MODEL) bad++;
  mdl.b2[7] = 0.0f;
  mdl.w2[5] = 0x7F80;  // +inf in bf16
  if (vsbpp_model_load(write("inf.bin", &mdl, sizeof mdl).c_str(), &d) != VSBPP_E_MODEL) bad++;
  mdl.w2[5] = 0;
  const int32_t rc = vsbpp_model_load(write("ok.bin", &mdl, sizeof mdl).c_str(), &d);
  // without a GPU the checks pass and the device copy reports the device
  if (rc != VSBPP_OK && rc != VSBPP_E_DEVICE && rc != VSBPP_E_NOMEM) bad++;
  vsbpp_model_free(d);
  std::printf("host driver: %d failures\n", bad);
  return bad ? 1 : 0;
}
