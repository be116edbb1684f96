// Wavefront primitives and the counter-based generator used by every
// packing kernel (gfx950, 64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// The LLVM intrinsic behind v_writelane_b32 (this compiler has no builtin
// for it): returns v with lane l replaced by x, both wave-uniform.
extern "C" __device__ int vsbpp_amdgcn_writelane(int x, int l, int v) __asm(
    "llvm.amdgcn.writelane.i32");

namespace vsbpp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ int32_t readlane(int32_t v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ uint64_t readlane(uint64_t v, int l) {
  uint32_t lo = readlane((uint32_t)v, l), hi = readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
// v with lane l (wave-uniform) set to x (wave-uniform), by v_writelane_b32
__device__ __forceinline__ int32_t writelane(int32_t v, int32_t x, int l) {
  return vsbpp_amdgcn_writelane(x, l, v);
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// DPP move with an explicit fill value for lanes the control does not write.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t fill, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, ROWS, 0xF, false);
}

// DPP controls (GFX9 encoding)
constexpr int kQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;
constexpr int kRowShr1 = 0x111;

// Unsigned minimum over the 64 lanes; the result is wave-uniform.  All lanes
// must be active.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  constexpr uint32_t I = 0xFFFFFFFFu;
  v = min(v, dpp<kQuadSwap1>(I, v));
  v = min(v, dpp<kQuadSwap2>(I, v));
  v = min(v, dpp<kRowHalfMirror>(I, v));
  v = min(v, dpp<kRowMirror>(I, v));
  v = min(v, dpp<kRowBcast15, 0xA>(I, v));
  v = min(v, dpp<kRowBcast31, 0xC>(I, v));
  return readlane(v, 63);
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint64_t dpp64(uint64_t fill, uint64_t v) {
  uint32_t lo = dpp<CTRL, ROWS>((uint32_t)fill, (uint32_t)v);
  uint32_t hi = dpp<CTRL, ROWS>((uint32_t)(fill >> 32), (uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min(uint64_t v) {
  constexpr uint64_t I = ~0ull;
  v = min(v, dpp64<kQuadSwap1>(I, v));
  v = min(v, dpp64<kQuadSwap2>(I, v));
  v = min(v, dpp64<kRowHalfMirror>(I, v));
  v = min(v, dpp64<kRowMirror>(I, v));
  v = min(v, dpp64<kRowBcast15, 0xA>(I, v));
  v = min(v, dpp64<kRowBcast31, 0xC>(I, v));
  return readlane(v, 63);
}

__device__ __forceinline__ int32_t wave_min(int32_t v) {
  return (int32_t)(wave_min((uint32_t)v ^ 0x80000000u) ^ 0x80000000u);
}

// Inclusive prefix maximum over the 64 lanes of non-negative values (all
// lanes active): row shifts within each row of 16, then the last lane of each
// row carried into the following rows.
__device__ __forceinline__ int32_t wave_incl_max(int32_t v) {
  v = max(v, (int32_t)dpp<0x111>(0u, (uint32_t)v));  // row_shr:1
  v = max(v, (int32_t)dpp<0x112>(0u, (uint32_t)v));  // row_shr:2
  v = max(v, (int32_t)dpp<0x114>(0u, (uint32_t)v));  // row_shr:4
  v = max(v, (int32_t)dpp<0x118>(0u, (uint32_t)v));  // row_shr:8
  v = max(v, (int32_t)dpp<kRowBcast15, 0xA>(0u, (uint32_t)v));
  v = max(v, (int32_t)dpp<kRowBcast31, 0xC>(0u, (uint32_t)v));
  return v;
}

// v of the lane below (lane 0: 0), by a wavefront shift
__device__ __forceinline__ int32_t wave_shr1(int32_t v) {
  return (int32_t)dpp<0x138>(0u, (uint32_t)v);  // wave_shr:1
}

// Inclusive prefix sum within each row of 16 lanes (all lanes active): four
// DPP row shifts that bring in 0 past the row's start.
__device__ __forceinline__ int32_t row_incl_sum(int32_t v) {
  v += (int32_t)dpp<0x111>(0u, (uint32_t)v);  // row_shr:1
  v += (int32_t)dpp<0x112>(0u, (uint32_t)v);  // row_shr:2
  v += (int32_t)dpp<0x114>(0u, (uint32_t)v);  // row_shr:4
  v += (int32_t)dpp<0x118>(0u, (uint32_t)v);  // row_shr:8
  return v;
}

// Inclusive prefix sum over the 64 lanes (all lanes active).
__device__ __forceinline__ int32_t wave_incl_sum(int32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  Output k of the generator
// whose state starts at `seed`: the state seed + (k+1)*gamma through the
// published 64-bit finaliser.
// ---------------------------------------------------------------------------
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;

// the published finaliser applied to a generator state
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t s) {
  s ^= s >> 30;
  s *= 0xbf58476d1ce4e5b9ull;
  s ^= s >> 27;
  s *= 0x94d049bb133111ebull;
  return s ^ (s >> 31);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  return splitmix64_mix(seed + (k + 1ull) * kGolden);
}

// generator streams (one key per purpose, derived from the instance seed)
constexpr uint64_t kStreamRule1 = 1, kStreamH1 = 2, kStreamH2 = 3;

__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return splitmix64(seed, stream);
}

// Rule 3 criterion: FF/BF/WF with equal probability, floor(3*hi32 / 2^32).
__device__ __forceinline__ int draw_criterion(uint64_t key, uint64_t counter) {
  uint64_t hi = splitmix64(key, counter) >> 32;
  return (int)((hi * 3ull) >> 32);
}

// The second heuristic's draws: one output per permutation packing, its high
// word h; the criterion of placement t is digit t+1 of h / 2^32 in base 3.
// With u = h: criterion = floor(3u / 2^32), then u = 3u mod 2^32, per
// placement (digits_next).
__device__ __forceinline__ uint32_t digits_word(uint64_t key, uint64_t counter) {
  return (uint32_t)(splitmix64(key, counter) >> 32);
}
__device__ __forceinline__ int digits_next(uint32_t& u) {
  const int c = (int)__umulhi(u, 3u);
  u *= 3u;
  return c;
}

// Rule 1 distribution: keyed permutation of [0,m) from a 4-round balanced
// Feistel network on 2h bits (2^(2h) >= m, round function = generator output
// for counter (round << 32 | right half)), restricted to [0,m) by cycle
// walking (Black & Rogaway, CT-RSA 2002).
struct Rule1Perm {
  uint64_t key;
  uint32_t h, mask, m;
  __device__ void init(uint64_t seed, uint32_t m_) {
    m = m_;
    uint32_t bits = 0;
    while ((1u << bits) < m && bits < 31) ++bits;
    h = (bits + 1) >> 1;
    mask = (1u << h) - 1u;
    key = stream_key(seed, kStreamRule1);
  }
  __device__ __forceinline__ uint32_t round_trip(uint32_t x) const {
    uint32_t l = x >> h, r = x & mask;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      uint32_t f = (uint32_t)splitmix64(key, ((uint64_t)i << 32) | r) & mask;
      uint32_t t = l ^ f;
      l = r;
      r = t;
    }
    return (l << h) | r;
  }
  __device__ uint32_t at(uint32_t q) const {
    if (m <= 1) return 0;
    uint32_t y = round_trip(q);
    while (y >= m) y = round_trip(y);
    return y;
  }
};

}  // namespace vsbpp
