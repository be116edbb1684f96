// Key layout and helpers shared by the plain FF/BF/WF kernels (one
// wavefront per instance, and several wavefronts per instance).
//
// A bin's key: high part its room (BF/FF) or R - room (WF), low part its
// position in the scan array; the candidate key for item w is key -/+ (w <<
// SH), and non-fitting bins wrap above TOP.  Position p lives at (p & ~255) +
// ((p & 63) << 2) + ((p >> 6) & 3), so one 4-key vector load per lane covers
// a group of 256 positions with unit-stride lanes.
#pragma once
#include "device_common.h"
#include "kernels.h"

namespace vsbpp {
namespace {

template <typename K>
struct KeyT;
template <>
struct KeyT<uint32_t> {
  static constexpr int SH = 16;
  static constexpr uint32_t R = 0x7FFFu;
  static constexpr uint32_t TOP = 0x80000000u;
  static constexpr uint32_t POS = 0xFFFFu;
  using Pid = uint16_t;
};
template <>
struct KeyT<uint64_t> {
  static constexpr int SH = 32;
  static constexpr uint64_t R = 0x7FFFFFFFull;
  static constexpr uint64_t TOP = 0x8000000000000000ull;
  static constexpr uint64_t POS = 0xFFFFFFFFull;
  using Pid = uint32_t;
};

constexpr int FF = 0, BF = 1, WF = 2;

__device__ __forceinline__ int kidx(int p) {
  return (p & ~255) + ((p & 63) << 2) + ((p >> 6) & 3);
}

// One key written by the lane that holds it.  Position p belongs to lane
// p & 63, and relative to that lane's first key (keys + 4 * lane, `mine`) it
// sits (p & ~255) + ((p >> 6) & 3) entries on: an offset the whole wavefront
// shares, so the address is the lane's own base plus a scalar.
template <typename K>
__device__ __forceinline__ void put_key(K* mine, int lane, int p, K v) {
  if (lane == (p & 63)) mine[(p & ~255) + ((p >> 6) & 3)] = v;
}

template <typename K>
__device__ __forceinline__ void load_group(const K* keys, int g, int lane, K (&k)[4]) {
  if constexpr (sizeof(K) == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(keys + (g << 8) + (lane << 2));
    k[0] = v.x; k[1] = v.y; k[2] = v.z; k[3] = v.w;
  } else {
    const ulonglong2* p = reinterpret_cast<const ulonglong2*>(keys + (g << 8) + (lane << 2));
    const ulonglong2 a = p[0], b = p[1];
    k[0] = a.x; k[1] = a.y; k[2] = b.x; k[3] = b.y;
  }
}

template <typename K>
__device__ __forceinline__ void fill_group(K* keys, int g, int lane, K v) {
  if constexpr (sizeof(K) == 4) {
    *reinterpret_cast<uint4*>(keys + (g << 8) + (lane << 2)) = make_uint4(v, v, v, v);
  } else {
    ulonglong2* p = reinterpret_cast<ulonglong2*>(keys + (g << 8) + (lane << 2));
    ulonglong2 e;
    e.x = v;
    e.y = v;
    p[0] = e;
    p[1] = e;
  }
}

template <int CRIT, typename K>
__device__ __forceinline__ K empty_key() {
  using T = KeyT<K>;
  return CRIT == WF ? ((T::R << T::SH) | T::POS) : (K)0;
}

template <int CRIT, typename K>
__device__ __forceinline__ K room_of(K key) {
  using T = KeyT<K>;
  return CRIT == WF ? T::R - (key >> T::SH) : (key >> T::SH);
}

// Stable compaction of the live positions (room >= T).  Returns the new
// count and leaves the tail of the last 256-position group empty.
template <int CRIT, typename K>
__device__ int compact(K* keys, typename KeyT<K>::Pid* pid, int nlive, int32_t T, int lane) {
  using KT = KeyT<K>;
  const int ng = (nlive + 255) >> 8;
  int newn = 0;
  for (int g = 0; g < ng; ++g) {
    K k[4];
    load_group(keys, g, lane, k);
    typename KT::Pid pv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pv[j] = pid[(g << 8) + (j << 6) + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pos = (g << 8) + (j << 6) + lane;
      const bool live = pos < nlive && room_of<CRIT>(k[j]) >= (K)T;
      const uint64_t lm = ballot(live);
      if (live) {
        const int np = newn + lanes_below(lm);
        keys[kidx(np)] = (k[j] & ~KT::POS) | (K)np;
        pid[np] = pv[j];
      }
      newn += __popcll(lm);
    }
  }
  if (newn & 255) {
    const int g = newn >> 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pos = (g << 8) + (j << 6) + lane;
      if (pos >= newn) keys[kidx(pos)] = empty_key<CRIT, K>();
    }
  }
  return newn;
}

}  // namespace
}  // namespace vsbpp
