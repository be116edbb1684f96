// Plain First/Best/Worst Fit (paper Section 1) over whole item lists, one
// 64-lane wavefront per instance.
//
// Per item (the hot step): every live bin tests in parallel whether the item
// fits (Rule 4 applicability) and a wave reduction picks the bin:
//   FF: ballot over 64-bin rows in position order, first set lane;
//   BF: min of (room_after << SH | position);
//   WF: min of ((R - room_after) << SH | position);
// lowest position wins ties by construction, and positions keep bin-creation
// order, so that is the lowest bin index.  When nothing fits, a bin of type
// max{k : B_k >= w} (or B_1) is appended.
//
// Bin state lives in LDS as one key per bin whose high part encodes the room
// left (BF/FF: room, WF: R - room) and whose low part is the bin's position
// in the scan array, so the candidate key for item w is key -/+ (w << SH) and
// non-fitting bins wrap above TOP.  A bin whose room is below the smallest
// weight still to come can never be chosen again; every 64 items such dead
// bins are removed by a stable in-wave compaction, which keeps positions in
// creation order.  A separate LDS array maps positions to bin ids.
//
// LDS layout of keys: position p lives at (p & ~255) + ((p & 63) << 2) +
// ((p >> 6) & 3), so one 4-key vector load per lane covers 256 positions with
// unit-stride lanes.
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

template <int CRIT, typename K>
__global__ void __launch_bounds__(256) k_plain(BatchArgs a, int wpb, int lds_per_wave) {
  using KT = KeyT<K>;
  using Pid = typename KT::Pid;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave = uniform((int)(threadIdx.x >> 6));
  unsigned char* base = smem + (size_t)wave * lds_per_wave;
  K* keys = reinterpret_cast<K*>(base);
  const size_t pid_bytes = ((size_t)a.slots * sizeof(Pid) + 15) & ~(size_t)15;
  Pid* pid = reinterpret_cast<Pid*>(base + (size_t)a.slots * sizeof(K));
  int32_t* smin = reinterpret_cast<int32_t*>(base + (size_t)a.slots * sizeof(K) + pid_bytes);

  int cursor = blockIdx.x * wpb + wave;
  for (;;) {
    int slot;
    if (a.queue) {
      int v = 0;
      if (lane == 0) v = atomicAdd(a.queue, 1);
      slot = uniform(readlane(v, 0));
    } else {
      slot = cursor;
      cursor += gridDim.x * wpb;
    }
    if (slot >= a.num) break;
    const int inst = a.sched ? uniform(a.sched[slot]) : slot;
    const int64_t off = a.item_off[inst];
    const int64_t m64 = a.item_off[inst + 1] - off;
    const int c0 = a.cap_off[inst];
    const int n = a.cap_off[inst + 1] - c0;
    int err = 0;
    if (m64 < 1 || m64 > a.max_items || n < 1 || n > kMaxTypes || n > a.max_types)
      err = kErrSize;
    int32_t cap_lane = 0, B1 = 0;
    if (!err) {
      cap_lane = lane < n ? a.caps[c0 + lane] : 0;
      const int32_t prev = (lane > 0 && lane < n) ? a.caps[c0 + lane - 1] : 0x7FFFFFFF;
      if (ballot(lane < n && (cap_lane <= 0 || cap_lane >= prev))) err = kErrCaps;
      B1 = readlane(cap_lane, 0);
      if (!err && B1 > a.max_cap) err = kErrSize;
    }
    const int m = (int)m64;
    const int nch = (m + 63) >> 6;
    if (!err) {
      // validation and per-chunk suffix minima of the weights in position order
      bool badw = false, bado = false;
      int32_t run = 0x7FFFFFFF;
      for (int c = nch - 1; c >= 0; --c) {
        const int q = (c << 6) + lane;
        int32_t wq = 0x7FFFFFFF;
        if (q < m) {
          const int32_t wd = a.w[off + q];
          badw |= (wd < 1 || wd > B1);
          int item = q;
          if (a.order) {
            item = a.order[off + q];
            if ((unsigned)item >= (unsigned)m) {
              bado = true;
              item = q;
            }
            wq = a.w[off + item];
          } else {
            wq = wd;
          }
        }
        run = min(run, wave_min(wq));
        if (lane == 0) smin[c] = run;
      }
      if (ballot(badw)) err = kErrWeight;
      else if (ballot(bado)) err = kErrOption;
    }
    if (err) {
      if (lane == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      continue;
    }

    int nlive = 0, nb = 0, dead = 0;
    int32_t tprev = 0;
    int64_t cost = 0;
    int32_t typebuf = 0;
    for (int c = 0; c < nch; ++c) {
      const int32_t T = uniform(smin[c]);
      if (nlive > 0 && (dead > 0 || T > tprev)) {
        nlive = uniform(compact<CRIT, K>(keys, pid, nlive, T, lane));
        dead = 0;
      }
      tprev = T;
      const int q = (c << 6) + lane;
      int item = q;
      int32_t wv = 0;
      if (q < m) {
        if (a.order) item = a.order[off + q];
        wv = a.w[off + item];
      }
      // positions are stable until the next compaction, so each item records
      // its bin's position and the ids are read once at the end of the chunk
      int32_t mypos = 0;
      const int cnt = min(kWave, m - (c << 6));
      for (int jj = 0; jj < cnt; ++jj) {
        const int32_t w = readlane(wv, jj);
        const K wk = (K)w << KT::SH;
        int p = -1;
        K nk = 0;
        const int ng = uniform((nlive + 255) >> 8);
        if constexpr (CRIT == FF) {
          for (int g = 0; g < ng && p < 0; ++g) {
            K k[4];
            load_group(keys, g, lane, k);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint64_t fm = ballot(k[j] >= wk);
              if (fm) {
                const int l = __builtin_ctzll(fm);
                p = (g << 8) + (j << 6) + l;
                nk = readlane(k[j], l) - wk;
                break;
              }
            }
          }
        } else {
          K best = ~(K)0;
          int g = 0;
          for (; g + 1 < ng; g += 2) {
            K k[4], k2[4];
            load_group(keys, g, lane, k);
            load_group(keys, g + 1, lane, k2);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              best = min(best, CRIT == WF ? k[j] + wk : k[j] - wk);
              best = min(best, CRIT == WF ? k2[j] + wk : k2[j] - wk);
            }
          }
          if (g < ng) {
            K k[4];
            load_group(keys, g, lane, k);
#pragma unroll
            for (int j = 0; j < 4; ++j) best = min(best, CRIT == WF ? k[j] + wk : k[j] - wk);
          }
          best = wave_min(best);
          if (best < KT::TOP) {
            p = (int)(best & KT::POS);
            nk = best;
          }
        }
        if (p >= 0) {
          // Rule 4: place into the chosen open bin
          if (lane == (p & 63)) keys[kidx(p)] = nk;
          if (room_of<CRIT>(nk) < (K)T) ++dead;
        } else {
          // nothing fits: open a bin of the chosen type
          const uint64_t fm = ballot(lane < n && cap_lane >= w);
          const int t = a.type_rule == 1 ? 0 : (int)__popcll(fm) - 1;
          const int32_t Bt = readlane(cap_lane, t);
          const K room = (K)(Bt - w);
          p = nlive;
          nlive = uniform(nlive + 1);
          const int id = nb;
          nb = uniform(nb + 1);
          if ((p & 255) == 0) fill_group(keys, p >> 8, lane, empty_key<CRIT, K>());
          const K key = CRIT == WF ? (((KT::R - room) << KT::SH) | (K)p) : ((room << KT::SH) | (K)p);
          if (lane == (p & 63)) keys[kidx(p)] = key;
          if (lane == 0) pid[p] = (Pid)id;
          typebuf = lane == (id & 63) ? t : typebuf;
          if ((id & 63) == 63) a.types[off + (id - 63) + lane] = typebuf;
          cost += Bt;
          if (room < (K)T) ++dead;
        }
        mypos = lane == jj ? p : mypos;
      }
      if (q < m) a.assign[off + item] = (int32_t)pid[mypos];
    }
    if ((nb & 63) && lane < (nb & 63)) a.types[off + (nb & ~63) + lane] = typebuf;
    if (lane == 0) {
      a.nbins[inst] = nb;
      a.cost[inst] = cost;
    }
  }
}

template <int CRIT, typename K>
hipError_t launch_one(const BatchArgs& a, int wpb, size_t lds_per_wave, int grid, hipStream_t s) {
  const size_t lds = lds_per_wave * (size_t)wpb;
  auto kern = k_plain<CRIT, K>;
  static bool raised = false;
  if (lds > 65536 && !raised) {
    hipError_t e = allow_max_dynamic_lds(kern);
    if (e != hipSuccess) return e;
    raised = true;
  }
  const int blocks = grid > 0 ? grid : (a.num + wpb - 1) / wpb;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, s, a, wpb, (int)lds_per_wave);
  return hipGetLastError();
}

template <int CRIT, typename K>
int occupancy(int wpb, size_t lds_per_wave) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K>, 64 * wpb,
                                                    lds_per_wave * (size_t)wpb) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace

size_t plain_lds_per_wave(int slots, int max_items, bool wide) {
  const size_t ks = wide ? 8 : 4, ps = wide ? 4 : 2;
  const size_t nch = ((size_t)max_items + 63) / 64;
  size_t b = (size_t)slots * ks;
  b += ((size_t)slots * ps + 15) & ~(size_t)15;
  b += (nch * 4 + 15) & ~(size_t)15;
  return b;
}

hipError_t launch_plain_grid(const BatchArgs& a, int crit, bool wide, int wpb,
                             size_t lds_per_wave, int grid, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  if (!wide) {
    if (crit == FF) return launch_one<FF, uint32_t>(a, wpb, lds_per_wave, grid, s);
    if (crit == BF) return launch_one<BF, uint32_t>(a, wpb, lds_per_wave, grid, s);
    return launch_one<WF, uint32_t>(a, wpb, lds_per_wave, grid, s);
  }
  if (crit == FF) return launch_one<FF, uint64_t>(a, wpb, lds_per_wave, grid, s);
  if (crit == BF) return launch_one<BF, uint64_t>(a, wpb, lds_per_wave, grid, s);
  return launch_one<WF, uint64_t>(a, wpb, lds_per_wave, grid, s);
}

hipError_t launch_plain(const BatchArgs& a, int crit, bool wide, int wpb, size_t lds_per_wave,
                        hipStream_t s) {
  return launch_plain_grid(a, crit, wide, wpb, lds_per_wave, 0, s);
}

int plain_blocks_per_cu(int crit, bool wide, int wpb, size_t lds_per_wave) {
  if (!wide) {
    if (crit == FF) return occupancy<FF, uint32_t>(wpb, lds_per_wave);
    if (crit == BF) return occupancy<BF, uint32_t>(wpb, lds_per_wave);
    return occupancy<WF, uint32_t>(wpb, lds_per_wave);
  }
  if (crit == FF) return occupancy<FF, uint64_t>(wpb, lds_per_wave);
  if (crit == BF) return occupancy<BF, uint64_t>(wpb, lds_per_wave);
  return occupancy<WF, uint64_t>(wpb, lds_per_wave);
}

}  // namespace vsbpp
