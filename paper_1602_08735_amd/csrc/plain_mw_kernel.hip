// Plain First/Best/Worst Fit (paper Section 1) with W = 2 or 4 wavefronts
// on one instance, for instances whose per-item scan covers many 256-position
// groups of live bins (thousands of items).
//
// The hot step is the one of the one-wavefront kernel -- every live bin
// tests the item in parallel (Rule 4 applicability) and a minimum over
// (room << 16 | position) keys picks the First/Best/Worst-Fit bin, lowest
// position on ties -- but the groups of the instance's key array are dealt to
// the W wavefronts: group g belongs to wavefront g % W, which alone reads and
// writes it between compactions.  Per item each wavefront scans its groups
// and leaves its DPP minimum in an LDS slot; after one workgroup barrier every
// wavefront takes the minimum of the W slots, so all of them make the same
// decision, and the owner of the chosen (or newly opened) position writes its
// key.  The slots alternate between two sets by item parity, so the next
// item's slots never overwrite ones still being read, and one barrier per
// item suffices.  At chunk boundaries (every 64 items) wavefront 0 writes the
// chunk's assignments and, when bins may have died (their room fell below the
// smallest weight still to come), compacts the whole array with the
// one-wavefront routine between two barriers.
//
// Scope: 32-bit keys (B_1 <= 32767, m <= 65535), no scorer, decision hooks,
// bound on the open bins or device region.
#include "block_common.h"
#include "device_common.h"
#include "kernels.h"
#include "plain_common.h"

namespace vsbpp {
namespace {

template <int CRIT, int W>
__global__ void __launch_bounds__(256) k_plain_mw(BatchArgs a) {
  using K = uint32_t;
  using KT = KeyT<K>;
  using Pid = uint16_t;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_caps[kMaxTypes];
  __shared__ __align__(16) uint32_t s_best[2][4];
  __shared__ int s_slot, s_flag, s_nlive;
  __shared__ int s_need[4];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = uniform((int)(tid >> 6));
  K* const keys = reinterpret_cast<K*>(smem);
  Pid* const pid = reinterpret_cast<Pid*>(smem + (size_t)a.slots * sizeof(K));
  int32_t* const smin = reinterpret_cast<int32_t*>(
      smem + (size_t)a.slots * sizeof(K) + (((size_t)a.slots * sizeof(Pid) + 15) & ~(size_t)15));
  K* const mine = keys + 4 * lane;

  int cursor = blockIdx.x;
  for (;;) {
    const int slot = next_slot(a, &cursor, &s_slot);
    if (slot >= a.num) break;
    const int inst = a.sched ? a.sched[slot] : slot;
    const int64_t off = a.item_off[inst];
    const int64_t m64 = a.item_off[inst + 1] - off;
    const int c0 = a.cap_off[inst];
    const int n = a.cap_off[inst + 1] - c0;
    const int m = m64 > 0x7FFFFFFF ? 0x7FFFFFFF : (int)m64;
    const int err =
        m64 > a.max_items ? kErrSize : validate_block(a, inst, off, m, c0, n, s_caps, &s_flag);
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      __syncthreads();
      continue;
    }
    const int32_t cap_lane = lane < n ? s_caps[lane] : 0;
    const int nch = (m + 63) >> 6;
    // per-chunk suffix minima of the weights in position order
    if (wave == 0) {
      int32_t run = 0x7FFFFFFF;
      for (int c = nch - 1; c >= 0; --c) {
        const int q = (c << 6) + lane;
        int32_t wq = 0x7FFFFFFF;
        if (q < m) wq = a.w[off + (a.order ? a.order[off + q] : q)];
        run = min(run, (int32_t)wave_min((uint32_t)wq));
        if (lane == 0) smin[c] = run;
      }
    }
    __syncthreads();

    int nlive = 0, nb = 0, par = 0;
    int32_t cost = 0, typebuf = 0;
    // least room this wavefront wrote since the last compaction (its groups)
    uint32_t minroom = 0xFFFFFFFFu;
    int32_t tprev = 0;
    for (int c = 0; c < nch; ++c) {
      const int32_t T = uniform(smin[c]);
      const int q = (c << 6) + lane;
      int item = q;
      int32_t wv = 0;
      if (q < m) {
        if (a.order) item = a.order[off + q];
        wv = a.w[off + item];
      }
      int32_t mypos = 0;
      const int cnt = min(kWave, m - (c << 6));
      for (int jj = 0; jj < cnt; ++jj) {
        const int32_t w = readlane(wv, jj);
        const K wk = (K)w << KT::SH;
        const int ng = uniform((nlive + 255) >> 8);
        K best = ~(K)0;
        for (int g = wave; g < ng; g += W) {
          K k[4];
          load_group(keys, g, lane, k);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if constexpr (CRIT == FF) {
              // the lowest fitting position: halves swapped, pos << 16 | room
              const K sw = (k[j] >> KT::SH) | (k[j] << KT::SH);
              best = min(best, k[j] >= wk ? sw : ~(K)0);
            } else {
              best = min(best, CRIT == WF ? k[j] + wk : k[j] - wk);
            }
          }
        }
        best = wave_min(best);
        if (lane == 0) s_best[par][wave] = best;
        __syncthreads();
        K gb = s_best[par][0];
#pragma unroll
        for (int v = 1; v < W; ++v) gb = min(gb, (K)s_best[par][v]);
        gb = uniform(gb);
        par ^= 1;
        int p = -1;
        K nk = 0;
        if constexpr (CRIT == FF) {
          if (gb != ~(K)0) {
            p = (int)(gb >> KT::SH);
            nk = (((gb & KT::POS) << KT::SH) | (K)p) - wk;
          }
        } else {
          if (gb < KT::TOP) {
            p = (int)(gb & KT::POS);
            nk = gb;
          }
        }
        if (p >= 0) {
          // Rule 4: the owner of position p updates its key
          if (wave == ((p >> 8) % W)) {
            put_key(mine, lane, p, nk);
            minroom = min(minroom, (uint32_t)room_of<CRIT>(nk));
          }
        } else {
          // nothing fits: a bin of the smallest type holding the item (or B_1)
          const uint64_t fm = ballot(cap_lane >= w);
          const int t = a.type_rule == 1 ? 0 : (int)__popcll(fm) - 1;
          const int32_t Bt = readlane(cap_lane, t);
          const K room = (K)(Bt - w);
          p = nlive;
          nlive = uniform(nlive + 1);
          const int id = nb;
          nb = uniform(nb + 1);
          if (wave == ((p >> 8) % W)) {
            if ((p & 255) == 0) fill_group(keys, p >> 8, lane, empty_key<CRIT, K>());
            const K key = CRIT == WF ? (((KT::R - room) << KT::SH) | (K)p)
                                     : ((room << KT::SH) | (K)p);
            if (lane == (p & 63)) {
              mine[(p & ~255) + ((p >> 6) & 3)] = key;
              pid[(p & ~63) + lane] = (Pid)id;
            }
            minroom = min(minroom, (uint32_t)room);
          }
          typebuf = lane == (id & 63) ? t : typebuf;
          if (wave == 0 && (id & 63) == 63) a.types[off + (id - 63) + lane] = typebuf;
          cost += Bt;
        }
        mypos = lane == jj ? p : mypos;
      }
      // chunk end: every key and id of the chunk is written
      const int32_t Tn = c + 1 < nch ? uniform(smin[c + 1]) : T;
      if (lane == 0) s_need[wave] = minroom < (uint32_t)Tn ? 1 : 0;
      __syncthreads();
      if (wave == 0 && q < m) a.assign[off + item] = (int32_t)pid[mypos];
      int need = Tn > tprev ? 1 : 0;
#pragma unroll
      for (int v = 0; v < W; ++v) need |= s_need[v];
      tprev = Tn;
      if (c + 1 < nch && nlive > 0 && need) {
        // every wavefront has passed the chunk's last key write (barrier
        // above); wavefront 0 compacts, the others wait for the new layout
        if (wave == 0) {
          const int nl = compact<CRIT, K>(keys, pid, nlive, Tn, lane);
          if (lane == 0) s_nlive = nl;
        }
        __syncthreads();
        nlive = uniform(s_nlive);
        minroom = 0xFFFFFFFFu;
      }
      // the slots of s_need are rewritten only after the next chunk's items,
      // each of which passes a barrier
    }
    if (wave == 0) {
      if ((nb & 63) && lane < (nb & 63)) a.types[off + (nb & ~63) + lane] = typebuf;
      if (lane == 0) {
        a.nbins[inst] = nb;
        a.cost[inst] = cost;
      }
    }
    __syncthreads();
  }
}

template <int CRIT, int W>
hipError_t launch_mw(const BatchArgs& a, size_t lds, int grid, hipStream_t s) {
  auto kern = k_plain_mw<CRIT, W>;
  static bool raised = false;
  if (lds > 65536 && !raised) {
    const hipError_t e = allow_max_dynamic_lds(kern);
    if (e != hipSuccess) return e;
    raised = true;
  }
  const int blocks = grid > 0 ? grid : a.num;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * W), lds, s, a);
  return hipGetLastError();
}

template <int CRIT, int W>
int occupancy_mw(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain_mw<CRIT, W>, 64 * W, lds) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace

size_t plain_mw_lds(int slots, int max_items) {
  const size_t nch = ((size_t)max_items + 63) / 64;
  return (size_t)slots * 4 + (((size_t)slots * 2 + 15) & ~(size_t)15) + ((nch * 4 + 15) & ~(size_t)15);
}

hipError_t launch_plain_mw(const BatchArgs& a, int crit, int wpi, int grid, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  const size_t lds = plain_mw_lds(a.slots, a.max_items);
  if (wpi == 2) {
    if (crit == FF) return launch_mw<FF, 2>(a, lds, grid, s);
    if (crit == BF) return launch_mw<BF, 2>(a, lds, grid, s);
    return launch_mw<WF, 2>(a, lds, grid, s);
  }
  if (crit == FF) return launch_mw<FF, 4>(a, lds, grid, s);
  if (crit == BF) return launch_mw<BF, 4>(a, lds, grid, s);
  return launch_mw<WF, 4>(a, lds, grid, s);
}

int plain_mw_blocks_per_cu(int crit, int wpi, size_t lds) {
  if (wpi == 2) {
    if (crit == FF) return occupancy_mw<FF, 2>(lds);
    if (crit == BF) return occupancy_mw<BF, 2>(lds);
    return occupancy_mw<WF, 2>(lds);
  }
  if (crit == FF) return occupancy_mw<FF, 4>(lds);
  if (crit == BF) return occupancy_mw<BF, 4>(lds);
  return occupancy_mw<WF, 4>(lds);
}

}  // namespace vsbpp
