// Plain First/Best/Worst Fit (paper Section 1) with several instances per
// wavefront: the 64 lanes split into segments of SEG lanes (16 or 32), one
// instance per segment, all segments stepping through their item lists in
// lockstep.
//
// Per item the hot step is the same as in the one-instance-per-wavefront
// kernel -- every live bin of the segment's instance tests the item in
// parallel (Rule 4 applicability) and a reduction inside the segment picks
// the First/Best/Worst-Fit bin with the lowest position winning ties -- but
// one instruction stream now serves 64 / SEG instances.  The segment
// reduction is a DPP minimum inside one 16-lane row (plus one lane swizzle
// across rows for 32-lane segments) that leaves the result in every lane of
// the segment, so all per-instance state (item weight, chosen position, bin
// counts, cost) stays in vector registers and nothing goes through the
// scalar unit per instance.
//
// Keys: as in the one-wavefront kernel, a bin's key is (room << 16 | pos)
// for FF/BF and ((32767 - room) << 16 | pos) for WF, pos its position in the
// segment's creation-ordered list of live bins.  A group of 4*SEG positions
// sits in LDS so that lane l of the segment reads positions l, l+SEG,
// l+2SEG, l+3SEG of the group as one 16-byte word.  Every segment scans the
// same number of groups G (the largest live count in the wavefront); groups
// past a segment's own live count hold empty keys, which never fit.  Bins
// whose room is below the smallest weight still to come are dropped by a
// stable compaction at chunk boundaries (every 64 items), as before.
#include "device_common.h"
#include "kernels.h"

namespace vsbpp {
namespace {

constexpr int FF = 0, BF = 1, WF = 2;
constexpr uint32_t kR = 0x7FFFu;
constexpr uint32_t kTop = 0x80000000u;
constexpr uint32_t kPos = 0xFFFFu;

// minimum inside each SEG-lane segment, left in every lane of the segment
template <int SEG>
__device__ __forceinline__ uint32_t seg_min(uint32_t v) {
  constexpr uint32_t I = 0xFFFFFFFFu;
  v = min(v, dpp<kQuadSwap1>(I, v));
  v = min(v, dpp<kQuadSwap2>(I, v));
  v = min(v, dpp<kRowHalfMirror>(I, v));
  v = min(v, dpp<kRowMirror>(I, v));
  if constexpr (SEG == 32) {
    // lane i <-> lane i ^ 16 inside each 32-lane half (bit-mask swizzle:
    // and 0x1F, or 0, xor 0x10)
    v = min(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
  }
  return v;
}

template <int SEG>
__device__ __forceinline__ int32_t seg_min_i(int32_t v) {
  return (int32_t)(seg_min<SEG>((uint32_t)v ^ 0x80000000u) ^ 0x80000000u);
}

template <int SEG>
__device__ __forceinline__ int kidx(int p) {
  constexpr int GS = 4 * SEG;
  return (p & ~(GS - 1)) + ((p & (SEG - 1)) << 2) + ((p / SEG) & 3);
}

template <int CRIT>
__device__ __forceinline__ uint32_t empty_key() {
  return CRIT == WF ? ((kR << 16) | kPos) : 0u;
}

template <int CRIT>
__device__ __forceinline__ uint32_t room_of(uint32_t key) {
  return CRIT == WF ? kR - (key >> 16) : (key >> 16);
}

// LDS bytes of one segment: keys (u32) and position -> bin id map (u16) for
// `slots` positions, per-chunk suffix minima, the chunk's weights and the
// chunk's chosen positions.
__host__ __device__ inline size_t seg_bytes(int slots, int max_items) {
  const size_t nch = ((size_t)max_items + 63) / 64;
  size_t b = (size_t)slots * 4;
  b += ((size_t)slots * 2 + 15) & ~(size_t)15;
  b += (nch * 4 + 15) & ~(size_t)15;
  b += 64 * 4 + 64 * 4;
  return b;
}

template <int CRIT, int SEG>
__global__ void __launch_bounds__(256) k_plain_seg(BatchArgs a, int wpb, int64_t seg_stride) {
  constexpr int NSEG = kWave / SEG;
  constexpr int GS = 4 * SEG;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int ls = lane & (SEG - 1);
  const int sg = lane / SEG;
  const int wave = uniform((int)(threadIdx.x >> 6));
  const size_t nch_bytes = (((size_t)a.max_items + 63) / 64 * 4 + 15) & ~(size_t)15;
  unsigned char* base = smem + ((size_t)wave * NSEG + sg) * (size_t)seg_stride;
  uint32_t* keys = reinterpret_cast<uint32_t*>(base);
  uint16_t* pid = reinterpret_cast<uint16_t*>(base + (size_t)a.slots * 4);
  int32_t* smin = reinterpret_cast<int32_t*>(base + (size_t)a.slots * 4 +
                                             (((size_t)a.slots * 2 + 15) & ~(size_t)15));
  int32_t* wbuf = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(smin) + nch_bytes);
  int32_t* posbuf = wbuf + 64;
  uint32_t* const mine = keys + 4 * ls;
  // this lane's bits of a 64-lane ballot: the segment's, and those below it
  const uint64_t segbits = ((1ull << SEG) - 1ull) << (sg * SEG);
  const uint64_t below = segbits & ((1ull << lane) - 1ull);

  int cursor = blockIdx.x * wpb + wave;
  for (;;) {
    int first;
    if (a.queue) {
      int v = 0;
      if (lane == 0) v = atomicAdd(a.queue, NSEG);
      first = uniform(readlane(v, 0));
    } else {
      first = cursor * NSEG;
      cursor += gridDim.x * wpb;
    }
    if (first >= a.num) break;
    const int slot = first + sg;
    const bool have = slot < a.num;
    const int inst = have ? (a.sched ? a.sched[slot] : slot) : 0;
    // per-segment instance state (uniform inside the segment)
    int64_t off = 0;
    int m = 0, n = 0, err = 0;
    int32_t cap_lane = 0, B1 = 0;
    if (have) {
      off = a.item_off[inst];
      const int64_t m64 = a.item_off[inst + 1] - off;
      const int c0 = a.cap_off[inst];
      n = a.cap_off[inst + 1] - c0;
      if (m64 < 1 || m64 > a.max_items || n < 1 || n > kMaxTypes || n > a.max_types) {
        err = kErrSize;
      } else {
        m = (int)m64;
        cap_lane = ls < n ? a.caps[c0 + ls] : 0;
        const int32_t prev = (ls > 0 && ls < n) ? a.caps[c0 + ls - 1] : 0x7FFFFFFF;
        const bool bad = ls < n && (cap_lane <= 0 || cap_lane >= prev);
        if (ballot(bad) & segbits) err = kErrCaps;
        B1 = seg_min_i<SEG>(ls == 0 ? -cap_lane : 0x7FFFFFFF);
        B1 = -B1;
        if (!err && B1 > a.max_cap) err = kErrSize;
      }
    }
    // validation and per-chunk suffix minima of the weights in position order
    const int my_nch = err ? 0 : (m + 63) >> 6;
    const int nch = (int)~wave_min(~(uint32_t)my_nch);
    {
      bool badw = false, bado = false;
      int32_t run = 0x7FFFFFFF;
      for (int c = nch - 1; c >= 0; --c) {
        int32_t cmin = 0x7FFFFFFF;
#pragma unroll
        for (int i = 0; i < 64 / SEG; ++i) {
          const int q = (c << 6) + ls + SEG * i;
          if (q < m) {
            const int32_t wd = a.w[off + q];
            badw |= (wd < 1 || wd > B1);
            int32_t wq = wd;
            if (a.order) {
              int item = a.order[off + q];
              if ((unsigned)item >= (unsigned)m) {
                bado = true;
                item = q;
              }
              wq = a.w[off + item];
            }
            cmin = min(cmin, wq);
          }
        }
        run = min(run, seg_min_i<SEG>(cmin));
        if (ls == 0 && c < my_nch) smin[c] = run;
      }
      if (!err && (ballot(badw) & segbits)) err = kErrWeight;
      if (!err && (ballot(bado) & segbits)) err = kErrOption;
    }
    if (have && err && ls == 0) {
      a.nbins[inst] = err;
      a.cost[inst] = 0;
    }
    if (err) m = 0;
    const int nchw = (int)~wave_min(~(uint32_t)((m + 63) >> 6));

    int nlive = 0, nb = 0;
    int32_t cost = 0;  // m <= 65535 and B_1 <= 32767: the cost fits int32
    uint32_t minroom = 0xFFFFFFFFu;
    int32_t tprev = 0;
    int32_t typebuf = 0;
    int G = 0;  // groups every segment scans (wave-uniform)
    for (int c = 0; c < nchw; ++c) {
      const bool inchunk = (c << 6) < m;
      const int32_t T = inchunk ? smin[c] : 0x7FFFFFFF;
      const bool cmp = inchunk && nlive > 0 && (minroom < (uint32_t)T || T > tprev);
      if (ballot(cmp)) {
        // stable compaction of the live positions (room >= T) of the
        // segments that need it; the others are left as they are
        int newn = 0;
        for (int g = 0; g < G; ++g) {
          const uint4 kv = *reinterpret_cast<const uint4*>(mine + g * GS);
          const uint32_t k[4] = {kv.x, kv.y, kv.z, kv.w};
          uint16_t pv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pv[j] = pid[g * GS + j * SEG + ls];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int pos = g * GS + j * SEG + ls;
            const bool live = cmp && pos < nlive && room_of<CRIT>(k[j]) >= (uint32_t)T;
            const uint64_t lm = ballot(live);
            if (live) {
              const int np = newn + (int)__popcll(lm & below);
              keys[kidx<SEG>(np)] = (k[j] & ~kPos) | (uint32_t)np;
              pid[np] = pv[j];
            }
            newn += (int)__popcll(lm & segbits);
          }
        }
        // positions past the new count hold empty keys up to the scanned groups
        for (int g = 0; g < G; ++g) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int pos = g * GS + j * SEG + ls;
            if (cmp && pos >= newn) mine[g * GS + j] = empty_key<CRIT>();
          }
        }
        if (cmp) {
          nlive = newn;
          minroom = 0xFFFFFFFFu;
        }
        const uint32_t most = ~wave_min(~(uint32_t)nlive);
        G = (int)((most + GS - 1) / GS);
      }
      if (inchunk) tprev = T;
      // the chunk's weights (in position order) and their item ids
      int itm[64 / SEG];
#pragma unroll
      for (int i = 0; i < 64 / SEG; ++i) {
        const int q = (c << 6) + ls + SEG * i;
        int item = q;
        int32_t wv = 0;
        if (q < m) {
          if (a.order) item = a.order[off + q];
          wv = a.w[off + item];
        }
        itm[i] = item;
        wbuf[ls + SEG * i] = wv;
      }
      const int cnt = (int)~wave_min(~(uint32_t)max(0, min(64, m - (c << 6))));
      for (int jj = 0; jj < cnt; ++jj) {
        const int32_t w = wbuf[jj];
        const bool act = (c << 6) + jj < m;
        const uint32_t wk = (uint32_t)w << 16;
        uint32_t best = 0xFFFFFFFFu;
        auto cand = [&](uint32_t key) -> uint32_t {
          if constexpr (CRIT == FF) return key >= wk ? ((key >> 16) | (key << 16)) : 0xFFFFFFFFu;
          else if constexpr (CRIT == WF) return key + wk;
          else return key - wk;
        };
        int g = 0;
        for (; g + 1 < G; g += 2) {
          const uint4 k0 = *reinterpret_cast<const uint4*>(mine + g * GS);
          const uint4 k1 = *reinterpret_cast<const uint4*>(mine + (g + 1) * GS);
          best = min(best, min(cand(k0.x), cand(k1.x)));
          best = min(best, min(cand(k0.y), cand(k1.y)));
          best = min(best, min(cand(k0.z), cand(k1.z)));
          best = min(best, min(cand(k0.w), cand(k1.w)));
        }
        if (g < G) {
          const uint4 k0 = *reinterpret_cast<const uint4*>(mine + g * GS);
          best = min(best, min(cand(k0.x), cand(k0.y)));
          best = min(best, min(cand(k0.z), cand(k0.w)));
        }
        best = seg_min<SEG>(best);
        bool fit;
        int p;
        uint32_t nk;
        if constexpr (CRIT == FF) {
          fit = best != 0xFFFFFFFFu;
          p = (int)(best >> 16);
          nk = (((best & kPos) << 16) | (uint32_t)p) - wk;
        } else {
          fit = best < kTop;
          p = (int)(best & kPos);
          nk = best;
        }
        fit = fit && act;
        if (fit) {
          // Rule 4: place into the chosen open bin
          if (ls == (p & (SEG - 1))) keys[kidx<SEG>(p)] = nk;
          minroom = min(minroom, room_of<CRIT>(nk));
        }
        const bool open = act && !fit;
        if (ballot(open)) {
          // nothing fits: open a bin of type max{k : B_k >= w}, or B_1
          const bool holds = cap_lane >= w && ls < n;
          const int t = a.type_rule == 1 ? 0 : (int)__popcll(ballot(holds) & segbits) - 1;
          const int32_t Bt = a.type_rule == 1 ? B1 : seg_min_i<SEG>(holds ? cap_lane : 0x7FFFFFFF);
          const uint32_t room = (uint32_t)(Bt - w);
          const int np = nlive + (open ? 1 : 0);
          // a segment entering group G: every segment's group G becomes empty
          // first (each scans it from now on)
          if (ballot(np > G * GS)) {
            *reinterpret_cast<uint4*>(mine + G * GS) =
                make_uint4(empty_key<CRIT>(), empty_key<CRIT>(), empty_key<CRIT>(),
                           empty_key<CRIT>());
            G = uniform(G + 1);
          }
          if (open) {
            p = nlive;
            nlive = np;
            const uint32_t key = CRIT == WF ? (((kR - room) << 16) | (uint32_t)p)
                                            : ((room << 16) | (uint32_t)p);
            if (ls == (p & (SEG - 1))) {
              keys[kidx<SEG>(p)] = key;
              pid[p] = (uint16_t)nb;
            }
            typebuf = ls == (nb & (SEG - 1)) ? t : typebuf;
            if ((nb & (SEG - 1)) == SEG - 1) a.types[off + (nb - (SEG - 1)) + ls] = typebuf;
            nb += 1;
            cost += Bt;
            minroom = min(minroom, room);
          }
        }
        if (act && ls == 0) posbuf[jj] = p;
      }
      // assignments of the chunk: positions are stable until the next
      // compaction, so each item's bin id is read once here
#pragma unroll
      for (int i = 0; i < 64 / SEG; ++i) {
        const int q = (c << 6) + ls + SEG * i;
        if (q < m) a.assign[off + itm[i]] = (int32_t)pid[posbuf[ls + SEG * i]];
      }
    }
    if (m > 0) {
      if ((nb & (SEG - 1)) && ls < (nb & (SEG - 1))) a.types[off + (nb & ~(SEG - 1)) + ls] = typebuf;
      if (ls == 0) {
        a.nbins[inst] = nb;
        a.cost[inst] = cost;
      }
    }
  }
}

template <int CRIT, int SEG>
hipError_t launch_seg(const BatchArgs& a, int wpb, int64_t seg_stride, int grid, hipStream_t s) {
  constexpr int NSEG = kWave / SEG;
  const size_t lds = (size_t)seg_stride * NSEG * (size_t)wpb;
  auto kern = k_plain_seg<CRIT, SEG>;
  static bool raised = false;
  if (lds > 65536 && !raised) {
    hipError_t e = allow_max_dynamic_lds(kern);
    if (e != hipSuccess) return e;
    raised = true;
  }
  const int waves = (a.num + NSEG - 1) / NSEG;
  const int blocks = grid > 0 ? grid : (waves + wpb - 1) / wpb;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, s, a, wpb, seg_stride);
  return hipGetLastError();
}

template <int CRIT, int SEG>
int seg_occupancy(int wpb, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain_seg<CRIT, SEG>, 64 * wpb, lds) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace

size_t plain_seg_stride(int slots, int max_items) {
  return (seg_bytes(slots, max_items) + 15) & ~(size_t)15;
}

hipError_t launch_plain_seg(const BatchArgs& a, int crit, int seg, int wpb, size_t seg_stride,
                            int grid, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  const int64_t st = (int64_t)seg_stride;
  if (seg == 16) {
    if (crit == FF) return launch_seg<FF, 16>(a, wpb, st, grid, s);
    if (crit == BF) return launch_seg<BF, 16>(a, wpb, st, grid, s);
    return launch_seg<WF, 16>(a, wpb, st, grid, s);
  }
  if (crit == FF) return launch_seg<FF, 32>(a, wpb, st, grid, s);
  if (crit == BF) return launch_seg<BF, 32>(a, wpb, st, grid, s);
  return launch_seg<WF, 32>(a, wpb, st, grid, s);
}

int plain_seg_blocks_per_cu(int crit, int seg, int wpb, size_t seg_stride) {
  const size_t lds = seg_stride * (size_t)(kWave / seg) * (size_t)wpb;
  if (seg == 16) {
    if (crit == FF) return seg_occupancy<FF, 16>(wpb, lds);
    if (crit == BF) return seg_occupancy<BF, 16>(wpb, lds);
    return seg_occupancy<WF, 16>(wpb, lds);
  }
  if (crit == FF) return seg_occupancy<FF, 32>(wpb, lds);
  if (crit == BF) return seg_occupancy<BF, 32>(wpb, lds);
  return seg_occupancy<WF, 32>(wpb, lds);
}

}  // namespace vsbpp
