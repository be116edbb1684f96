// The two hybrid-P-system heuristics (paper Sections 6.3 and 6.4).
//
// One workgroup per instance; every thread is one packer of the P system:
//   H1: thread <-> sublist S_I (s1 consecutive positions of the Rule-1 order);
//   H2: thread <-> (subset I, permutation rank r); a group of
//       roundup(S!, 64) threads covers the S! permutations of one subset and a
//       group minimum of (cost, r) picks the subset's packing.
// A packer starts with one empty bin of each type (Rule 2), takes its items in
// order (Rule 3, criterion drawn per placement), places each by FF/BF/WF among
// the bins it fits (Rule 4, lowest index on ties), opens a bin of the chosen
// type when none fits, and divides a bin once when its load reaches half its
// capacity (Rule 5).
//
// Packer bins live in LDS, per thread: words of bin b of thread t sit at
// (b >> 2) * 4*blockDim + 4*t + (b & 3), so one 16-byte load per lane reads
// four bins and lanes are unit-stride.  Output bin ids are canonical: used
// bins (load > 0) in creation order, packers in sublist/subset order; the
// per-instance id offsets come from a block scan over the packers.
#include <type_traits>

#include "device_common.h"
#include "kernels.h"
#include "block_common.h"

namespace vsbpp {
namespace {

constexpr int FF = 0, BF = 1, WF = 2;

template <typename K>
struct PK;
template <>
struct PK<uint32_t> {
  static constexpr int SH = 16;
  static constexpr int32_t R = 0x7FFF;
  static constexpr uint32_t TOP = 0x80000000u;
};
template <>
struct PK<uint64_t> {
  static constexpr int SH = 32;
  static constexpr int32_t R = 0x7FFFFFFF;
  static constexpr uint64_t TOP = 0x8000000000000000ull;
};

// Per-thread packer over LDS-resident bins.  With 32-bit keys (B_1 <= 32767)
// a bin is one word (capacity << 16 | room); with 64-bit keys room and
// capacity are two words in two arrays.  An empty slot (no bin) has room 0
// and capacity 0 (packed) or room -1 (split), so no item fits it.
template <typename K>
struct LanePacker {
  static constexpr bool kPacked = sizeof(K) == 4;
  int32_t* room;  // this thread's words (bin b at (b>>2)*stride + (b&3))
  int32_t* cap;   // split layout only
  int stride;     // 4 * blockDim
  uint64_t div;   // Rule-5 "already divided" marks
  int nb;

  __device__ __forceinline__ int widx(int b) const { return (b >> 2) * stride + (b & 3); }
  __device__ __forceinline__ int32_t room_at(int b) const {
    return kPacked ? (room[widx(b)] & 0xFFFF) : room[widx(b)];
  }
  __device__ __forceinline__ int32_t cap_at(int b) const {
    return kPacked ? (int32_t)((uint32_t)room[widx(b)] >> 16) : cap[widx(b)];
  }
  __device__ __forceinline__ void set_bin(int b, int32_t c, int32_t r) {
    if constexpr (kPacked) {
      room[widx(b)] = (int32_t)(((uint32_t)c << 16) | (uint32_t)r);
    } else {
      room[widx(b)] = r;
      cap[widx(b)] = c;
    }
  }

  // Rule 2: one empty bin per type, B_1 first (or B_n first with rev);
  // slots [n, nbslots) hold no bin.
  __device__ void init(const int32_t* scaps, int n, int nbslots, int rev) {
    for (int g = 0; g < (nbslots >> 2); ++g) {
      int4 r, c;
      int* rp = &r.x;
      int* cp = &c.x;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = (g << 2) + j;
        const int32_t v = b < n ? scaps[rev ? n - 1 - b : b] : 0;
        if constexpr (kPacked) {
          rp[j] = (int32_t)(((uint32_t)v << 16) | (uint32_t)v);
        } else {
          cp[j] = v;
          rp[j] = b < n ? v : -1;
        }
      }
      *reinterpret_cast<int4*>(room + g * stride) = r;
      if constexpr (!kPacked) *reinterpret_cast<int4*>(cap + g * stride) = c;
    }
    div = 0;
    nb = n;
  }

  // Places weight w with criterion crit; nbound is a wave-uniform upper bound
  // on nb.  Returns the bin index used.
  __device__ int place(int32_t w, int crit, int nbound, const int32_t* scaps, int n,
                       int type_rule) {
    using T = PK<K>;
    const int32_t mul = crit == BF ? 1 : (crit == WF ? -1 : 0);
    const int32_t add = crit == WF ? T::R : 0;
    K best = ~(K)0;
    const int ng = (nbound + 3) >> 2;
    for (int g = 0; g < ng; ++g) {
      const int4 r4 = *reinterpret_cast<const int4*>(room + g * stride);
      const int* rp = &r4.x;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t rm = kPacked ? (rp[j] & 0xFFFF) : rp[j];
        const int32_t after = rm - w;
        const int32_t sel = mul * after + add;
        K key = ((K)(uint32_t)sel << T::SH) | (K)((g << 2) + j);
        if (after < 0) key |= T::TOP;
        best = min(best, key);
      }
    }
    return apply(best < T::TOP ? (int)(best & (K)0xFF) : -1, w, scaps, n, type_rule);
  }

  // The bins First, Best and Worst Fit would choose for weight w (-1 when
  // nothing fits; lowest index on ties), the number of bins it fits, and the
  // room each choice leaves.  nbound as for place.
  __device__ void choices(int32_t w, int nbound, int* bff, int* bbf, int* bwf, int* nfit,
                          int32_t* aff, int32_t* abf, int32_t* awf) const {
    using T = PK<K>;
    K kb = ~(K)0, kw = ~(K)0;
    int f = 0x7FFFFFFF, cnt = 0;
    const int ng = (nbound + 3) >> 2;
    for (int g = 0; g < ng; ++g) {
      const int4 r4 = *reinterpret_cast<const int4*>(room + g * stride);
      const int* rp = &r4.x;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t rm = kPacked ? (rp[j] & 0xFFFF) : rp[j];
        const int32_t after = rm - w;
        const int idx = (g << 2) + j;
        const bool fits = after >= 0;
        cnt += fits ? 1 : 0;
        f = min(f, fits ? idx : 0x7FFFFFFF);
        kb = min(kb, fits ? ((K)(uint32_t)after << T::SH) | (K)idx : ~(K)0);
        kw = min(kw, fits ? ((K)(uint32_t)(T::R - after) << T::SH) | (K)idx : ~(K)0);
      }
    }
    *nfit = cnt;
    if (cnt == 0) {
      *bff = *bbf = *bwf = -1;
      return;
    }
    *bff = f;
    *bbf = (int)(kb & (K)0xFF);
    *bwf = (int)(kw & (K)0xFF);
    *aff = room_at(f) - w;
    *abf = (int32_t)(kb >> T::SH);
    *awf = T::R - (int32_t)(kw >> T::SH);
  }

  // Puts weight w into bin b (b < 0: a new bin of the smallest type holding
  // w, or B_1), then Rule 5.  Returns the bin index used.
  __device__ int apply(int b, int32_t w, const int32_t* scaps, int n, int type_rule) {
    int32_t bcap, broom;
    if (b >= 0) {
      broom = room_at(b);
      bcap = cap_at(b);
    } else {
      // nothing fits: open a bin (smallest capacity >= w, or B_1)
      int t = 0;
      if (type_rule != 1)
        for (int k = 1; k < n; ++k) t += scaps[k] >= w ? 1 : 0;
      bcap = scaps[t];
      broom = bcap;
      b = nb++;
    }
    broom -= w;
    set_bin(b, bcap, broom);
    // Rule 5: a bin at least half full divides once
    if (!((div >> b) & 1ull) && 2ll * (bcap - broom) >= (long long)bcap) {
      div |= 1ull << b;
      set_bin(nb, bcap, bcap);
      ++nb;
    }
    return b;
  }

  // bins with load > 0, as a bit mask over bin indices, and their cost
  __device__ uint64_t used(int64_t* cost) const {
    uint64_t u = 0;
    int64_t c = 0;
    for (int b = 0; b < nb; ++b) {
      const int32_t cb = cap_at(b);
      if (room_at(b) < cb) {
        u |= 1ull << b;
        c += cb;
      }
    }
    *cost = c;
    return u;
  }

  __device__ int type_of(int b, const int32_t* scaps, int n) const {
    const int32_t cb = cap_at(b);
    int t = 0;
    for (int k = 0; k < n; ++k)
      if (scaps[k] == cb) t = k;
    return t;
  }
};

// block-wide exclusive scan of v; returns the prefix and writes the total
__device__ int32_t block_excl_scan(int32_t v, int32_t* s_tmp, int32_t* total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int32_t incl = wave_incl_sum(v);
  if (lane == kWave - 1) s_tmp[wave] = incl;
  __syncthreads();
  int32_t before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const int32_t x = s_tmp[i];
    before += i < wave ? x : 0;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

__device__ int64_t block_sum64(int64_t v, int64_t* s_tmp) {
  const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
  if (lane == 0) s_tmp[wave] = v;
  __syncthreads();
  int64_t t = 0;
  for (int i = 0; i < nw; ++i) t += s_tmp[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint64_t inst_seed(const BatchArgs& a, int inst) {
  return a.seeds ? a.seeds[inst] : a.seed;
}

// ---------------------------------------------------------------------------
// Learned criterion of the first heuristic: a network scores FF, BF and WF
// where they would put the item into different bins (Rule 3's draw stands
// where they agree, where nothing fits, and for non-finite scores).  Every
// lane evaluates the network for its own packer: the weights sit in LDS as
// fp32 and every lane reads the same word (a broadcast), the first hidden
// layer is held in registers, and each second-layer unit, once formed, is
// folded into the three output chains in unit order -- so every unit is its
// bias followed by one fp32 fused-multiply-add chain over its inputs in
// index order.
// ---------------------------------------------------------------------------
struct H1Model {
  float w1[64 * 16];  // [l][i]
  float w2[64 * 64];  // [l][j]
  float w3[3 * 64];   // [k][j]
  float b1[64], b2[64], b3[4];
  int32_t n_out;
};
constexpr size_t kH1ModelBytes = (sizeof(H1Model) + 15) & ~(size_t)15;

__device__ __forceinline__ float bf16v(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

__device__ void stage_h1_model(const vsbpp_model* m, H1Model* s) {
  for (int e = threadIdx.x; e < 64 * 16; e += blockDim.x) s->w1[e] = bf16v(m->w1[e]);
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) s->w2[e] = bf16v(m->w2[e]);
  for (int e = threadIdx.x; e < 3 * 64; e += blockDim.x) s->w3[e] = bf16v(m->w3[e]);
  for (int e = threadIdx.x; e < 64; e += blockDim.x) {
    s->b1[e] = m->b1[e];
    s->b2[e] = m->b2[e];
    if (e < 3) s->b3[e] = m->b3[e];
  }
  if (threadIdx.x == 0) s->n_out = m->n_out;
}

// the criterion the network picks for features x, or `drawn`
__device__ int h1_score(const H1Model* md, const float (&x)[16], int drawn) {
  float h1[64];
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    float acc = md->b1[l];
#pragma unroll
    for (int i = 0; i < 16; i += 4) {
      const float4 wv = *reinterpret_cast<const float4*>(&md->w1[l * 16 + i]);
      acc = __builtin_fmaf(wv.x, x[i], acc);
      acc = __builtin_fmaf(wv.y, x[i + 1], acc);
      acc = __builtin_fmaf(wv.z, x[i + 2], acc);
      acc = __builtin_fmaf(wv.w, x[i + 3], acc);
    }
    h1[l] = acc > 0.0f ? acc : 0.0f;
  }
  float z0 = md->b3[0], z1 = md->b3[1], z2 = md->b3[2];
  for (int l = 0; l < 64; ++l) {
    float acc = md->b2[l];
#pragma unroll
    for (int j = 0; j < 64; j += 4) {
      const float4 wv = *reinterpret_cast<const float4*>(&md->w2[l * 64 + j]);
      acc = __builtin_fmaf(wv.x, h1[j], acc);
      acc = __builtin_fmaf(wv.y, h1[j + 1], acc);
      acc = __builtin_fmaf(wv.z, h1[j + 2], acc);
      acc = __builtin_fmaf(wv.w, h1[j + 3], acc);
    }
    const float h2 = acc > 0.0f ? acc : 0.0f;
    z0 = __builtin_fmaf(md->w3[l], h2, z0);
    z1 = __builtin_fmaf(md->w3[64 + l], h2, z1);
    z2 = __builtin_fmaf(md->w3[128 + l], h2, z2);
  }
  if (!(__builtin_isfinite(z0) && __builtin_isfinite(z1) && __builtin_isfinite(z2))) return drawn;
  int c = 0;
  float zc = z0;
  if (z1 > zc) {
    c = 1;
    zc = z1;
  }
  if (z2 > zc) c = 2;
  return c;
}

// ---------------------------------------------------------------------------
// First heuristic (Section 6.3).  LC: the learned-criterion variant (the
// criterion scored by the network when criterion_rule is 1, and the features
// of every contested placement dumped when asked).
// ---------------------------------------------------------------------------
template <typename K, bool LC>
__global__ void __launch_bounds__(LC ? kH1LearnedMaxBlock : 1024) k_h1(BatchArgs a, int nbslots) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_caps[kMaxTypes];
  __shared__ int32_t s_scan[16];
  __shared__ int64_t s_sum[16];
  __shared__ int s_flag;
  const int tid = threadIdx.x, B = blockDim.x;
  constexpr int kArrays = sizeof(K) == 4 ? 1 : 2;
  H1Model* md = reinterpret_cast<H1Model*>(smem);
  bool model_ok = true;
  if constexpr (LC) {
    if (a.criterion_rule == 1) {
      stage_h1_model(a.model, md);
      __syncthreads();
      model_ok = md->n_out >= 3 && md->n_out <= kMaxTypes;
    }
  }
  int32_t* lroom = reinterpret_cast<int32_t*>(smem + (LC ? kH1ModelBytes : 0));
  int32_t* lcap = lroom + (size_t)nbslots * B;
  int32_t* litem = lroom + (size_t)kArrays * nbslots * B;  // [s1][B]
  uint8_t* lloc = reinterpret_cast<uint8_t*>(litem + (size_t)a.s1 * B);  // [s1][B]

  LanePacker<K> pk;
  pk.room = lroom + 4 * tid;
  pk.cap = lcap + 4 * tid;
  pk.stride = 4 * B;

  __shared__ int s_slot;
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
    int err = m64 > a.max_items ? kErrSize
                                 : validate_block(a, inst, off, m, c0, n, s_caps, &s_flag);
    if (!err && !model_ok) err = kErrModel;
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      __syncthreads();
      continue;
    }
    const uint64_t seed = inst_seed(a, inst);
    Rule1Perm perm;
    perm.init(seed, (uint32_t)m);
    const uint64_t ck = stream_key(seed, kStreamH1);
    const int s1 = a.s1;
    const float inv_b1 = 1.0f / (float)s_caps[0];
    const int l = (m + s1 - 1) / s1;
    int32_t carry = 0;
    int64_t cost_acc = 0;
    for (int base_I = 0; base_I < l; base_I += B) {
      const int I = base_I + tid;
      const bool active = I < l;
      const int q0 = I * s1;
      const int k = active ? min(s1, m - q0) : 0;
      if (active) pk.init(s_caps, n, nbslots, a.rule2_order);
      for (int t = 0; t < s1; ++t) {
        if (t < k) {
          const int q = q0 + t;
          const int item = a.order ? a.order[off + q] : (int)perm.at((uint32_t)q);
          const int32_t w = a.w[off + item];
          int crit = a.force_crit >= 0 ? a.force_crit : draw_criterion(ck, (uint64_t)q);
          int b;
          if constexpr (LC) {
            int bff, bbf, bwf, nfit;
            int32_t aff = 0, abf = 0, awf = 0;
            pk.choices(w, min(nbslots, n + 2 * t), &bff, &bbf, &bwf, &nfit, &aff, &abf, &awf);
            const bool contested = nfit > 0 && !(bff == bbf && bbf == bwf);
            if (contested) {
              float x[16];
#pragma unroll
              for (int i = 7; i < 16; ++i) x[i] = 0.0f;
              x[0] = (float)w * inv_b1;
              x[1] = (float)t * (1.0f / (float)k);
              x[2] = (float)aff * inv_b1;
              x[3] = (float)abf * inv_b1;
              x[4] = (float)awf * inv_b1;
              x[5] = (float)nfit * (1.0f / 16.0f);
              x[6] = (float)pk.nb * (1.0f / 32.0f);
              if (a.criterion_rule == 1) crit = h1_score(md, x, crit);
              if (a.feat_out) {
                float4* fo = reinterpret_cast<float4*>(a.feat_out + 16 * (off + q));
                fo[0] = make_float4(x[0], x[1], x[2], x[3]);
                fo[1] = make_float4(x[4], x[5], x[6], 0.0f);
                fo[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                fo[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
              }
            }
            if (a.info_out) a.info_out[off + q] = contested ? 1 : 0;
            b = pk.apply(nfit == 0 ? -1 : (crit == 0 ? bff : (crit == 1 ? bbf : bwf)), w,
                         s_caps, n, a.type_rule);
          } else {
            b = pk.place(w, crit, min(nbslots, n + 2 * t), s_caps, n, a.type_rule);
          }
          litem[t * B + tid] = item;
          lloc[t * B + tid] = (uint8_t)b;
        }
      }
      int64_t c = 0;
      uint64_t u = 0;
      if (active) u = pk.used(&c);
      int32_t total;
      const int32_t before = block_excl_scan((int32_t)__popcll(u), s_scan, &total);
      const int32_t gbase = carry + before;
      if (active) {
        for (int t = 0; t < k; ++t) {
          const int b = lloc[t * B + tid];
          const int rank = (int)__popcll(u & ((1ull << b) - 1ull));
          a.assign[off + litem[t * B + tid]] = gbase + rank;
        }
        uint64_t uu = u;
        int r = 0;
        while (uu) {
          const int b = __builtin_ctzll(uu);
          uu &= uu - 1;
          a.types[off + gbase + r] = pk.type_of(b, s_caps, n);
          ++r;
        }
      }
      carry += total;
      cost_acc += block_sum64(c, s_sum);
    }
    if (tid == 0) {
      a.nbins[inst] = carry;
      a.cost[inst] = cost_acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Second heuristic (Section 6.4)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int factorial_small(int k) {
  int f = 1;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// r-th permutation of 0..k-1 in lexicographic order, as 4-bit digits
// (digit t = the item placed t-th).
__device__ __forceinline__ uint32_t nth_perm(int r, int k) {
  uint32_t avail = 0x543210u;
  uint32_t out = 0;
  for (int t = 0; t < k; ++t) {
    const int f = factorial_small(k - 1 - t);
    const int d = r / f;
    r -= d * f;
    const uint32_t v = (avail >> (4 * d)) & 0xFu;
    const uint32_t lowmask = (1u << (4 * d)) - 1u;
    avail = (avail & lowmask) | ((avail >> (4 * d + 4)) << (4 * d));
    out |= v << (4 * t);
  }
  return out;
}

constexpr int kMaxSubset = 6;

// H2 over LanePacker bins for wide batches (B_1 > 32767 or more than 65535
// items: 64-bit keys); narrower batches take k_h2s below.
template <typename K>
__global__ void __launch_bounds__(1024) k_h2(BatchArgs a, int nbslots, int group) {
  static_assert(sizeof(K) == 8, "k_h2 runs wide batches only");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_caps[kMaxTypes];
  using GK = typename std::conditional<sizeof(K) == 4, uint32_t, uint64_t>::type;
  constexpr int kRankBits = sizeof(K) == 4 ? 10 : 16;
  __shared__ GK s_wmin[16];
  __shared__ int s_flag;
  const int tid = threadIdx.x, B = blockDim.x;
  const int spr = B / group;  // subsets per round
  constexpr int kArrays = sizeof(K) == 4 ? 1 : 2;
  int32_t* lroom = reinterpret_cast<int32_t*>(smem);
  int32_t* lcap = lroom + (size_t)nbslots * B;
  int32_t* s_item = lroom + (size_t)kArrays * nbslots * B;  // [spr][6]
  int32_t* s_w = s_item + spr * kMaxSubset;                // [spr][6]
  int32_t* s_loc = s_w + spr * kMaxSubset;                 // [spr][6] canonical local id
  int32_t* s_typ = s_loc + spr * kMaxSubset;               // [spr][6]
  int32_t* s_u = s_typ + spr * kMaxSubset;                 // [spr]
  int32_t* s_base = s_u + spr;                             // [spr]
  int64_t* s_cst = reinterpret_cast<int64_t*>(s_base + spr);  // [spr], 8-byte aligned

  LanePacker<K> pk;
  pk.room = lroom + 4 * tid;
  pk.cap = lcap + 4 * tid;
  pk.stride = 4 * B;
  const int g = tid / group, r = tid - g * group;
  const int lane = lane_id(), wave = tid >> 6, wpg = group >> 6;

  __shared__ int s_slot;
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
    const int err = m64 > a.max_items ? kErrSize
                                       : validate_block(a, inst, off, m, c0, n, s_caps, &s_flag);
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      __syncthreads();
      continue;
    }
    const uint64_t seed = inst_seed(a, inst);
    Rule1Perm perm;
    perm.init(seed, (uint32_t)m);
    const uint64_t ck = stream_key(seed, kStreamH2);
    const int S = min(a.s2, m);
    const int P = factorial_small(S);
    const int l = (m + S - 1) / S;
    // permutation of rank r of a full subset (the same for every subset)
    const uint32_t pm_full = r < P ? nth_perm(r, S) : 0u;
    int32_t carry = 0;
    int64_t cost_acc = 0;
    for (int base_I = 0; base_I < l; base_I += spr) {
      const int I = base_I + g;
      const int q0 = I * S;
      const int k = I < l ? min(S, m - q0) : 0;
      const int kf = factorial_small(k);
      const bool active = k > 0 && r < kf;
      // stage the subset's items
      if (r < k) {
        const int q = q0 + r;
        const int item = a.order ? a.order[off + q] : (int)perm.at((uint32_t)q);
        s_item[g * kMaxSubset + r] = item;
        s_w[g * kMaxSubset + r] = a.w[off + item];
      }
      __syncthreads();
      GK key = ~(GK)0;
      uint64_t locs = 0;
      uint64_t u = 0;
      int64_t c = 0;
      if (active) {
        pk.init(s_caps, n, nbslots, a.rule2_order);
        const uint32_t pm = k == S ? pm_full : nth_perm(r, k);
        uint32_t cu = digits_word(ck, (uint64_t)I * (uint64_t)P + (uint64_t)r);
        for (int t = 0; t < k; ++t) {
          const int d = (pm >> (4 * t)) & 0xF;
          const int32_t w = s_w[g * kMaxSubset + d];
          const int drawn = digits_next(cu);
          const int crit = a.force_crit >= 0 ? a.force_crit : drawn;
          const int b = pk.place(w, crit, min(nbslots, n + 2 * t), s_caps, n, a.type_rule);
          locs |= (uint64_t)b << (6 * d);
        }
        u = pk.used(&c);
        key = ((GK)c << kRankBits) | (GK)r;
      }
      // group minimum of (cost, rank): lowest rank on ties
      GK gm = wave_min(key);
      if (wpg > 1) {
        if (lane == 0) s_wmin[wave] = gm;
        __syncthreads();
        gm = ~(GK)0;
        for (int i = 0; i < wpg; ++i) gm = min(gm, s_wmin[g * wpg + i]);
      }
      if (active && key == gm) {
        for (int d = 0; d < k; ++d) {
          const int b = (int)((locs >> (6 * d)) & 63u);
          s_loc[g * kMaxSubset + d] = (int)__popcll(u & ((1ull << b) - 1ull));
        }
        uint64_t uu = u;
        int rr = 0;
        while (uu) {
          const int b = __builtin_ctzll(uu);
          uu &= uu - 1;
          s_typ[g * kMaxSubset + rr] = pk.type_of(b, s_caps, n);
          ++rr;
        }
        s_u[g] = rr;
        s_cst[g] = c;
      }
      if (r == 0 && k == 0) {
        s_u[g] = 0;
        s_cst[g] = 0;
      }
      __syncthreads();
      if (tid == 0) {
        int32_t run = carry;
        for (int i = 0; i < spr; ++i) {
          s_base[i] = run;
          run += s_u[i];
          cost_acc += s_cst[i];
        }
        carry = run;
      }
      __syncthreads();
      if (r < k) {
        a.assign[off + s_item[g * kMaxSubset + r]] = s_base[g] + s_loc[g * kMaxSubset + r];
      }
      if (r < s_u[g] && k > 0) {
        a.types[off + s_base[g] + r] = s_typ[g * kMaxSubset + r];
      }
      __syncthreads();
    }
    if (tid == 0) {
      a.nbins[inst] = carry;
      a.cost[inst] = cost_acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Second heuristic with 32-bit bin words (B_1 <= 32767), the common case.
//
// Bin b of lane l of wavefront v is one word of the workgroup's LDS array A,
// at (v * nbslots + b) * 64 + l, with the bin's type k < 32:
//   A = room << 10 | b << 5 | k.
// Slot b of a lane is 64 words (256 bytes) past its slot 0, so its address
// is one shift-add, two slots are one ds_read2st64, and every lane of a wave
// reads and writes its own bank whatever slot it addresses.
// The candidate key of weight w in bin b (W10 = w << 10, R = 32767):
//   BF: A - W10                  least room after, then lowest b; a bin the
//                                item does not fit wraps to >= 2^31
//   WF: (A ^ ~1023) + XW         = (R - room + w) << 10 | b << 5 | k: most
//                                room after, then lowest b; no fit >= 2^25.
//                                The xor turns room into 2^22-1 - room and
//                                XW = (R + w - (2^22-1)) << 10 shifts it back
//   FF: (A - W10) & (2^31|1023)  b << 5 | k, or >= 2^31
// All three are ((A ^ s) + x) & mask, one xor-add and one mask per bin with
// per-lane s, x and mask.  Every fitting key is below 2^25 and every other
// one is not, so the least key also names the bin's type.  Slots without a
// bin hold room 0 (A = b << 5): nothing fits them.  The used-bin mask and
// the cost are kept as the items go, so a packer needs no final pass over
// its bins.
//
// Rule-1 positions, their weights and the bin each item opens when nothing
// fits are resolved a chunk of rounds at a time by the whole workgroup, and
// every packer starts from a per-instance template of its Rule-2 bins.  The
// first placement of a packing meets only those bins, so the chunk step also
// records, per position and criterion, the bin it takes there: a packing's
// first item needs no scan.  A
// round (spr subsets) needs two barriers: one for the group minimum, one
// before the bin counts of all groups are read.  The winner's own wave then
// writes its assignment and bin types, one lane per item and one per bin,
// reading the winner's bins from LDS: in program order before that wave's
// next round overwrites them, and no other wave writes them.
// ---------------------------------------------------------------------------
constexpr int32_t kR5 = 32767;

// slot b of the packer whose slot 0 is `first`
__device__ __forceinline__ int32_t* slot_at(int32_t* first, int b) { return first + 64 * b; }

// At most 64 VGPRs: eight wavefronts per SIMD instead of seven at 65.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_h2s(BatchArgs a, int nbslots, int group) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) int32_t s_caps[kMaxTypes];
  // per criterion c, the constants of its key ((A ^ s) + x) & mask with
  // x = (W10 ^ nm) + ad: {s, nm, ad, mask}, one 16-byte read per placement
  __shared__ __align__(16) uint32_t s_keyc[4 * 3];
  // per bin type k: {B_k, the word of an empty bin of type k in slot 0
  // (B_k << 10 | k), (floor(B_k / 2) + 1) << 10, 0}
  __shared__ __align__(16) int4 s_type[kMaxTypes];
  __shared__ uint32_t s_wmin[16];
  __shared__ int s_flag;
  __shared__ int s_slot;
  const int tid = threadIdx.x, B = blockDim.x;
  const int spr = B / group;  // subsets per round
  int32_t* arrA = reinterpret_cast<int32_t*>(smem);
  int32_t* tmplA = arrA + (size_t)nbslots * B;  // [nbslots]
  // [B] per chunk position: the first placement's bin for each criterion
  // (below)
  uint32_t* s_first = reinterpret_cast<uint32_t*>(tmplA + nbslots);
  // [B] per chunk position: {w << 10, the type of the bin the item opens
  // when nothing fits | item << 5}, one 8-byte read per placement
  int2* s_cwt = reinterpret_cast<int2*>(s_first + B);
  int32_t* s_u = tmplA + nbslots + 3 * B;       // [spr] used bins
  int32_t* s_cst = s_u + spr;                   // [spr] subset cost
  int32_t* myA = arrA + ((tid >> 6) * nbslots) * 64 + (tid & 63);
  const int g = tid / group, r = tid - g * group;
  const int lane = lane_id(), wave = tid >> 6, wpg = group >> 6;
  // this packer's part of its generator state: output I * P + r of the H2
  // stream has state key + (I * P + r + 1) * gamma, whose part
  // (r + 1) * gamma is fixed for the thread (kept opaque, so that the
  // compiler does not fold the two products back into one per round)
  uint64_t st_lane = (uint64_t)(r + 1) * kGolden;
  asm volatile("" : "+v"(st_lane));
  if (tid < 12) {
    const int c = tid >> 2, f = tid & 3;
    const bool wf = c == WF;
    const uint32_t v = f == 0   ? (wf ? 0xFFFFFC00u : 0u)
                       : f == 1 ? (wf ? 0u : 0xFFFFFFFFu)
                       : f == 2 ? (wf ? (uint32_t)(kR5 - 0x3FFFFF) << 10 : 1u)
                                : (c == FF ? 0x800003FFu : 0xFFFFFFFFu);
    s_keyc[tid] = v;
  }
  __syncthreads();

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
    const int err = m64 > a.max_items ? kErrSize
                                       : validate_block(a, inst, off, m, c0, n, s_caps, &s_flag);
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      __syncthreads();
      continue;
    }
    // Rule 2 template: bins 0..n-1 empty with their capacity as room, in
    // type order (B_1 first) or increasing capacity (B_n first)
    if (tid < nbslots) {
      const int ty = a.rule2_order ? n - 1 - tid : tid;
      const int32_t room = tid < n ? s_caps[ty] : 0;
      tmplA[tid] = (room << 10) | (tid << 5) | (tid < n ? ty : 0);
    }
    if (tid < n)
      s_type[tid] = make_int4(s_caps[tid], (s_caps[tid] << 10) | tid,
                              ((s_caps[tid] >> 1) + 1) << 10, 0);
    const uint64_t seed = inst_seed(a, inst);
    Rule1Perm perm;
    perm.init(seed, (uint32_t)m);
    const uint64_t ck = stream_key(seed, kStreamH2);
    const int S = min(a.s2, m);
    const int P = factorial_small(S);
    const int l = (m + S - 1) / S;
    const int per_round = spr * S;
    const int chunk_rounds = B / per_round;  // >= 1: group >= 64 >= S
    const uint32_t pm_full = r < P ? nth_perm(r, S) : 0u;
    int32_t carry = 0;
    int64_t cost_acc = 0;
    int cq = 0;  // first position of the current chunk
    for (int base_I = 0, rnd = 0; base_I < l; base_I += spr, ++rnd) {
      if (rnd % chunk_rounds == 0) {
        // resolve the chunk's positions: item ids and weights
        __syncthreads();
        cq = base_I * S;
        const int q = cq + tid;
        if (tid < chunk_rounds * per_round && q < m) {
          const int item = a.order ? a.order[off + q] : (int)perm.at((uint32_t)q);
          const int32_t w = a.w[off + item];
          // the bin this item opens when nothing fits: the smallest capacity
          // >= w (the capacities decrease, so the last of those), or B_1
          int t = 0;
          if (a.type_rule != 1)
            for (int kk = 1; kk < n; ++kk) t += s_caps[kk] >= w ? 1 : 0;
          // item < 2^16: this kernel takes instances of at most 65535 items
          s_cwt[tid] = make_int2(w << 10, t | (item << 5));
          // Its first placement in any permutation finds the Rule-2 bins
          // of the template, and B_1 among them holds it (no weight exceeds
          // B_1): per criterion c, the low ten bits (slot << 5 | type) of the
          // least key over those bins, at bit 10c.
          uint32_t f = 0;
          for (int c = 0; c < 3; ++c) {
            const uint32_t xx = ((uint32_t)(w << 10) ^ s_keyc[4 * c + 1]) + s_keyc[4 * c + 2];
            uint32_t best = 0xFFFFFFFFu;
            for (int b = 0; b < n; ++b)
              best = min(best, (((uint32_t)tmplA[b] ^ s_keyc[4 * c]) + xx) & s_keyc[4 * c + 3]);
            f |= (best & 1023u) << (10 * c);
          }
          s_first[tid] = f;
        }
        __syncthreads();
      }
      // a group is a whole number of wavefronts, so the subset, its size
      // and its permutation count are wave-uniform
      const int I = uniform(base_I + g);
      const int q0 = I * S;
      const int k = uniform(I < l ? min(S, m - q0) : 0);
      const int kf = uniform(factorial_small(k));
      const bool active = k > 0 && r < kf;
      const int lq = q0 - cq;  // the subset's first position in the chunk
      uint32_t key = 0xFFFFFFFFu;
      uint32_t used = 0, locs = 0, pmv = 0;
      int32_t cost = 0;
      if (active) {
        // bins not used yet and bins not divided yet, one bit per slot
        uint32_t nused = 0xFFFFFFFFu;
        for (int gi = 0; gi < (nbslots >> 2); ++gi) {
          const int4 tv = *reinterpret_cast<const int4*>(tmplA + 4 * gi);
          int32_t* const p = myA + 256 * gi;
          p[0] = tv.x;
          p[64] = tv.y;
          p[128] = tv.z;
          p[192] = tv.w;
        }
        const uint32_t pm = k == S ? pm_full : nth_perm(r, k);
        pmv = pm;
        // A forced criterion c runs the same digit iteration from a word
        // whose every digit is c: 0, 2^31 (3 * 2^31 = 2^32 + 2^31) and
        // 2^32 - 1 (its deficit from 2^32 triples per step and stays below
        // 3^6 over at most six placements).
        uint32_t cu = a.force_crit >= 0
                          ? (a.force_crit == 0 ? 0u : (a.force_crit == 1 ? 0x80000000u : 0xFFFFFFFFu))
                          : (uint32_t)(splitmix64_mix(ck + (uint64_t)I * (uint64_t)P * kGolden +
                                                      st_lane) >> 32);
        int nb = n;
        // slot groups that hold a bin of some packer of the wave
        // (wave-uniform; every packer starts with the n Rule-2 bins, and a
        // placement adds at most two, so one ballot per placement keeps
        // 4 ng at or above every packer's count)
        int ng = (n + 3) >> 2;
        int sh = 0;
        // Puts the item (W10 = w << 10; tw: the type of the bin it opens
        // when nothing fits, in the low five bits) into the bin whose key's
        // low bits are bt when found, else into a new bin at the next free
        // slot.  Both cases run the same straight-line code: permutations of
        // a wave take different branches, and selects cost less than both
        // branch bodies.
        auto place = [&](bool found, uint32_t bt, uint32_t W10, uint32_t tw) {
          const int b = found ? (int)((bt >> 5) & 31u) : nb;
          const int type = (int)((found ? bt : tw) & 31u);
          int32_t* const pb = slot_at(myA, b);
          const int32_t word = *pb;  // a free slot holds an empty bin word
          const int4 ty = s_type[type];
          // the bin's word after the item: the chosen bin's, or an empty bin
          // of the item's type in slot b, with the room lowered by w (it
          // fits, so the low fields are untouched)
          const int32_t nw = (found ? word : (ty.y | (b << 5))) - (int32_t)W10;
          *pb = nw;
          nb += found ? 0 : 1;
          // a bin's first item adds its capacity to the cost (bit b of nused
          // sign-extended: all ones or zero)
          cost += ty.x & __builtin_amdgcn_sbfe((int32_t)nused, b, 1);
          nused &= ~(1u << b);
          // Rule 5: a bin at least half full (2 room <= cap, i.e. room <=
          // floor(cap / 2)) divides once, adding an empty bin of its type at
          // the next free slot.  Rooms only fall, so a bin divides at the
          // one placement that takes its room from above floor(cap / 2) to
          // at most that: the word before it (nw + W10, whose room field is
          // the room before) is at least H = (floor(cap / 2) + 1) << 10 and
          // the word after it is below H.  Every bin starts with room cap >
          // floor(cap / 2).  Without a division the slot after the last bin
          // is rewritten with the empty word it already holds (room 0, type
          // 0), which no scan picks.
          const uint32_t H = (uint32_t)ty.z;
          const bool split = (uint32_t)nw < H && (uint32_t)nw + W10 >= H;
          const int nbn = nb;
          nb += split ? 1 : 0;
          *slot_at(myA, nbn) = (split ? ty.y : 0) | (nbn << 5);
          // the bin of placement t, 5 bits at 5t
          locs |= (uint32_t)b << sh;
          sh += 5;
          if (ballot(nb > 4 * ng)) ++ng;
        };
        {
          // the first placement from the chunk's table: criterion digit c
          // picks bits 10c.. of the item's entry (the template's bins only;
          // one of them always holds the item)
          const int d = pm & 0xF;
          const int2 wt = s_cwt[lq + d];
          const uint32_t f = s_first[lq + d];
          const uint32_t c = __umulhi(cu, 3u);
          cu *= 3u;
          place(true, f >> (10u * c), (uint32_t)wt.x, (uint32_t)wt.y);
        }
        for (int t = 1; t < k; ++t) {
          const int d = (pm >> (4 * t)) & 0xF;
          const int2 wt = s_cwt[lq + d];
          const uint32_t W10 = (uint32_t)wt.x;  // w << 10
          // the criterion digit floor(3u / 2^32) times 16, the byte offset of
          // its key constants: floor(48u / 2^32) with the low four bits cleared
          const uint32_t koff = __umulhi(cu, 48u) & 0x30u;
          cu *= 3u;
          // x = XW or -W10, as (W10 ^ nm) + ad
          const uint4 kc = *reinterpret_cast<const uint4*>(
              reinterpret_cast<const unsigned char*>(s_keyc) + koff);
          const uint32_t sx = kc.x;
          const uint32_t x = (W10 ^ kc.y) + kc.z;
          const uint32_t msk = kc.w;
          // two groups per LDS round trip, then an odd last group alone
          uint32_t best = 0xFFFFFFFFu;
          int gi = 0;
          for (; gi + 1 < ng; gi += 2) {
            const uint32_t* const pg = reinterpret_cast<const uint32_t*>(myA + 256 * gi);
            const uint4 v = make_uint4(pg[0], pg[64], pg[128], pg[192]);
            const uint4 u = make_uint4(pg[256], pg[320], pg[384], pg[448]);
            const uint32_t k0 = ((v.x ^ sx) + x) & msk, k1 = ((v.y ^ sx) + x) & msk;
            const uint32_t k2 = ((v.z ^ sx) + x) & msk, k3 = ((v.w ^ sx) + x) & msk;
            const uint32_t k4 = ((u.x ^ sx) + x) & msk, k5 = ((u.y ^ sx) + x) & msk;
            const uint32_t k6 = ((u.z ^ sx) + x) & msk, k7 = ((u.w ^ sx) + x) & msk;
            // one three-way minimum per two keys
            best = min(min(best, k0), k1);
            best = min(min(best, k2), k3);
            best = min(min(best, k4), k5);
            best = min(min(best, k6), k7);
          }
          if (gi < ng) {
            const uint32_t* const pg = reinterpret_cast<const uint32_t*>(myA + 256 * gi);
            const uint4 v = make_uint4(pg[0], pg[64], pg[128], pg[192]);
            const uint32_t k0 = ((v.x ^ sx) + x) & msk, k1 = ((v.y ^ sx) + x) & msk;
            const uint32_t k2 = ((v.z ^ sx) + x) & msk, k3 = ((v.w ^ sx) + x) & msk;
            best = min(min(best, k0), k1);
            best = min(min(best, k2), k3);
          }
          // the chosen bin, or a new bin of the item's type (resolved with
          // its chunk) at the next free slot
          place(best < (1u << 25), best, W10, (uint32_t)wt.y);
        }
        used = ~nused;
        key = ((uint32_t)cost << 10) | (uint32_t)r;
      }
      // group minimum of (cost, rank): lowest rank on ties
      uint32_t gm = wave_min(key);
      if (lane == 0) s_wmin[wave] = gm;
      __syncthreads();
      gm = 0xFFFFFFFFu;
      for (int i = 0; i < wpg; ++i) gm = min(gm, s_wmin[g * wpg + i]);
      if (active && key == gm) {
        s_u[g] = (int32_t)__popc(used);
        s_cst[g] = cost;
      }
      if (r == 0 && k == 0) {
        s_u[g] = 0;
        s_cst[g] = 0;
      }
      __syncthreads();
      // canonical ids: this subset's bins follow those of earlier subsets.
      // Lane i < spr (<= 16) holds subset i's bin count and cost; prefix
      // sums over the first row give every wave the counts before its
      // subset and the round's total, and the first wave (which writes the
      // instance's cost) the round's cost (a round's cost fits int32: at
      // most 16 subsets of a few bins of capacity <= 32767).
      const int32_t pu = row_incl_sum(lane < spr ? s_u[lane] : 0);
      const int gw = uniform(g);  // a group is a whole number of wavefronts
      const int32_t before = carry + (gw > 0 ? readlane(pu, gw - 1) : 0);
      carry += readlane(pu, spr - 1);
      if (wave == 0) cost_acc += readlane(row_incl_sum(lane < spr ? s_cst[lane] : 0), spr - 1);
      // the winner's wave writes its result: lane t the item of placement
      // t, lane b the type of bin slot b if used
      const int wr = (int)(gm & 1023u);  // the winning rank
      if (k > 0 && wave == g * wpg + (wr >> 6)) {
        const uint32_t wused = readlane(used, wr & 63);
        const uint32_t wlocs = readlane(locs, wr & 63);
        const uint32_t wpm = readlane(pmv, wr & 63);
        if (lane < k) {
          const int b = (int)((wlocs >> (5 * lane)) & 31u);
          const int d = (int)((wpm >> (4 * lane)) & 0xFu);
          a.assign[off + (s_cwt[lq + d].y >> 5)] =
              before + (int)__popc(wused & ((1u << b) - 1u));
        }
        if (lane < 32 && ((wused >> lane) & 1u)) {
          a.types[off + before + (int)__popc(wused & ((1u << lane) - 1u))] =
              *slot_at(arrA + ((g * wpg + (wr >> 6)) * nbslots) * 64 + (wr & 63), lane) & 31;
        }
      }
    }
    if (tid == 0) {
      a.nbins[inst] = carry;
      a.cost[inst] = cost_acc;
    }
    __syncthreads();
  }
}

template <typename Kern>
hipError_t raise_lds(Kern kern, size_t lds, bool& done) {
  if (lds > 65536 && !done) {
    const hipError_t e = allow_max_dynamic_lds(kern);
    if (e != hipSuccess) return e;
    done = true;
  }
  return hipSuccess;
}

// minimum (cost, index) over num costs, lowest index on ties
__global__ void __launch_bounds__(1024) k_best_of(const int64_t* cost, int32_t num, int64_t* out) {
  __shared__ int64_t sc[1024];
  __shared__ int64_t si[1024];
  int64_t bc = 0x7FFFFFFFFFFFFFFFll, bi = 0x7FFFFFFFFFFFFFFFll;
  for (int i = threadIdx.x; i < num; i += blockDim.x) {
    const int64_t c = cost[i];
    if (c < bc) {
      bc = c;
      bi = i;
    }
  }
  sc[threadIdx.x] = bc;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      const int64_t c2 = sc[threadIdx.x + st], i2 = si[threadIdx.x + st];
      if (c2 < sc[threadIdx.x] || (c2 == sc[threadIdx.x] && i2 < si[threadIdx.x])) {
        sc[threadIdx.x] = c2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = num > 0 ? sc[0] : -1;
    out[1] = num > 0 ? si[0] : -1;
  }
}

}  // namespace


size_t h1_lds_bytes(int nbslots, int s1, int block, bool wide, bool learned) {
  return (learned ? kH1ModelBytes : 0) +
         (size_t)block * ((wide ? 2 : 1) * 4 * (size_t)nbslots + 4 * (size_t)s1 + (size_t)s1);
}

int h2_group(int s2) {
  int fact = 1;
  for (int i = 2; i <= s2; ++i) fact *= i;
  return ((fact + 63) / 64) * 64;
}

size_t h2_lds_bytes(int nbslots, int block, int group, H2Kernel k) {
  const int spr = block / group;
  if (k == H2Kernel::kSlim)  // bin array A, its template, chunk, per-subset results
    return 4 * ((size_t)nbslots * block + (size_t)nbslots + 3 * (size_t)block + 2 * (size_t)spr);
  return (size_t)block * (k == H2Kernel::kWide ? 2 : 1) * 4 * (size_t)nbslots +
         (size_t)spr * (4 * kMaxSubset * 4 + 2 * 4) + (size_t)spr * 8;
}


hipError_t launch_h1_grid(const BatchArgs& a, bool wide, int nbslots, int block, int grid,
                          hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  const bool lc = h1_learned(a);
  const size_t lds = h1_lds_bytes(nbslots, a.s1, block, wide, lc);
  const int blocks = grid > 0 ? grid : a.num;
  hipError_t e;
  if (!wide && !lc) {
    { static bool done1 = false; e = raise_lds(k_h1<uint32_t, false>, lds, done1); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h1<uint32_t, false>), dim3(blocks), dim3(block), lds, s, a, nbslots);
  } else if (!lc) {
    { static bool done2 = false; e = raise_lds(k_h1<uint64_t, false>, lds, done2); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h1<uint64_t, false>), dim3(blocks), dim3(block), lds, s, a, nbslots);
  } else if (!wide) {
    { static bool done3 = false; e = raise_lds(k_h1<uint32_t, true>, lds, done3); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h1<uint32_t, true>), dim3(blocks), dim3(block), lds, s, a, nbslots);
  } else {
    { static bool done4 = false; e = raise_lds(k_h1<uint64_t, true>, lds, done4); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h1<uint64_t, true>), dim3(blocks), dim3(block), lds, s, a, nbslots);
  }
  return hipGetLastError();
}


hipError_t launch_h2_grid(const BatchArgs& a, H2Kernel k, int nbslots, int block, int grid,
                          hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  const int group = h2_group(a.s2);
  if (block < group) block = group;
  block = (block / group) * group;
  const size_t lds = h2_lds_bytes(nbslots, block, group, k);
  const int blocks = grid > 0 ? grid : a.num;
  hipError_t e;
  if (k == H2Kernel::kSlim) {
    { static bool done3 = false; e = raise_lds(k_h2s, lds, done3); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_h2s, dim3(blocks), dim3(block), lds, s, a, nbslots, group);
  } else {
    { static bool done5 = false; e = raise_lds(k_h2<uint64_t>, lds, done5); }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_h2<uint64_t>, dim3(blocks), dim3(block), lds, s, a, nbslots, group);
  }
  return hipGetLastError();
}

namespace {
template <typename Kern>
int occ(Kern kern, int block, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}
}  // namespace

int h1_blocks_per_cu(bool wide, int block, size_t lds, bool learned) {
  if (learned)
    return wide ? occ(k_h1<uint64_t, true>, block, lds) : occ(k_h1<uint32_t, true>, block, lds);
  return wide ? occ(k_h1<uint64_t, false>, block, lds) : occ(k_h1<uint32_t, false>, block, lds);
}

int h2_blocks_per_cu(H2Kernel k, int block, size_t lds) {
  return k == H2Kernel::kSlim ? occ(k_h2s, block, lds) : occ(k_h2<uint64_t>, block, lds);
}

namespace {
__global__ void k_queue_reset(int32_t* q) {
  if (threadIdx.x == 0) *q = 0;
}

// Instances by decreasing item count, ties by index (bitonic sort of 64-bit
// keys in LDS, one workgroup; num <= kLptMax).
__global__ void __launch_bounds__(1024) k_lpt(const int64_t* item_off, int32_t num, int32_t* sched) {
  __shared__ uint64_t keys[kLptMax];
  int P = 1;
  while (P < num) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    uint64_t k = ~0ull;
    if (i < num) {
      int64_t m = item_off[i + 1] - item_off[i];
      if (m < 0) m = 0;
      if (m > 0x7FFFFFFF) m = 0x7FFFFFFF;
      k = ((uint64_t)(0xFFFFFFFFu - (uint32_t)m) << 32) | (uint32_t)i;
    }
    keys[i] = k;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = keys[i], y = keys[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            keys[i] = y;
            keys[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < num; i += blockDim.x) sched[i] = (int32_t)(keys[i] & 0xFFFFFFFFu);
}
}  // namespace

hipError_t launch_queue_reset(int32_t* queue, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
  return hipGetLastError();
}

hipError_t launch_lpt_schedule(const int64_t* item_off, int32_t num, int32_t* sched,
                               hipStream_t s) {
  if (num <= 0 || num > kLptMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lpt, dim3(1), dim3(1024), 0, s, item_off, num, sched);
  return hipGetLastError();
}

hipError_t launch_best_of(const int64_t* cost, int32_t num, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_best_of, dim3(1), dim3(1024), 0, s, cost, num, out);
  return hipGetLastError();
}

}  // namespace vsbpp
