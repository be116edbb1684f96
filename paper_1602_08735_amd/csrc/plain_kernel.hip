// Plain First/Best/Worst Fit (paper Section 1) over whole item lists, one
// 64-lane wavefront per instance.
//
// Per item (the hot step): every live bin tests in parallel whether the item
// fits (Rule 4 applicability) and a wave reduction picks the bin:
//   FF: min of (position << SH | room) over the fitting bins (the key with
//       its halves swapped);
//   BF: min of (room_after << SH | position);
//   WF: min of ((R - room_after) << SH | position);
// lowest position wins ties by construction, and positions keep bin-creation
// order, so that is the lowest bin index.  When nothing fits, a bin of type
// max{k : B_k >= w} (or B_1) is appended.
//
// An item heavier than an upper bound on every bin's room fits nowhere and
// skips the scan.  Plain runs (no scorer, hooks or bound on the open bins)
// open the bins of a run of such items together: each lane of a 64-item
// chunk knows the bin its item would open, and a prefix maximum over the
// lanes of those bins' rooms finds where the run ends.
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
#include "plain_common.h"

namespace vsbpp {
namespace {

// ---------------------------------------------------------------------------
// Learned scorer (bin type or bin choice), evaluated by one wavefront: lane l
// computes hidden unit l of both hidden layers and lane k output k (each unit
// is its bias, then an fp32 fused-multiply-add chain over its inputs in index
// order; the hidden units then take ReLU).
//
// The model is staged once per workgroup at the start of LDS as fp32, laid
// out so that lane l reads its rows of W2 and W3 as unit-stride 16-byte words
// at immediate offsets; its row of W1 and its biases stay in registers.  A
// layer's inputs pass once through LDS so that every 16-lane row holds them
// all, and reach the lanes of a row through DPP row broadcasts inside the
// fma instructions.
// Keeping W2 and W3 out of registers holds a scorer wavefront under 128 VGPRs,
// so four of them fit a SIMD and a batch of one instance per wavefront runs
// in a single wave of residency.
// ---------------------------------------------------------------------------
struct ModelLds {
  float w1[4 * 64 * 4];    // [i/4][l][4]
  float w2[16 * 64 * 4];   // [j/4][l][4]
  float w3[16 * 16 * 4];   // [j/4][k][4]
  float b1[64], b2[64], b3[16];
  int32_t n_out;
};

constexpr size_t kModelLdsBytes = (sizeof(ModelLds) + 15) & ~(size_t)15;

__device__ __forceinline__ float bf16f(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

__device__ void stage_model(const vsbpp_model* m, ModelLds* s) {
  for (int e = threadIdx.x; e < 64 * 16; e += blockDim.x) {
    const int l = e >> 4, i = e & 15;
    s->w1[(((i >> 2) * 64) + l) * 4 + (i & 3)] = bf16f(m->w1[e]);
  }
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int l = e >> 6, j = e & 63;
    s->w2[(((j >> 2) * 64) + l) * 4 + (j & 3)] = bf16f(m->w2[e]);
  }
  for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
    const int k = e >> 6, j = e & 63;
    s->w3[(((j >> 2) * 16) + k) * 4 + (j & 3)] = bf16f(m->w3[e]);
  }
  for (int e = threadIdx.x; e < 64; e += blockDim.x) {
    s->b1[e] = m->b1[e];
    s->b2[e] = m->b2[e];
    if (e < 16) s->b3[e] = m->b3[e];
  }
  if (threadIdx.x == 0) {
    const int n = m->n_out;
    s->n_out = n < 1 ? 1 : (n > 16 ? 16 : n);
  }
}

// The lane's own row of W1 and its biases, held in registers for the whole
// kernel (lane l: hidden unit l of both layers, output l for l < 16).
struct MlpRegs {
  float w1[16];
  float b1, b2, b3;
  int n_out;  // wave-uniform
};

__device__ void load_mlp_regs(const ModelLds* md, int lane, MlpRegs& r) {
#pragma unroll
  for (int ib = 0; ib < 4; ++ib) {
    const float4 wv = *reinterpret_cast<const float4*>(&md->w1[(ib * 64 + lane) * 4]);
    r.w1[ib * 4] = wv.x;
    r.w1[ib * 4 + 1] = wv.y;
    r.w1[ib * 4 + 2] = wv.z;
    r.w1[ib * 4 + 3] = wv.w;
  }
  r.b1 = md->b1[lane];
  r.b2 = md->b2[lane];
  r.b3 = md->b3[lane & 15];
  r.n_out = uniform(md->n_out);
}

// Sixteen steps of an index-order fma chain whose multiplicands come from a
// row: step i is acc = fma(x of lane i of the lane's own 16-lane row, w[i],
// acc).  The row value reaches every lane through the DPP row broadcast
// (row_newbcast) of v_fmac_f32, so the activations need no LDS broadcast
// reads; fma is exact before its one rounding, so the operand order inside it
// changes nothing.  The compiler neither forms this instruction from its DPP
// builtins nor sees wait states inside an asm statement, so the blocks carry
// their own: a layer's first block starts with five (a DPP read after a VALU
// write of EXEC needs five), the others with two (after a VALU write of the
// DPP source, should the compiler move x between blocks), and a layer's last
// block ends with two for whatever reads acc next.
#define VSBPP_FMA_ROW16_BODY(PRE, POST)                                                     \
  asm volatile(PRE                                                                          \
               "v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"    \
               "v_fmac_f32_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"   \
               "v_fmac_f32_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"   \
               "v_fmac_f32_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"  \
               "v_fmac_f32_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"  \
               "v_fmac_f32_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"  \
               "v_fmac_f32_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"  \
               "v_fmac_f32_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"  \
               "v_fmac_f32_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf" POST \
               : "+v"(acc)                                                                  \
               : "v"(x), "v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3]), "v"(w[4]), "v"(w[5]),  \
                 "v"(w[6]), "v"(w[7]), "v"(w[8]), "v"(w[9]), "v"(w[10]), "v"(w[11]),         \
                 "v"(w[12]), "v"(w[13]), "v"(w[14]), "v"(w[15]))

template <bool FIRST, bool LAST>
__device__ __forceinline__ float fma_row16(float acc, float x, const float (&w)[16]) {
  if constexpr (FIRST && LAST)
    VSBPP_FMA_ROW16_BODY("s_nop 4\n\t", "\n\ts_nop 1");
  else if constexpr (FIRST)
    VSBPP_FMA_ROW16_BODY("s_nop 4\n\t", "");
  else if constexpr (LAST)
    VSBPP_FMA_ROW16_BODY("s_nop 1\n\t", "\n\ts_nop 1");
  else
    VSBPP_FMA_ROW16_BODY("s_nop 1\n\t", "");
  return acc;
}
#undef VSBPP_FMA_ROW16_BODY

// A layer's 64 activations (one per lane) rearranged so that every 16-lane
// row holds them all: component q of lane l's result is the activation of
// lane 16q + (l & 15).  The wavefront writes them transposed into hbuf[0..63]
// and each lane reads four consecutive words back.
__device__ __forceinline__ float4 rows_of(float* hbuf, float h, int lane) {
  hbuf[((lane & 15) << 2) + (lane >> 4)] = h;
  return *reinterpret_cast<const float4*>(&hbuf[(lane & 15) << 2]);
}

// four 16-byte words at p, p + stride, p + 2 stride, p + 3 stride (floats)
__device__ __forceinline__ void load16(const float* p, int stride, float (&w)[16]) {
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) {
    const float4 v = *reinterpret_cast<const float4*>(p + jb * stride);
    w[4 * jb] = v.x;
    w[4 * jb + 1] = v.y;
    w[4 * jb + 2] = v.z;
    w[4 * jb + 3] = v.w;
  }
}

// Scores of outputs 0..n_out-1 end up in lanes 0..n_out-1 (others: junk).
// hbuf: 128 floats of LDS scratch of this wavefront; the 16 features sit at
// hbuf[64..79].
__device__ float mlp_forward_wave(const ModelLds* md, const MlpRegs& r, float* hbuf, int lane) {
  // features 0..15 in every row
  const float xf = hbuf[64 + (lane & 15)];
  // the weights of each block of sixteen inputs are read one block ahead:
  // W2's first block during layer 1, W3's first during W2's last
  float w[2][16];
  load16(&md->w2[lane * 4], 64 * 4, w[0]);
  float acc = fma_row16<true, true>(r.b1, xf, r.w1);
  const float4 h1 = rows_of(hbuf, acc > 0.0f ? acc : 0.0f, lane);
  // this lane's row of W2, four 16-byte words per block
  const int k = lane & 15;
  acc = r.b2;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < 3)
      load16(&md->w2[((4 * q + 4) * 64 + lane) * 4], 64 * 4, w[(q + 1) & 1]);
    else
      load16(&md->w3[k * 4], 16 * 4, w[(q + 1) & 1]);
    const float xq = q == 0 ? h1.x : (q == 1 ? h1.y : (q == 2 ? h1.z : h1.w));
    if (q == 0)
      acc = fma_row16<true, false>(acc, xq, w[0]);
    else if (q == 3)
      acc = fma_row16<false, true>(acc, xq, w[1]);
    else
      acc = fma_row16<false, false>(acc, xq, w[q & 1]);
  }
  const float4 h2 = rows_of(hbuf, acc > 0.0f ? acc : 0.0f, lane);
  // output k = lane & 15 on every row (rows 1..3 repeat row 0's work: the
  // broadcasts need the whole row active)
  float o = r.b3;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < 3) load16(&md->w3[((4 * q + 4) * 16 + k) * 4], 16 * 4, w[(q + 1) & 1]);
    const float xq = q == 0 ? h2.x : (q == 1 ? h2.y : (q == 2 ? h2.z : h2.w));
    if (q == 0)
      o = fma_row16<true, false>(o, xq, w[0]);
    else if (q == 3)
      o = fma_row16<false, true>(o, xq, w[1]);
    else
      o = fma_row16<false, false>(o, xq, w[q & 1]);
  }
  return o;
}

// Largest of the floats in lanes 0..15 (none NaN), as seen by lane 0: the
// reduction runs on an order-preserving integer image of the values.
__device__ __forceinline__ float row0_max(float f) {
  const uint32_t b = __float_as_uint(f);
  uint32_t v = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  v = max(v, dpp<kQuadSwap1>(0u, v));
  v = max(v, dpp<kQuadSwap2>(0u, v));
  v = max(v, dpp<kRowHalfMirror>(0u, v));
  v = max(v, dpp<kRowMirror>(0u, v));
  v = readlane(v, 0);
  return __uint_as_float((v & 0x80000000u) ? (v & 0x7FFFFFFFu) : ~v);
}

// inclusive suffix minimum over lanes [lane, 63]
__device__ __forceinline__ int32_t wave_suffix_min(int32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t o = __shfl_down(v, d, kWave);
    if (lane + d < kWave) v = min(v, o);
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// SPILL: the wavefront's arrays (keys, position->id map, suffix minima) sit
// in a device region of per_wave bytes per instance instead of LDS, for
// instances whose bins do not fit a workgroup's LDS (plain runs only).
// OPT bit 0: the bounded-active-bins code is compiled in (and taken when
// a.active_limit > 0); unbounded plain runs use the instantiation without it.
// OPT bit 1 (extended runs): the per-bin loads of the downsized cost of
// entries that name a source instance are kept; other runs go without them.
// OPT bit 2 (extended runs): the learned bin-type rule alone, with no
// decision hooks, bin choice or bound on the open bins, whose option checks
// then fold away.
template <int CRIT, typename K, bool EXT, bool SPILL, int OPT>
__global__ void __launch_bounds__(512) k_plain(BatchArgs a, int wpb, int64_t per_wave) {
  constexpr bool BND = (OPT & 1) != 0;
  constexpr bool DSL = EXT && (OPT & 2) != 0;
  constexpr bool LEAN = EXT && (OPT & 4) != 0;
  static_assert(!(LEAN && (BND || DSL)), "the lean learned run has no bound and no loads");
  static_assert(!(EXT && SPILL), "decision hooks and the scorer run from LDS");
  using KT = KeyT<K>;
  using Pid = typename KT::Pid;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id();
  const int wave = uniform((int)(threadIdx.x >> 6));
  // the scorer's weights sit at the start of LDS: every weight read is then
  // one aligned 16-byte word at an immediate offset from the lane's base
  ModelLds* md = reinterpret_cast<ModelLds*>(smem);
  const size_t model_bytes = (EXT && plain_scored(a)) ? kModelLdsBytes : 0;
  const size_t pid_bytes = ((size_t)a.slots * sizeof(Pid) + 15) & ~(size_t)15;
  const size_t smin_bytes = (((size_t)a.max_items + 63) / 64 * 4 + 15) & ~(size_t)15;
  K* keys;
  Pid* pid;
  int32_t* smin;
  int32_t* hist;
  float* hbuf;
  int32_t* bload;  // downsized cost of source-instance entries: load of every bin id
  auto carve = [&](unsigned char* base) {
    keys = reinterpret_cast<K*>(base);
    pid = reinterpret_cast<Pid*>(base + (size_t)a.slots * sizeof(K));
    smin = reinterpret_cast<int32_t*>(base + (size_t)a.slots * sizeof(K) + pid_bytes);
    hist = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(smin) + smin_bytes);
    hbuf = reinterpret_cast<float*>(hist + 16);
    bload = reinterpret_cast<int32_t*>(hbuf + 128);
  };
  const bool dsl = DSL && plain_ds_loads(a);
  if constexpr (!SPILL) carve(smem + model_bytes + (size_t)wave * (size_t)per_wave);
  MlpRegs mregs;
  if constexpr (EXT) {
    if (plain_scored(a)) {
      stage_model(a.model, md);
      __syncthreads();
      load_mlp_regs(md, lane, mregs);
    }
  }

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
    if constexpr (SPILL) carve(a.spill + (size_t)inst * (size_t)per_wave);
    K* const mine = keys + 4 * lane;
    // inputs come from instance `src_i` (entries may share an instance)
    const int src_i = (EXT && !LEAN && a.src) ? uniform(a.src[inst]) : inst;
    const int64_t off = a.item_off[src_i];
    const int64_t m64 = a.item_off[src_i + 1] - off;
    const int c0 = a.cap_off[src_i];
    const int n = a.cap_off[src_i + 1] - c0;
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
    // the bin choice scores two outputs (keep, open)
    if constexpr (EXT) {
      if (!err && !LEAN && a.choice_rule == 2 && md->n_out < 2) err = kErrModel;
    }
    const int m = (int)m64;
    const int nch = (m + 63) >> 6;
    int64_t total = 0;
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
        if constexpr (EXT) total += wave_sum64(q < m ? (int64_t)wq : 0);
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
    // decision state (extended runs only)
    int fd = -1, ft1 = -1, ft2 = -1, nev = 0;
    // weight placed so far: int32 with 32-bit keys (m <= 65535, B_1 <= 32767)
    typename std::conditional<sizeof(K) == 4, int32_t, int64_t>::type placed = 0;
    // lanes 0..4 and 8..12 hold the bucket thresholds 1..5, the others never pass
    int32_t thr_lane = 0x7FFFFFFF;
    float inv_cap_lane = 0.0f;
    // 1/B_1 and 1/m of the decision features, once per instance
    float inv_b1 = 0.0f, inv_m = 0.0f;
    // Decision features are computed one per lane (feature i in lane i):
    // each is a product F * G of fp32 values, F a converted integer (lane 2:
    // a quotient) and G a reciprocal (lanes 5..10: 1/max(bins, 1)).  The
    // parts that are constants of the instance: fa_base (F's integer: B_2..B_5
    // in lanes 11..14 for type decisions), fg_base (G: 1/B_1 or 1/m), and
    // the histogram slot each lane reads (lanes 5..10 buckets 0..5, the
    // others a slot that stays 0).
    int32_t fa_base = 0;
    float fg_base = 0.0f;
    int32_t hslot = 7;
    if constexpr (EXT) {
      if (!LEAN && a.force) {
        fd = uniform(a.force[3 * (int64_t)inst]);
        ft1 = uniform(a.force[3 * (int64_t)inst + 1]);
        ft2 = uniform(a.force[3 * (int64_t)inst + 2]);
      }
      // room r is in bucket floor(6r/(B_1+1)) = number of k in 1..5 with
      // r >= ceil(k(B_1+1)/6)
      if ((lane & 7) < 5 && lane < 16)
        thr_lane = (int32_t)(((int64_t)((lane & 7) + 1) * (B1 + 1) + 5) / 6);
      if (lane < 8) hist[lane] = 0;
      // features that are constants of the instance: B_2..B_5 over B_1, and
      // lane k's 1/B_k for the fill of the smallest fitting type
      inv_b1 = uniform_f(1.0f / (float)B1);
      inv_m = uniform_f(1.0f / (float)m);
      inv_cap_lane = lane < n ? 1.0f / (float)cap_lane : 0.0f;
      // lane l in 11..14 reads B_{l-10} from lane l - 10 (0 beyond n)
      const int32_t cap_up = __shfl(cap_lane, lane >= 11 && lane <= 14 ? lane - 10 : 0, kWave);
      if ((LEAN || a.choice_rule == 0) && lane >= 11 && lane <= 14) fa_base = cap_up;
      fg_base = (lane == 1 || lane == 4) ? inv_m : inv_b1;
      if (lane >= 5 && lane <= 10) hslot = lane - 5;
    }
    // rooms and capacities are int32.  The buckets of r0 (lanes 0..4) and r1
    // (lanes 8..12) in one ballot: bits 0..4 and 8..12 of it.
    auto buckets = [&](int32_t r0, int32_t r1) -> uint64_t {
      return ballot((lane < 8 ? r0 : r1) >= thr_lane);
    };

    int nlive = 0, nb = 0;
    // least room written since the last compaction (a closed bin counts as
    // room 0): some bin is dead at the next chunk iff it is below that
    // chunk's bound, or the bound has risen anyway
    uint32_t minroom = 0xFFFFFFFFu;
    int32_t tprev = 0;
    // with 32-bit keys m <= 65535 and B_1 <= 32767, so the cost fits int32
    using Cost = typename std::conditional<sizeof(K) == 4, int32_t, int64_t>::type;
    Cost cost = 0;
    // Upper bound on the room of every bin in the scan array: an item heavier
    // than it fits nowhere, so its scan is skipped.  Rooms only shrink, a new
    // bin raises the bound, and a scan that finds no fit sets it to the
    // largest room exactly.
    int32_t ub = 0;  // rooms are int32 with either key width
    // Plain runs open the bins of a run of such items together (below):
    // their costs and least room per lane, folded in at the end.
    // (not compiled into the instantiations with the bounded-bins code)
    constexpr bool runs = !EXT && !BND;
    Cost costv = 0;
    for (int c = 0; c < nch; ++c) {
      const int32_t T = uniform(smin[c]);
      if (nlive > 0 && (minroom < (uint32_t)T || T > tprev)) {
        nlive = uniform(compact<CRIT, K>(keys, pid, nlive, T, lane));
        minroom = 0xFFFFFFFFu;
      }
      tprev = T;
      const int q = (c << 6) + lane;
      int item = q;
      int32_t wv = 0;
      if (q < m) {
        if (a.order) item = a.order[off + q];
        wv = a.w[off + item];
      }
      int32_t sfx = 0x7FFFFFFF, next_min = 0x7FFFFFFF;
      if (EXT || (BND && a.active_limit > 0)) {
        sfx = wave_suffix_min(q < m ? wv : 0x7FFFFFFF, lane);
        if (c + 1 < nch) next_min = uniform(smin[c + 1]);
      }
      // positions are stable until the next compaction, so each item records
      // its bin's position and the ids are read once at the end of the chunk
      int32_t mypos = 0;
      const int cnt = min(kWave, m - (c << 6));
      // Runs of new bins (plain runs): the bin each item of the chunk opens
      // if nothing fits it, its type tv, capacity btv and room rv
      int32_t tv = 0, btv = 0, rv = 0;
      uint32_t minroomv = 0xFFFFFFFFu;
      if (runs) {
        if (LEAN || a.type_rule != 1)
          for (int k = 1; k < n; ++k) tv += readlane(cap_lane, k) >= wv ? 1 : 0;
        btv = __shfl(cap_lane, tv, kWave);
        rv = q < m ? btv - wv : 0;
      }
      for (int jj = 0; jj < cnt; ++jj) {
        const int32_t w = readlane(wv, jj);
        if (runs && w > ub) {
          // Items jj, jj+1, ... open bins without a scan for as long as each
          // is heavier than the bound, which every bin opened before it in
          // the run raises to at least that bin's room.  Lane l (l >= jj)
          // compares its weight with max(ub, rooms of lanes jj..l-1); the
          // run ends at the first lane that does not exceed it (item jj
          // does: its weight is above ub).  The run's bins take positions
          // nlive.. and ids nb.. in item order, as one at a time would.
          const int32_t rin = lane >= jj ? rv : 0;
          const int32_t rsh = wave_shr1(rin);
          const int32_t x = lane == jj ? ub : (lane > jj ? rsh : 0);
          const int32_t pm = wave_incl_max(x);
          const uint64_t smask = ballot(lane >= jj && lane < cnt && wv > pm);
          // run length: the set bits of smask from bit jj (bit jj is set:
          // pm = ub in lane jj).  All 64 set (jj = 0, a full chunk) leaves no
          // clear bit to find, so that case is taken apart; the run always
          // holds item jj, so the loop advances.
          const uint64_t rest = ~(smask >> jj);
          int L = rest == 0 ? kWave - jj : (int)__builtin_ctzll(rest);
          L = L < 1 ? 1 : L;
          const bool run = lane >= jj && lane < jj + L;
          const int pos = nlive + (lane - jj);
          // a 256-position group that starts inside the run starts empty
          const int g0 = (nlive + 255) >> 8;
          if ((g0 << 8) < nlive + L) fill_group(keys, g0, lane, empty_key<CRIT, K>());
          const K room = (K)rin;
          if (run) {
            const K key = CRIT == WF ? (((KT::R - room) << KT::SH) | (K)pos)
                                     : ((room << KT::SH) | (K)pos);
            keys[kidx(pos)] = key;
            pid[pos] = (Pid)(nb + (lane - jj));
          }
          mypos = run ? pos : mypos;
          costv += run ? (Cost)btv : (Cost)0;
          minroomv = run ? min(minroomv, (uint32_t)rin) : minroomv;
          if (run) a.types[off + nb + (lane - jj)] = tv;
          ub = max(ub, readlane(max(pm, rin), jj + L - 1));
          nlive = uniform(nlive + L);
          nb = uniform(nb + L);
          jj += L - 1;
          continue;
        }
        const K wk = (K)w << KT::SH;
        int p = -1;
        K nk = 0;
        if (w <= ub) {
          // some bin may hold the item: scan the live groups.  First Fit
          // takes the lowest position among the fitting bins (a key with its
          // halves swapped is pos << SH | room, so the least of those names
          // the first fit and its room); Best and Worst Fit the least
          // candidate key.  FF/BF also keep the largest key, whose room
          // bounds every room.
          const int ng = uniform((nlive + 255) >> 8);
          auto cand = [&](K key) -> K {
            if constexpr (CRIT == FF) {
              const K sw = (key >> KT::SH) | (key << KT::SH);
              return key >= wk ? sw : ~(K)0;
            } else {
              return CRIT == WF ? key + wk : key - wk;
            }
          };
          K best = ~(K)0;
          K kmax = 0;
          int g = 0;
          for (; g + 1 < ng; g += 2) {
            K k[4], k2[4];
            load_group(keys, g, lane, k);
            load_group(keys, g + 1, lane, k2);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              best = min(best, min(cand(k[j]), cand(k2[j])));
              if constexpr (CRIT != WF) kmax = max(kmax, max(k[j], k2[j]));
            }
          }
          if (g < ng) {
            K k[4];
            load_group(keys, g, lane, k);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              best = min(best, cand(k[j]));
              if constexpr (CRIT != WF) kmax = max(kmax, k[j]);
            }
          }
          best = wave_min(best);
          if (CRIT == FF ? best != ~(K)0 : best < KT::TOP) {
            if constexpr (CRIT == FF) {
              p = (int)(best >> KT::SH);
              nk = (((best & KT::POS) << KT::SH) | (K)p) - wk;
            } else {
              p = (int)(best & KT::POS);
              nk = best;
            }
          } else if constexpr (CRIT == WF) {
            // no key wrapped: best is the least key plus w, and the least
            // key holds the largest room (no groups: no bins, no room)
            ub = ng > 0 ? (int32_t)(KT::R - ((best - wk) >> KT::SH)) : 0;
          } else {
            ub = (int32_t)(~wave_min(~kmax) >> KT::SH);
          }
        }
        // Decision features, feature i in lane i (i < 16), and a copy at
        // hbuf[64..79] for the scorer.  Features 0..10: the item, the items
        // after it, the bins so far and their room histogram; `ext` puts
        // features 11..15 in lanes 11..15 of F's integer (bin choice), and
        // g15 is lane 15's G (type decisions: 1/B_t of the smallest type
        // holding the item).
        auto lane_features = [&](auto ext, float g15) -> float {
          const int qq = (c << 6) + jj;
          const int rem = m - qq - 1;
          const int64_t rsum = total - (int64_t)placed - w;
          int32_t after = jj + 1 < kWave ? readlane(sfx, jj + 1) : 0x7FFFFFFF;
          after = min(after, next_min);
          int32_t fa = hist[hslot] + fa_base;
          fa = writelane(fa, w, 0);
          fa = writelane(fa, rem, 1);
          fa = writelane(fa, after, 3);
          fa = writelane(fa, nb, 4);
          fa = ext(fa);
          // with 32-bit keys m <= 65535 and B_1 <= 32767, so the remaining
          // weight fits int32 (whose conversion rounds as int64's does)
          const float frs = sizeof(K) == 4 ? (float)(int32_t)rsum : (float)rsum;
          // one division for all: lane 2 the mean weight after the item
          // (rem = 0 leaves rsum = 0, a quotient 0), the others 1/max(bins, 1)
          const float num = __int_as_float(writelane(__float_as_int(1.0f), __float_as_int(frs), 2));
          const int32_t den = writelane(nb > 0 ? nb : 1, rem > 0 ? rem : 1, 2);
          const float qt = num / (float)den;
          const float f = lane == 2 ? qt : (float)fa;
          float g = (lane >= 5 && lane <= 10) ? qt : fg_base;
          g = __int_as_float(writelane(__float_as_int(g), __float_as_int(g15), 15));
          float xl = f * g;
          // no item after this one: feature 3 is 1
          if (rem == 0) xl = __int_as_float(writelane(__float_as_int(xl), __float_as_int(1.0f), 3));
          hbuf[64 + lane] = xl;
          return xl;
        };
        if constexpr (EXT) {
          // Bin choice (largest type rule, downsizing): every bin has capacity
          // B_1 and costs c(L), the smallest capacity >= its load L.  The
          // placement into the criterion's bin is contested when c(L + w) >
          // c(L); the capacities are distinct and decreasing, so that is when
          // fewer types hold L + w than hold L.
          if (!LEAN && a.choice_rule != 0 && p >= 0) {
            const int32_t ra = (int32_t)room_of<CRIT>(nk);  // room after the item
            const int32_t L = B1 - ra - w;
            const uint64_t hb = ballot(cap_lane >= L);
            const uint64_t ha = ballot(cap_lane >= L + w);
            if (hb != ha) {
              const int d = nev;
              nev = uniform(nev + 1);
              const bool dump = d == fd && (a.feat_out || a.info_out);
              bool open = false;
              if (a.choice_rule == 2 || dump) {
                const int32_t cb = readlane(cap_lane, (int)__popcll(hb) - 1);
                const int32_t ca = readlane(cap_lane, (int)__popcll(ha) - 1);
                const int32_t cw = readlane(cap_lane, (int)__popcll(ballot(cap_lane >= w)) - 1);
                const float xl = lane_features(
                    [&](int32_t fa) {
                      fa = writelane(fa, ra, 11);
                      fa = writelane(fa, ca - cb, 12);
                      fa = writelane(fa, cw, 13);
                      fa = writelane(fa, ca - L - w, 14);
                      return writelane(fa, cb - L, 15);
                    },
                    inv_b1);
                if (a.choice_rule == 2) {
                  const float z = mlp_forward_wave(md, mregs, hbuf, lane);
                  const float z0 = __uint_as_float(readlane(__float_as_uint(z), 0));
                  const float z1 = __uint_as_float(readlane(__float_as_uint(z), 1));
                  // a new bin only on a strictly larger score; non-finite
                  // scores keep the criterion's bin
                  open = __builtin_isfinite(z0) && __builtin_isfinite(z1) && z1 > z0;
                }
                if (dump) {
                  if (a.feat_out && lane < 16) a.feat_out[16 * (int64_t)inst + lane] = xl;
                  if (a.info_out && lane == 0) {
                    a.info_out[2 * (int64_t)inst] = 3;      // keep and open both allowed
                    a.info_out[2 * (int64_t)inst + 1] = 0;  // the plain choice keeps
                  }
                }
              }
              if (!LEAN && fd >= 0) {  // forced decisions (rollouts) only
                const int ft = d == fd ? ft1 : (d == fd + 1 ? ft2 : -1);
                if (ft == 0 || ft == 1) open = ft == 1;
              }
              if (open) p = -1;
            }
          }
        }
        if (p >= 0) {
          // Rule 4: place into the chosen open bin
          put_key(mine, lane, p, nk);
          if (dsl && lane == 0) bload[pid[p]] += w;
          const K rnew = room_of<CRIT>(nk);
          minroom = min(minroom, (uint32_t)rnew);
          if constexpr (EXT) {
            // the bin moves from the bucket of its old room to that of its
            // new one: lane 0 takes it out, lane 1 puts it in
            const uint64_t ge = buckets((int32_t)rnew + w, (int32_t)rnew);
            const int b0 = (int)__popcll(ge & 0x1Full), b1 = (int)__popcll(ge & 0x1F00ull);
            if (b0 != b1 && lane < 2) atomicAdd(&hist[lane == 0 ? b0 : b1], lane == 0 ? -1 : 1);
          }
        } else {
          // nothing fits: open a bin of the chosen type
          if (BND && a.active_limit > 0) {
            // Bounded runs: at most active_limit bins are open, and a bin
            // that must open while that many are open first closes the
            // fullest (least room, lowest index on ties).  A bin whose room
            // is below every weight still to come can never take an item and
            // is fuller than any other, so closing it at once changes no
            // placement: the open bins that count are the live ones, and the
            // key list is already in creation order.  The closed bin's key
            // takes room 0, which no scan picks and compaction removes.
            const int32_t tj = min(readlane(sfx, jj), next_min);
            const int ngl = uniform((nlive + 255) >> 8);
            K best = ~(K)0;
            int open = 0;
            for (int g = 0; g < ngl; ++g) {
              K k[4];
              load_group(keys, g, lane, k);
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int pos = (g << 8) + (j << 6) + lane;
                const K r = room_of<CRIT>(k[j]);
                const bool live = pos < nlive && r >= (K)tj;
                open += (int)__popcll(ballot(live));
                best = min(best, live ? ((r << KT::SH) | (K)pos) : ~(K)0);
              }
            }
            if (open >= a.active_limit) {
              const int pf = (int)(wave_min(best) & KT::POS);
              put_key(mine, lane, pf, CRIT == WF ? ((KT::R << KT::SH) | (K)pf) : (K)pf);
              minroom = 0;
            }
          }
          // types holding the item (lanes >= n hold capacity 0 and w >= 1)
          const uint64_t fm = ballot(cap_lane >= w);
          const int smallest = (int)__popcll(fm) - 1;
          int t = (!LEAN && a.type_rule == 1) ? 0 : smallest;
          // under the bin choice the decisions are contested placements, and
          // a bin opened because nothing fits has type 0 (largest type rule)
          if (EXT && (LEAN || a.choice_rule == 0)) {
            const int d = nev;
            if (!LEAN) nev = uniform(nev + 1);
            const bool dump = !LEAN && d == fd && (a.feat_out || a.info_out);
            // features only where the scorer has a choice (or a dump asks)
            if (((LEAN || a.type_rule == 2) && smallest > 0) || dump) {
              // lanes 11..14: B_2..B_5 over B_1, lane 15: w over B_t
              const float xl = lane_features(
                  [&](int32_t fa) { return writelane(fa, w, 15); },
                  __uint_as_float(readlane(__float_as_uint(inv_cap_lane), smallest)));
              // with one type holding the item the scorer has nothing to choose
              if ((LEAN || a.type_rule == 2) && smallest > 0) {
                const float z = mlp_forward_wave(md, mregs, hbuf, lane);
                const int kmax = min(n, mregs.n_out);
                // lanes 0..kmax-1 hold the scores; the choice is the lowest
                // feasible type (one holding the item) whose score equals the
                // largest feasible score
                const bool in = lane < kmax;
                const bool feas = in && cap_lane >= w;
                const float mx = row0_max(feas ? z : -__builtin_inff());
                const int bi = (int)__builtin_ctzll(ballot(feas && z == mx));
                // the scorer only proposes: non-finite scores fall back
                t = ballot(in && !__builtin_isfinite(z)) == 0ull ? bi : smallest;
              }
              if (dump) {
                if (a.feat_out && lane < 16) a.feat_out[16 * (int64_t)inst + lane] = xl;
                if (a.info_out && lane == 0) {
                  a.info_out[2 * (int64_t)inst] = (int32_t)fm;
                  a.info_out[2 * (int64_t)inst + 1] = smallest;
                }
              }
            }
            if (!LEAN && fd >= 0) {  // forced decisions (rollouts) only
              const int ft = d == fd ? ft1 : (d == fd + 1 ? ft2 : -1);
              if (ft >= 0 && ft < n && ((fm >> ft) & 1ull)) t = ft;
            }
          }
          const int32_t Bt = readlane(cap_lane, t);
          const K room = (K)(Bt - w);
          ub = max(ub, (int32_t)room);
          p = nlive;
          nlive = uniform(nlive + 1);
          const int id = nb;
          nb = uniform(nb + 1);
          if ((p & 255) == 0) fill_group(keys, p >> 8, lane, empty_key<CRIT, K>());
          const K key = CRIT == WF ? (((KT::R - room) << KT::SH) | (K)p)
                                   : ((room << KT::SH) | (K)p);
          // the lane that holds position p also writes its id (pid + lane is
          // that lane's base in the position -> id map)
          if (lane == (p & 63)) {
            mine[(p & ~255) + ((p >> 6) & 3)] = key;
            pid[(p & ~63) + lane] = (Pid)id;
          }
          if (dsl && lane == 0) bload[id] = w;
          const bool out_types = !EXT || LEAN || !a.src;
          if (out_types && lane == 0) a.types[off + id] = t;
          cost += Bt;
          minroom = min(minroom, (uint32_t)room);
          if constexpr (EXT) {
            const int bn = (int)__popcll(buckets((int32_t)room, (int32_t)room) & 0x1Full);
            if (lane == 0) hist[bn] += 1;
          }
        }
        if constexpr (EXT) placed += w;
        mypos = writelane(mypos, p, jj);
      }
      if (runs) minroom = min(minroom, wave_min(minroomv));
      if ((!EXT || LEAN || !a.src) && q < m) a.assign[off + item] = (int32_t)pid[mypos];
    }
    if (runs) cost += (Cost)wave_sum64((int64_t)costv);
    int64_t out_cost = cost;
    if (dsl) {
      // downsized cost: every bin at the smallest capacity holding its load
      int64_t ds = 0;
      for (int id = lane; id < nb; id += kWave) {
        const int32_t l = bload[id];
        int32_t c = B1;
        for (int k = 1; k < n; ++k) {
          const int32_t ck = readlane(cap_lane, k);
          c = ck >= l ? ck : c;
        }
        ds += c;
      }
      out_cost = wave_sum64(ds);
    }
    if (lane == 0) {
      a.nbins[inst] = nb;
      a.cost[inst] = out_cost;
      if (EXT && !LEAN && a.count_out) a.count_out[inst] = nev;
    }
  }
}

template <int CRIT, typename K, bool EXT, bool SPILL, int OPT>
hipError_t launch_one(const BatchArgs& a, int wpb, size_t per_wave, int grid, hipStream_t s) {
  const size_t lds = SPILL ? 0
                           : per_wave * (size_t)wpb +
                                 (EXT ? plain_lds_block_extra(plain_scored(a)) : 0);
  auto kern = k_plain<CRIT, K, EXT, SPILL, OPT>;
  static bool raised = false;
  if (lds > 65536 && !raised) {
    hipError_t e = allow_max_dynamic_lds(kern);
    if (e != hipSuccess) return e;
    raised = true;
  }
  const int blocks = grid > 0 ? grid : (a.num + wpb - 1) / wpb;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, s, a, wpb, (int64_t)per_wave);
  return hipGetLastError();
}

template <int CRIT, typename K>
hipError_t launch_sel(const BatchArgs& a, int wpb, size_t per_wave, int grid, hipStream_t s) {
  if (a.spill) return launch_one<CRIT, K, false, true, 1>(a, wpb, per_wave, grid, s);
  if (plain_ext(a)) {
    if (plain_lean_learned(a)) return launch_one<CRIT, K, true, false, 4>(a, wpb, per_wave, grid, s);
    return plain_ds_loads(a) ? launch_one<CRIT, K, true, false, 3>(a, wpb, per_wave, grid, s)
                             : launch_one<CRIT, K, true, false, 1>(a, wpb, per_wave, grid, s);
  }
  return a.active_limit > 0 ? launch_one<CRIT, K, false, false, 1>(a, wpb, per_wave, grid, s)
                            : launch_one<CRIT, K, false, false, 0>(a, wpb, per_wave, grid, s);
}

template <int CRIT, typename K>
int occupancy(int wpb, size_t per_wave, bool ext, bool learned, bool spill, bool bounded,
              bool dsl, bool lean) {
  int n = 0;
  hipError_t e;
  if (spill) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, false, true, 1>,
                                                     64 * wpb, 0);
  } else {
    const size_t lds = per_wave * (size_t)wpb + (ext ? plain_lds_block_extra(learned) : 0);
    if (ext && lean)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, true, false, 4>,
                                                       64 * wpb, lds);
    else if (ext && dsl)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, true, false, 3>,
                                                       64 * wpb, lds);
    else if (ext)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, true, false, 1>,
                                                       64 * wpb, lds);
    else if (bounded)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, false, false, 1>,
                                                       64 * wpb, lds);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<CRIT, K, false, false, 0>,
                                                       64 * wpb, lds);
  }
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace

size_t plain_lds_per_wave(int slots, int max_items, bool wide, bool ext, bool ds_loads) {
  const size_t ks = wide ? 8 : 4, ps = wide ? 4 : 2;
  const size_t nch = ((size_t)max_items + 63) / 64;
  size_t b = (size_t)slots * ks;
  b += ((size_t)slots * ps + 15) & ~(size_t)15;
  b += (nch * 4 + 15) & ~(size_t)15;
  if (ext) b += 16 * 4 + 128 * 4;  // room histogram + hidden-layer scratch
  if (ext && ds_loads) b += ((size_t)max_items * 4 + 15) & ~(size_t)15;  // bin loads
  return b;
}

size_t plain_lds_block_extra(bool learned) { return learned ? kModelLdsBytes : 0; }

hipError_t launch_plain_grid(const BatchArgs& a, int crit, bool wide, int wpb,
                             size_t lds_per_wave, int grid, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  if (!wide) {
    if (crit == FF) return launch_sel<FF, uint32_t>(a, wpb, lds_per_wave, grid, s);
    if (crit == BF) return launch_sel<BF, uint32_t>(a, wpb, lds_per_wave, grid, s);
    return launch_sel<WF, uint32_t>(a, wpb, lds_per_wave, grid, s);
  }
  if (crit == FF) return launch_sel<FF, uint64_t>(a, wpb, lds_per_wave, grid, s);
  if (crit == BF) return launch_sel<BF, uint64_t>(a, wpb, lds_per_wave, grid, s);
  return launch_sel<WF, uint64_t>(a, wpb, lds_per_wave, grid, s);
}


int plain_blocks_per_cu(const BatchArgs& a, int crit, bool wide, int wpb, size_t lds_per_wave) {
  const bool ext = plain_ext(a), learned = plain_scored(a), spill = a.spill != nullptr;
  const bool bnd = a.active_limit > 0, dsl = plain_ds_loads(a), lean = plain_lean_learned(a);
  const size_t lw = lds_per_wave;
  if (!wide) {
    if (crit == FF) return occupancy<FF, uint32_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
    if (crit == BF) return occupancy<BF, uint32_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
    return occupancy<WF, uint32_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
  }
  if (crit == FF) return occupancy<FF, uint64_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
  if (crit == BF) return occupancy<BF, uint64_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
  return occupancy<WF, uint64_t>(wpb, lw, ext, learned, spill, bnd, dsl, lean);
}

}  // namespace vsbpp
