// Exact optimum of small VSBPP instances (m <= 12 items), a batch at a time.
//
// Cost model of the problem statement (Section 1, formal definition): a bin
// of type k costs its capacity B_k, a packing costs the sum over its used bins.  A block of items
// (the contents of one bin) therefore costs the smallest capacity that holds
// its total weight, and the optimum is the cheapest partition of the items
// into blocks.  The kernel evaluates it by dynamic programming over item
// subsets:
//   f(0) = 0,   f(S) = min over blocks T of S that contain the lowest item of S
//                      of  c(T) + f(S \ T),
// with c(T) the cheapest capacity >= sum of T (infinite when the total
// exceeds B_1).  Requiring the lowest item of S in T visits every partition
// once, as a sequence of blocks ordered by their lowest item.
//
// gfx950 layout: one workgroup per instance (a static stride over the batch
// when the grid is smaller), every table in LDS at fixed offsets from 0:
//   G[P(S)] = f(S) << 12           the optimum of S
//   C[P(T)] = (c(T) << 12) | T      the block cost, the block in the low bits
//                                    (c(T) = INF when T fits no bin)
//   B[S]    = the first block of the optimal partition of S chosen
// so G[P(S\T)] + C[P(T)] is a candidate key whose minimum over T is the
// optimum with the smallest block mask among the optimal ones.  Subsets are
// processed by popcount: every subset of popcount k depends only on smaller
// ones, so one layer is one parallel step.  In layer k each subset has
// 2^(k-1) candidate blocks; a group of g lanes shares a subset (g = 2^(k-6)
// clamped to [1,64], so each lane takes 32 candidates when there are that
// many: the per-subset set-up is then small next to the candidates).  The
// lane fixes the lowest log2(g) free items of the block by its index and
// walks the subsets of the other free items in Gray-code order, one item
// toggled per step.
//
// P(X) = X ^ (X >> 6) is a bijection of 12-bit masks that folds the high
// items into the low address bits, so the lanes of a group, which differ in
// up to six items, spread over the LDS banks.  P is linear over GF(2):
// P(S\T) = P(S) ^ P(T), and a Gray step toggles P(T) by a per-subset
// constant, so each candidate costs two XORs, two LDS reads, an addition
// and a minimum.
//
// Keys are 32-bit when m * B_1 < 2^19 (f < 2^19, so a key stays below 2^31
// and INF = 2^31 cannot overflow), else 64-bit (f < 2^35, INF = 2^62).
#include "device_common.h"
#include "kernels.h"

namespace vsbpp {
namespace {

constexpr int kSubsets = 1 << kExactMaxItems;
constexpr int kBinomW = kExactMaxItems + 1;   // row width of the binomial table
constexpr uint32_t kBlockBits = 0xFFFu;       // block mask in the low 12 bits of a key
constexpr int32_t kErrDevice = -7;            // VSBPP_E_DEVICE

template <typename K>
struct ExactKey;
template <>
struct ExactKey<uint32_t> {
  static constexpr uint32_t kInf = 1u << 31;
};
template <>
struct ExactKey<uint64_t> {
  static constexpr uint64_t kInf = 1ull << 62;
};

__device__ __forceinline__ uint32_t shfl_xor_k(uint32_t v, int d) {
  return (uint32_t)__shfl_xor((int)v, d, kWave);
}
__device__ __forceinline__ uint64_t shfl_xor_k(uint64_t v, int d) {
  const uint32_t lo = shfl_xor_k((uint32_t)v, d), hi = shfl_xor_k((uint32_t)(v >> 32), d);
  return ((uint64_t)hi << 32) | lo;
}

// the fold permutation of 12-bit masks
__device__ __forceinline__ uint32_t fold(uint32_t x) { return x ^ (x >> 6); }

// LDS layout (bytes from 0; the kernel has no other LDS)
template <typename K>
struct ExactLds {
  // (every table starts on its element size; G on a multiple of its size)
  static constexpr uint32_t kG = 0;
  static constexpr uint32_t kC = kG + sizeof(K) * kSubsets;
  static constexpr uint32_t kB = kC + sizeof(K) * kSubsets;
  static constexpr uint32_t kList = kB + 2 * kSubsets;
  static constexpr uint32_t kBinom = kList + 2 * kSubsets;
  static constexpr uint32_t kLayer = kBinom + 4 * kBinomW * kBinomW;
  static constexpr uint32_t kCaps = kLayer + 4 * 16;
  static constexpr uint32_t kW = kCaps + 4 * kMaxTypes;
  static constexpr uint32_t kBlocks = kW + 4 * kExactMaxItems;
  static constexpr uint32_t kNb = kBlocks + 4 * kExactMaxItems;
  static constexpr uint32_t kFlag = kNb + 4;
  static constexpr uint32_t kHalf = (kFlag + 4 + 7) & ~7u;  // int64 sums, items 0-5 / 6-11
  static constexpr uint32_t kBytes = kHalf + 8 * 128;
};

template <typename K>
size_t exact_dyn_lds() {
  return ExactLds<K>::kBytes;
}

// a load from an LDS byte address
template <typename K>
__device__ __forceinline__ K lds_load(uint32_t addr) {
  return *reinterpret_cast<const __attribute__((address_space(3))) K*>(addr);
}

// IT candidates of one lane.  pt = LDS address of the G table plus
// P(T) * sizeof(K) for the first block (the table base is aligned to the
// table size, so XORs below that size leave it intact); ps = P(S) * sizeof(K);
// flip[j] = the P-image (bytes) of the j-th Gray item.
template <int IT, typename K>
__device__ __forceinline__ K run_candidates(uint32_t pt, uint32_t ps, const uint32_t (&flip)[5]) {
  using L = ExactLds<K>;
  K best = ~(K)0;
#pragma unroll
  for (int t = 0; t < IT; ++t) {
    const K v = lds_load<K>(pt ^ ps) + lds_load<K>(pt + (L::kC - L::kG));
    best = min(best, v);
    if (t + 1 < IT) pt ^= flip[__builtin_ctz(t + 1)];
  }
  return best;
}

// Three 512-thread workgroups per CU (LDS ~51 KB each) need six waves per
// SIMD, so at most 80 VGPRs.
template <typename K>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
k_exact(BatchArgs a) {
  using L = ExactLds<K>;
  extern __shared__ __align__(16) unsigned char smem[];
  K* sG = reinterpret_cast<K*>(smem + L::kG);
  K* sC = reinterpret_cast<K*>(smem + L::kC);
  uint16_t* sB = reinterpret_cast<uint16_t*>(smem + L::kB);
  uint16_t* sList = reinterpret_cast<uint16_t*>(smem + L::kList);
  int32_t* s_binom = reinterpret_cast<int32_t*>(smem + L::kBinom);
  int32_t* s_layer = reinterpret_cast<int32_t*>(smem + L::kLayer);
  int32_t* s_caps = reinterpret_cast<int32_t*>(smem + L::kCaps);
  int32_t* s_w = reinterpret_cast<int32_t*>(smem + L::kW);
  uint32_t* s_blocks = reinterpret_cast<uint32_t*>(smem + L::kBlocks);
  int32_t* s_nb = reinterpret_cast<int32_t*>(smem + L::kNb);
  int32_t* s_flag = reinterpret_cast<int32_t*>(smem + L::kFlag);
  int64_t* s_half = reinterpret_cast<int64_t*>(smem + L::kHalf);
  constexpr K kInf = ExactKey<K>::kInf;
  constexpr uint32_t kSz = sizeof(K);
  const int tid = threadIdx.x, nt = blockDim.x;
  // LDS byte address of the G table (the low 32 bits of the flat address)
  const uint32_t g_base = (uint32_t)(uintptr_t)(smem + L::kG);
  if (g_base & (kSz * kSubsets - 1)) {
    // the XOR addressing needs the table on a table-size boundary (it starts
    // at LDS address 0, as the kernel has no static LDS)
    for (int inst = blockIdx.x; inst < a.num; inst += gridDim.x)
      if (tid == 0) a.nbins[inst] = kErrDevice;
    return;
  }
  // true on every thread when p holds on any (three barriers)
  auto block_any = [&](bool p) {
    if (tid == 0) *s_flag = 0;
    __syncthreads();
    if (p) *s_flag = 1;
    __syncthreads();
    const bool r = *s_flag != 0;
    __syncthreads();
    return r;
  };
  // Binomial coefficients C(p, r), p, r <= 12 (exact integer products).
  for (int e = tid; e < kBinomW * kBinomW; e += nt) {
    const int p = e / kBinomW, r = e % kBinomW;
    int c = r <= p ? 1 : 0;
    for (int i = 1; i <= r && r <= p; ++i) c = c * (p - r + i) / i;
    s_binom[e] = c;
  }
  __syncthreads();
  if (tid <= kExactMaxItems + 1) {
    int o = 0;
    for (int j = 0; j < tid; ++j) o += s_binom[kExactMaxItems * kBinomW + j];
    s_layer[tid] = o;
  }
  __syncthreads();
  // Every 12-bit mask, ordered by popcount and then by value.  The position
  // of a k-subset among the k-subsets in increasing order is its
  // combinatorial rank sum_i C(b_i, i) over its set bits b_1 < ... < b_k;
  // the k-subsets of the low m bits are the first C(m, k) of the layer.
  for (int x = tid; x < kSubsets; x += nt) {
    int rank = 0, i = 0;
    for (int b = 0; b < kExactMaxItems; ++b)
      if ((x >> b) & 1) {
        ++i;
        rank += s_binom[b * kBinomW + i];
      }
    sList[s_layer[i] + rank] = (uint16_t)x;
  }
  __syncthreads();

  for (int inst = blockIdx.x; inst < a.num; inst += gridDim.x) {
    const int64_t off = a.item_off[inst], m64 = a.item_off[inst + 1] - off;
    const int c0 = a.cap_off[inst], n = a.cap_off[inst + 1] - c0;
    int err = (m64 < 1 || m64 > a.max_items || m64 > kExactMaxItems || n < 1 ||
               n > kMaxTypes || n > a.max_types)
                  ? kErrSize
                  : 0;
    const int m = err ? 0 : (int)m64;
    if (tid < kMaxTypes) s_caps[tid] = (!err && tid < n) ? a.caps[c0 + tid] : 0;
    if (tid < kExactMaxItems) s_w[tid] = tid < m ? a.w[off + tid] : 0;
    __syncthreads();
    int bad = 0;
    if (!err && tid < n) {
      const int32_t c = s_caps[tid];
      bad = (c <= 0 || (tid > 0 && c >= s_caps[tid - 1])) ? 1 : 0;
    }
    if (block_any(bad) && !err) err = kErrCaps;
    const int32_t B1 = s_caps[0];
    if (!err && B1 > a.max_cap) err = kErrSize;
    const int badw = (!err && tid < m && (s_w[tid] < 1 || s_w[tid] > B1)) ? 1 : 0;
    if (block_any(badw) && !err) err = kErrWeight;
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      continue;  // uniform: err depends only on values every thread has read
    }

    // block totals from two 64-entry tables (items 0-5 and 6-11), then the
    // block costs at the folded positions
    const uint32_t full = (1u << m) - 1u;
    if (tid < 128) {
      const int h = tid >> 6, x = tid & 63;
      int64_t sum = 0;
      for (int j = 0; j < 6; ++j) sum += ((x >> j) & 1) ? s_w[6 * h + j] : 0;
      s_half[tid] = sum;
    }
    __syncthreads();
    for (uint32_t T = tid; T <= full; T += nt) {
      const int64_t sum = s_half[T & 63] + s_half[64 + (T >> 6)];
      K c = kInf | (K)T;
      if (T != 0 && sum <= B1) {
        int32_t cap = B1;
        for (int k = 1; k < n; ++k)
          if (s_caps[k] >= sum) cap = s_caps[k];
        c = ((K)cap << 12) | (K)T;
      }
      sC[fold(T)] = c;
    }
    if (tid == 0) sG[0] = 0;  // fold(0) = 0
    __syncthreads();

    // layers by popcount
    for (int k = 1; k <= m; ++k) {
      const int lg = min(6, max(0, k - 6));
      const int g = 1 << lg;
      const int hi_bits = k - 1 - lg;  // free items walked in Gray order, 0..5
      const int iters = 1 << hi_bits;
      const int groups = nt >> lg;
      const int gid = tid >> lg, lig = tid & (g - 1);
      const int nS = s_binom[m * kBinomW + k];
      const uint16_t* list = sList + s_layer[k];
      for (int base = 0; base < nS; base += groups) {
        const int s = base + gid;
        const bool act = s < nS;
        // an idle group works on the one-item set {0}: in bounds, not stored
        const uint32_t S = act ? (uint32_t)list[s] : 1u;
        const uint32_t low = S & (0u - S);
        uint32_t rem = S ^ low, U = 0;
        // the lane's index fixes the lowest lg free items ...
        for (int j = 0; j < lg; ++j) {
          const uint32_t b = rem & (0u - rem);
          if ((lig >> j) & 1) U |= b;
          rem ^= b;
        }
        // ... and the others are toggled in Gray-code order
        uint32_t flip[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const uint32_t b = rem & (0u - rem);
          flip[j] = fold(b) * kSz;
          rem ^= b;
        }
        const uint32_t pt = g_base | (fold(U | low) * kSz), ps = fold(S) * kSz;
        K best;
        switch (hi_bits) {
          case 0: best = run_candidates<1, K>(pt, ps, flip); break;
          case 1: best = run_candidates<2, K>(pt, ps, flip); break;
          case 2: best = run_candidates<4, K>(pt, ps, flip); break;
          case 3: best = run_candidates<8, K>(pt, ps, flip); break;
          case 4: best = run_candidates<16, K>(pt, ps, flip); break;
          default: best = run_candidates<32, K>(pt, ps, flip); break;
        }
        (void)iters;
        for (int d = 1; d < g; d <<= 1) best = min(best, shfl_xor_k(best, d));
        if (act && lig == 0) {
          sG[fold(S)] = best & ~(K)kBlockBits;
          sB[S] = (uint16_t)(best & (K)kBlockBits);
        }
      }
      __syncthreads();
    }

    // the optimal partition, block by block from the full set
    if (tid == 0) {
      uint32_t S = full;
      int b = 0;
      // at most m blocks, each a non-empty subset of what is left
      while (S && b < m) {
        const uint32_t T = (uint32_t)sB[S] & S;
        if (!T) break;
        s_blocks[b++] = T;
        S ^= T;
      }
      *s_nb = b;
      a.nbins[inst] = b;
      a.cost[inst] = (int64_t)(sG[fold(full)] >> 12);
    }
    __syncthreads();
    const int nb = *s_nb;
    if (tid < m) {
      int b = 0;
      while (b < nb && !((s_blocks[b] >> tid) & 1u)) ++b;
      a.assign[off + tid] = b < nb ? b : -1;
    }
    if (tid < nb) {
      const int32_t cap = (int32_t)(sC[fold(s_blocks[tid])] >> 12);
      int t = 0;
      for (int k = 0; k < n; ++k)
        if (s_caps[k] == cap) t = k;
      a.types[off + tid] = t;
    }
    __syncthreads();
  }
}

// Raises the kernel's dynamic LDS limit above 64 KiB (64-bit keys) once.
template <typename K>
hipError_t prepare() {
  static const hipError_t e =
      exact_dyn_lds<K>() > 65536 ? allow_max_dynamic_lds(k_exact<K>) : hipSuccess;
  return e;
}

template <typename K>
hipError_t launch_t(const BatchArgs& a, int block, int grid, hipStream_t s) {
  const hipError_t e = prepare<K>();
  if (e != hipSuccess) return e;
  if (grid <= 0 || grid > a.num) grid = a.num;
  hipLaunchKernelGGL(k_exact<K>, dim3(grid), dim3(block), exact_dyn_lds<K>(), s, a);
  return hipGetLastError();
}

template <typename K>
int blocks_per_cu_t(int block) {
  int nb = 0;
  if (prepare<K>() != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_exact<K>, block,
                                                   exact_dyn_lds<K>()) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace

bool exact_wide(const BatchArgs& a) {
  return (int64_t)a.max_items * (int64_t)a.max_cap >= (int64_t)1 << 19;
}

hipError_t launch_exact(const BatchArgs& a, int block, int grid, hipStream_t s) {
  if (a.num <= 0) return hipSuccess;
  return exact_wide(a) ? launch_t<uint64_t>(a, block, grid, s)
                       : launch_t<uint32_t>(a, block, grid, s);
}

int exact_blocks_per_cu(const BatchArgs& a, int block) {
  // resident workgroups per CU, by key width, for the one block size in use
  static const int n32 = blocks_per_cu_t<uint32_t>(block);
  static const int n64 = blocks_per_cu_t<uint64_t>(block);
  return exact_wide(a) ? n64 : n32;
}

}  // namespace vsbpp
