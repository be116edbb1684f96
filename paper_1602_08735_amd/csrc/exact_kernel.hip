// Exact optimum of small VSBPP instances (m <= 12 items), a batch at a time.
//
// Cost model of the problem statement (Section 2): a bin of type k costs its
// capacity B_k, a packing costs the sum over its used bins.  A block of items
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
// when the grid is smaller), every table in LDS:
//   F[S] = (f(S) << 12) | T*(S)   the optimum of S and the block it starts with
//   C[T] = (c(T) << 12) | T       the block cost with the block in the low bits
//                                  (c(T) = INF when T does not fit any bin)
// so one key addition (F[S\T] with its low bits cleared) + C[T] gives a
// candidate whose minimum is the optimum with the smallest block mask among
// the optimal ones.  Subsets are processed by popcount: every subset of
// popcount k depends only on smaller ones, so one layer is one parallel
// step.  In layer k each subset has 2^(k-1) candidate blocks; a group of g
// lanes shares a subset (g = 2^(k-4) clamped to [1,64], so each lane takes at
// least 8 candidates when there are that many) and lane l visits the
// candidates whose index is l mod g: the index is kept "deposited" into the
// bits of the subset, and advancing it by g is one masked addition.  The
// group then reduces its minimum with cross-lane exchanges.
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

template <typename K>
size_t exact_dyn_lds() {
  return 2 * sizeof(K) * kSubsets + sizeof(uint16_t) * kSubsets;
}

template <typename K>
__global__ void __launch_bounds__(512) k_exact(BatchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  K* sF = reinterpret_cast<K*>(smem);
  K* sC = sF + kSubsets;
  uint16_t* sList = reinterpret_cast<uint16_t*>(sC + kSubsets);
  __shared__ int32_t s_binom[kBinomW * kBinomW];
  __shared__ int32_t s_layer[kExactMaxItems + 2];
  __shared__ int32_t s_caps[kMaxTypes];
  __shared__ int32_t s_w[kExactMaxItems];
  __shared__ uint32_t s_blocks[kExactMaxItems];
  __shared__ int32_t s_nb;
  constexpr K kInf = ExactKey<K>::kInf;
  const int tid = threadIdx.x, nt = blockDim.x;

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
    if (__syncthreads_or(bad) && !err) err = kErrCaps;
    const int32_t B1 = s_caps[0];
    if (!err && B1 > a.max_cap) err = kErrSize;
    const int badw = (!err && tid < m && (s_w[tid] < 1 || s_w[tid] > B1)) ? 1 : 0;
    if (__syncthreads_or(badw) && !err) err = kErrWeight;
    if (err) {
      if (tid == 0) {
        a.nbins[inst] = err;
        a.cost[inst] = 0;
      }
      continue;  // uniform: err depends only on values every thread has read
    }

    // block costs
    const uint32_t full = (1u << m) - 1u;
    int32_t wr[kExactMaxItems];
#pragma unroll
    for (int j = 0; j < kExactMaxItems; ++j) wr[j] = s_w[j];
    for (uint32_t T = tid; T <= full; T += nt) {
      int64_t sum = 0;
#pragma unroll
      for (int j = 0; j < kExactMaxItems; ++j) sum += ((T >> j) & 1u) ? wr[j] : 0;
      K c = kInf | (K)T;
      if (T != 0 && sum <= B1) {
        int32_t cap = B1;
        for (int k = 1; k < n; ++k)
          if (s_caps[k] >= sum) cap = s_caps[k];
        c = ((K)cap << 12) | (K)T;
      }
      sC[T] = c;
    }
    if (tid == 0) sF[0] = 0;
    __syncthreads();

    // layers by popcount
    for (int k = 1; k <= m; ++k) {
      const int lg = min(6, max(0, k - 4));
      const int g = 1 << lg;
      const int iters = (1 << (k - 1)) >> lg;
      const int groups = nt >> lg;
      const int gid = tid >> lg, lig = tid & (g - 1);
      const int nS = s_binom[m * kBinomW + k];
      const uint16_t* list = sList + s_layer[k];
      for (int base = 0; base < nS; base += groups) {
        const int s = base + gid;
        const bool act = s < nS;
        // an idle group works on the one-item set {0}: in bounds, not stored
        const uint32_t S = act ? (uint32_t)list[s] : 1u;
        const uint32_t low = S & (0u - S), R = S ^ low;
        // deposit the lane's index into the bits of R; D = deposit of g
        uint32_t U = 0, rem = R;
        for (int j = 0; j < lg; ++j) {
          const uint32_t b = rem & (0u - rem);
          if ((lig >> j) & 1) U |= b;
          rem ^= b;
        }
        const uint32_t D = rem & (0u - rem);
        K best = ~(K)0;
        for (int i = 0; i < iters; ++i) {
          const uint32_t T = U | low;
          const K v = (sF[S ^ T] & ~(K)kBlockBits) + sC[T];
          best = min(best, v);
          U = ((U | ~R) + D) & R;
        }
        for (int d = 1; d < g; d <<= 1) best = min(best, shfl_xor_k(best, d));
        if (act && lig == 0) sF[S] = best;
      }
      __syncthreads();
    }

    // the optimal partition, block by block from the full set
    if (tid == 0) {
      uint32_t S = full;
      int b = 0;
      // at most m blocks, each a non-empty subset of what is left
      while (S && b < m) {
        const uint32_t T = (uint32_t)(sF[S] & (K)kBlockBits) & S;
        if (!T) break;
        s_blocks[b++] = T;
        S ^= T;
      }
      s_nb = b;
      a.nbins[inst] = b;
      a.cost[inst] = (int64_t)(sF[full] >> 12);
    }
    __syncthreads();
    const int nb = s_nb;
    if (tid < m) {
      int b = 0;
      while (b < nb && !((s_blocks[b] >> tid) & 1u)) ++b;
      a.assign[off + tid] = b < nb ? b : -1;
    }
    if (tid < nb) {
      const int b = tid;
      const int32_t cap = (int32_t)(sC[s_blocks[b]] >> 12);
      int t = 0;
      for (int k = 0; k < n; ++k)
        if (s_caps[k] == cap) t = k;
      a.types[off + b] = t;
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
