// Kernel-side argument block and launch entry points shared by the C-ABI
// host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vsbpp.h"

namespace vsbpp {

// error codes written to nbins[i] for instances that fail device-side checks
// (same values as the public VSBPP_E_* codes)
constexpr int32_t kErrSize = -2, kErrCaps = -3, kErrWeight = -4, kErrOption = -6;

constexpr int kMaxTypes = 16;

struct BatchArgs {
  const int32_t* w;         // CSR weights
  const int64_t* item_off;  // [num+1]
  const int32_t* caps;      // CSR capacities, strictly decreasing per instance
  const int32_t* cap_off;   // [num+1]
  const int32_t* order;     // optional CSR ordering (local item ids), or null
  const uint64_t* seeds;    // optional per-instance generator keys, or null
  uint64_t seed;            // key used when seeds is null
  int32_t* assign;          // [sum m]
  int32_t* types;           // [sum m]
  int32_t* nbins;           // [num]
  int64_t* cost;            // [num]
  int32_t num;              // instances
  int32_t max_items;        // per-instance bound guaranteed by the caller
  int32_t max_cap;          // bound on B_1 guaranteed by the caller
  int32_t max_types;        // bound on n guaranteed by the caller
  int32_t type_rule;        // 0 smallest fit, 1 largest
  int32_t force_crit;       // -1 or 0/1/2 (H1/H2 only)
  int32_t active_limit;     // plain FF/BF/WF: bins open at once (0: no limit)
  int32_t downsize;         // 1: a pass after packing gives every bin its smallest type
  int32_t criterion_rule;   // H1: 0 Rule 3's draw, 1 the model picks FF/BF/WF
  int32_t rule2_order;      // H1/H2: Rule 2's empty bins B_1 first (0) or B_n first (1)
  int32_t choice_rule;      // plain FF/BF/WF (largest type, downsizing): 0 off, 1 contested
                            // placements are the decisions, 2 the model keeps or opens
  int32_t s1;               // H1 items per sublist
  int32_t s2;               // H2 subset size
  int32_t slots;            // plain kernel: LDS key slots per wavefront
  int32_t* queue;           // persistent mode: work counter (zeroed before the launch), or null
  const int32_t* sched;     // optional processing order of the instances (LPT), or null
  // decision hooks and the scorer (plain FF/BF/WF only)
  const int32_t* src;       // entry -> source instance, or null
  const int32_t* force;     // [3*num] (d, t1, t2), or null
  float* feat_out;          // [16*num], or null
  int32_t* info_out;        // [2*num], or null
  int32_t* count_out;       // [num] decisions of each run, or null
  const vsbpp_model* model; // type_rule 2
  // plain kernel: a device region of per-wave bytes per instance that holds
  // the wavefront's arrays when they do not fit LDS, or null
  unsigned char* spill;
};

// Next instance for a wavefront (plain kernel) or a workgroup (H1/H2): a
// static stride over the grid, or a global work counter in persistent mode.
// `slot` is a per-caller cursor for the static mode.

// Lets `kern` use all of the device's LDS per workgroup that its own static
// LDS leaves free (needed above 64 KiB of dynamic LDS); once per kernel.
template <typename Kern>
hipError_t allow_max_dynamic_lds(Kern kern) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  int dev = 0, maxb = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&maxb, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             maxb - (int)fa.sharedSizeBytes);
}

// LDS budget reserved for the static LDS of the H1/H2 kernels
constexpr int kStaticLdsReserve = 1024;

// Launch helpers (defined next to their kernels).  They return a hipError_t.
// ext: decision hooks or the scorer in use
// ds_loads: per-bin loads kept for the downsized cost of entries that name a
// source instance (their bin types are not written, so no pass follows)
size_t plain_lds_per_wave(int slots, int max_items, bool wide, bool ext = false,
                          bool ds_loads = false);
__host__ __device__ inline bool plain_ds_loads(const BatchArgs& a) {
  return a.downsize && a.src;
}
size_t plain_lds_block_extra(bool learned);
inline bool plain_ext(const BatchArgs& a) {
  return a.src || a.force || a.feat_out || a.info_out || a.count_out || a.type_rule == 2 ||
         a.choice_rule == 2;
}
// plain runs with the learned bin-type rule alone: no decision hooks, bin
// choice or bound on the open bins (a lean instantiation of the scorer kernel)
inline bool plain_lean_learned(const BatchArgs& a) {
  return a.type_rule == 2 && a.choice_rule == 0 && !a.src && !a.force && !a.feat_out &&
         !a.info_out && !a.count_out && a.active_limit == 0;
}
// plain runs that evaluate the network (bin-type scorer or bin choice)
__host__ __device__ inline bool plain_scored(const BatchArgs& a) {
  return a.type_rule == 2 || a.choice_rule == 2;
}
// learned: the variant that scores the criterion (or dumps its features)
size_t h1_lds_bytes(int nbslots, int s1, int block, bool wide, bool learned = false);
// H1 runs that take the criterion-scoring variant
inline bool h1_learned(const BatchArgs& a) {
  return a.criterion_rule == 1 || a.feat_out || a.info_out;
}
constexpr int32_t kErrModel = -9;
// largest workgroup of the criterion-scoring H1 variant (its network needs
// more than 128 registers per lane)
constexpr int kH1LearnedMaxBlock = 512;
// H2 kernels: one 32-bit key word per bin with a chunk of resolved positions
// (the fast form), 64-bit bins (wide batches)
enum class H2Kernel { kSlim, kWide };
size_t h2_lds_bytes(int nbslots, int block, int group, H2Kernel k);
int h2_group(int s2);
hipError_t launch_best_of(const int64_t* cost, int32_t num, int64_t* out, hipStream_t s);

// per-instance (sum of weights, LB_cap, LB_big); LB_cap is exact when the
// smallest capacity is <= 8192, else the sum of weights
hipError_t launch_bounds(int32_t num, const int32_t* w, const int64_t* item_off,
                         const int32_t* caps, const int32_t* cap_off, int64_t* out,
                         hipStream_t s);

// downsizing pass over a packed batch (bin types and costs rewritten)
hipError_t launch_downsize(const BatchArgs& a, hipStream_t s);

// exact optimum of instances with at most 12 items (subset dynamic
// programme, one workgroup of `block` threads (128..512, a multiple of 64)
// per instance; grid = 0: one workgroup per instance, else a static stride)
constexpr int kExactMaxItems = 12;
bool exact_wide(const BatchArgs& a);
hipError_t launch_exact(const BatchArgs& a, int block, int grid, hipStream_t s);
int exact_blocks_per_cu(const BatchArgs& a, int block);

// scheduling helpers
hipError_t launch_queue_reset(int32_t* queue, hipStream_t s);
// instances sorted by decreasing item count (ties by index); num <= kLptMax
constexpr int kLptMax = 8192;
hipError_t launch_lpt_schedule(const int64_t* item_off, int32_t num, int32_t* sched, hipStream_t s);

// launch shapes; grid = 0 means one wavefront/workgroup per instance
hipError_t launch_plain_grid(const BatchArgs& a, int crit, bool wide, int waves_per_block,
                             size_t lds_per_wave, int grid, hipStream_t s);
// plain FF/BF/WF with several instances per wavefront: `seg` lanes (16 or
// 32) per instance, 32-bit keys, no scorer, hooks, bound or device region
size_t plain_seg_stride(int slots, int max_items);
hipError_t launch_plain_seg(const BatchArgs& a, int crit, int seg, int wpb, size_t seg_stride,
                            int grid, hipStream_t s);
int plain_seg_blocks_per_cu(int crit, int seg, int wpb, size_t seg_stride);
// plain FF/BF/WF with wpi = 2 or 4 wavefronts per instance (one workgroup
// each), 32-bit keys, no scorer, hooks, bound or device region; LDS bytes per
// workgroup for a.slots key slots
size_t plain_mw_lds(int slots, int max_items);
hipError_t launch_plain_mw(const BatchArgs& a, int crit, int wpi, int grid, hipStream_t s);
int plain_mw_blocks_per_cu(int crit, int wpi, size_t lds);
hipError_t launch_h1_grid(const BatchArgs& a, bool wide, int nb_regs, int block_threads,
                          int grid, hipStream_t s);
hipError_t launch_h2_grid(const BatchArgs& a, H2Kernel k, int nb_regs, int block_threads,
                          int grid, hipStream_t s);
// resident workgroups per CU for a launch shape (for persistent grids)
int plain_blocks_per_cu(const BatchArgs& a, int crit, bool wide, int waves_per_block,
                        size_t lds_per_wave);
int h1_blocks_per_cu(bool wide, int block_threads, size_t lds, bool learned = false);
int h2_blocks_per_cu(H2Kernel k, int block_threads, size_t lds);

}  // namespace vsbpp
