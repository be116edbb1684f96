// Host-side runtime shared by the C-ABI entry points: device probing, launch
// shapes and the enqueue sequence of one batch run.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.h"

namespace vsbpp {

struct DevInfo {
  bool probed = false;
  bool ok = false;
  int max_lds_block = 65536;
  int cus = 1;
};

// Probes the current device once (thread-safe); ok is false without a gfx950.
const DevInfo& device_info();

struct LaunchCfg {
  int mode = 0;   // 0 grid over the batch, 1 persistent
  int lpt = 0;    // largest instances first
  int wpb = 4;    // FF/BF/WF wavefronts per workgroup
  int block = 256;  // H1/H2 workgroup size
  int seg = 64;   // FF/BF/WF lanes per instance (64, or 16/32: several
                  // instances per wavefront)
  int wpi = 1;    // FF/BF/WF wavefronts per instance (1, or 2/4 sharing one
                  // instance's bins)
};

// Plain runs that the several-instances-per-wavefront kernel takes: 32-bit
// keys, no scorer, decision hooks or bound on the open bins.
bool seg_eligible(const BatchArgs& a, int heuristic);
// Plain runs that the several-wavefronts-per-instance kernel takes.
bool mw_eligible(const BatchArgs& a, int heuristic);

// Shape-independent checks of a launch configuration for a batch; returns a
// VSBPP_E_* code or 0.
int32_t check_cfg(const LaunchCfg& c, int heuristic, const BatchArgs& a);
LaunchCfg default_cfg(int heuristic, const BatchArgs& a);
std::vector<LaunchCfg> candidate_cfgs(int heuristic, const BatchArgs& a);

// Bytes of the device region a plain FF/BF/WF run needs when an instance's
// bins do not fit a workgroup's LDS (num instances x the per-wavefront
// arrays), 0 when they fit; -1 when they fit neither (decision hooks and the
// scorer run from LDS only).  The region goes in BatchArgs::spill.
int64_t plain_spill_bytes(const BatchArgs& a, int heuristic);

// Records the HIP failure behind a VSBPP_E_DEVICE for vsbpp_last_error.
void set_last_error(const char* where, hipError_t e);

// Options with the caller's struct (any declared size) over the defaults.
vsbpp_options resolve_options(const vsbpp_options* opt);

// Kernel arguments of a device batch under resolved options (no scorer, no
// decision hooks, no device region).
BatchArgs batch_args(const vsbpp_batch& b, const vsbpp_options& o);

// Host-visible checks shared by the batch entry points: the batch
// descriptor's pointers and bounds, the heuristic and the options.  Returns a
// VSBPP_E_* code or 0.
int32_t check_batch(const vsbpp_batch* b, int32_t heuristic, const vsbpp_options& o);

// Enqueues one run: [queue reset] [LPT schedule] pack kernel.  `queue` and
// `sched` are device workspace (may be null when the configuration needs
// neither).  Returns a VSBPP_* code.
int32_t enqueue_batch(BatchArgs a, int heuristic, const LaunchCfg& c, int32_t* queue,
                      int32_t* sched, hipStream_t s);

}  // namespace vsbpp
