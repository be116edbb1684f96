// Batch runs with a chosen launch shape for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  A plan keeps its work counter and instance schedule in
// a workspace it allocates; here they sit in one file-scope device array,
// one copy per GPU, whose address is looked up once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/vsbpp.h"
#include "host_internal.h"
#include "kernels.h"

// [0] work counter of persistent launches; [1 .. kLptMax] the largest-first
// instance schedule.  32 KiB + 4 bytes per GPU, held until the process ends.
// Host code never names this array as a device address: it uses the address
// hipGetSymbolAddress returns for the current device.
static constexpr int kScratchInts = 1 + vsbpp::kLptMax;
static __device__ __align__(256) int32_t scratch[kScratchInts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device, with the device current).
int32_t scratch_ptr(int32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    vsbpp::set_last_error("hipGetDevice", e);
    (void)hipGetLastError();
    return VSBPP_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) return VSBPP_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      vsbpp::set_last_error("hipGetSymbolAddress(scratch)", e);
      (void)hipGetLastError();
      return VSBPP_E_DEVICE;
    }
    g_scratch[dev] = static_cast<int32_t*>(p);
  }
  *out = g_scratch[dev];
  return VSBPP_OK;
}

}  // namespace

extern "C" int32_t vsbpp_pack_batch_static(const vsbpp_batch* b, int32_t heuristic,
                                           const vsbpp_options* opt,
                                           const vsbpp_launch* launch, void* hip_stream) {
  vsbpp_options o = vsbpp::resolve_options(opt);
  const bool learned = o.type_rule == VSBPP_TYPE_LEARNED;
  if (learned) o.type_rule = VSBPP_TYPE_SMALLEST_FIT;  // for the shared checks
  int32_t rc = vsbpp::check_batch(b, heuristic, o);
  if (rc != VSBPP_OK) return rc;
  // no model argument: the learned rules cannot run here
  if (learned || o.criterion_rule == 1 || o.choice_rule == 2) return VSBPP_E_MODEL;
  if (b->num_instances == 0) return VSBPP_OK;
  vsbpp::BatchArgs a = vsbpp::batch_args(*b, o);
  vsbpp::LaunchCfg c = vsbpp::default_cfg(heuristic, a);
  if (launch) {
    c.mode = launch->mode;
    c.lpt = launch->lpt;
    c.wpb = launch->waves_per_block;
    c.block = launch->block_threads;
    c.seg = launch->lanes_per_instance == 0 ? 64 : launch->lanes_per_instance;
    c.wpi = launch->waves_per_instance == 0 ? 1 : launch->waves_per_instance;
  }
  // the schedule holds at most kLptMax instances
  if (c.lpt == 1 && a.num > vsbpp::kLptMax) return VSBPP_E_SIZE;
  rc = vsbpp::check_cfg(c, heuristic, a);
  if (rc != VSBPP_OK) return rc;
  if (!vsbpp::device_info().ok) return VSBPP_E_DEVICE;
  int32_t* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc != VSBPP_OK) return rc;
  // No device region for bins beyond LDS: such plain runs return
  // VSBPP_E_SIZE from the enqueue (a.spill stays null).  The counter is reset
  // by a kernel on the stream before the pack kernel reads it.
  return vsbpp::enqueue_batch(a, heuristic, c, ws, ws + 1, (hipStream_t)hip_stream);
}
