// C-ABI entry points: argument checks, launch planning and the synchronous
// host-pointer path.  Every packing step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/vsbpp.h"
#include "host_internal.h"
#include "kernels.h"

namespace {

using vsbpp::BatchArgs;

}  // namespace

namespace vsbpp {
int32_t check_options_public(const vsbpp_options& o);
int32_t check_heuristic_options_public(const vsbpp_options& o, int32_t heuristic);
vsbpp_options resolve_options(const vsbpp_options* opt);
}  // namespace vsbpp

namespace {

int32_t check_instance(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                       int32_t heuristic, const vsbpp_options& o, bool check_order) {
  if (!w || !caps) return VSBPP_E_NULL;
  if (m < 1 || n < 1 || n > vsbpp::kMaxTypes) return VSBPP_E_SIZE;
  for (int32_t k = 0; k < n; ++k) {
    if (caps[k] <= 0) return VSBPP_E_CAPS;
    if (k > 0 && caps[k] >= caps[k - 1]) return VSBPP_E_CAPS;
  }
  for (int32_t j = 0; j < m; ++j)
    if (w[j] < 1 || w[j] > caps[0]) return VSBPP_E_WEIGHT;
  if (heuristic < VSBPP_FF || heuristic > VSBPP_H2) return VSBPP_E_HEURISTIC;
  if (check_order && o.order) {
    std::vector<char> seen((size_t)m, 0);
    for (int32_t q = 0; q < m; ++q) {
      const int32_t j = o.order[q];
      if (j < 0 || j >= m || seen[(size_t)j]) return VSBPP_E_OPTION;
      seen[(size_t)j] = 1;
    }
  }
  return VSBPP_OK;
}

int32_t check_options(const vsbpp_options& o) {
  if (o.h1_items_per_sublist < 1 || o.h1_items_per_sublist > 16) return VSBPP_E_OPTION;
  if (o.h2_subset_size < 1 || o.h2_subset_size > 6) return VSBPP_E_OPTION;
  if (o.type_rule != VSBPP_TYPE_SMALLEST_FIT && o.type_rule != VSBPP_TYPE_LARGEST)
    return VSBPP_E_OPTION;
  if (o.force_criterion < -1 || o.force_criterion > VSBPP_WF) return VSBPP_E_OPTION;
  if (o.active_limit < 0) return VSBPP_E_OPTION;
  if (o.downsize != 0 && o.downsize != 1) return VSBPP_E_OPTION;
  if (o.criterion_rule != 0 && o.criterion_rule != 1) return VSBPP_E_OPTION;
  if (o.choice_rule < 0 || o.choice_rule > 2) return VSBPP_E_OPTION;
  if (o.rule2_order < 0 || o.rule2_order > 1) return VSBPP_E_OPTION;
  return VSBPP_OK;
}

// options that only some heuristics take
int32_t check_heuristic_options(const vsbpp_options& o, int32_t heuristic) {
  if (o.active_limit > 0 && heuristic > VSBPP_WF) return VSBPP_E_OPTION;
  if (o.rule2_order != 0 && heuristic <= VSBPP_WF) return VSBPP_E_OPTION;  // no Rule 2
  if (o.criterion_rule == 1 && (heuristic != VSBPP_H1 || o.force_criterion != -1))
    return VSBPP_E_OPTION;
  // the bin choice compares bins by their downsized capacity: plain rules,
  // bins opened at B_1, every bin downsized, no bound on the open bins
  if (o.choice_rule != 0 &&
      (heuristic > VSBPP_WF || o.type_rule != VSBPP_TYPE_LARGEST || o.downsize != 1 ||
       o.active_limit != 0))
    return VSBPP_E_OPTION;
  return VSBPP_OK;
}

vsbpp_options resolve(const vsbpp_options* opt) {
  vsbpp_options o;
  vsbpp_options_init(&o);
  if (opt) {
    // accept older/shorter option structs: copy what the caller declares
    size_t sz = opt->struct_size;
    if (sz == 0 || sz > sizeof(o)) sz = sizeof(o);
    std::memcpy(&o, opt, sz);
    o.struct_size = sizeof(o);
  }
  return o;
}

std::mutex g_mu;

int round_up(int x, int to) { return ((x + to - 1) / to) * to; }

}  // namespace

namespace vsbpp {

const DevInfo& device_info() {
  static DevInfo info;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (!info.probed) {
    info.probed = true;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
      (void)hipGetLastError();
      return info;
    }
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
      (void)hipGetLastError();
      return info;
    }
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return info;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
            hipSuccess &&
        lds > 0)
      info.max_lds_block = lds;
    info.cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 1;
    info.ok = true;
  }
  return info;
}

namespace {

bool is_wide(const BatchArgs& a) { return a.max_cap > 0x7FFF || a.max_items > 0xFFFF; }

struct PlainShape {
  int slots;
  size_t per_wave;
  int max_wpb;
  bool spill;  // the per-wave arrays live in a device region, not LDS
};

int32_t plain_shape(const BatchArgs& a, PlainShape* sh) {
  const bool wide = is_wide(a);
  sh->slots = round_up(a.max_items, 256);
  if (!wide && sh->slots > 65536) return VSBPP_E_SIZE;
  const bool ext = plain_ext(a);
  sh->per_wave = plain_lds_per_wave(sh->slots, a.max_items, wide, ext, plain_ds_loads(a));
  const size_t extra = ext ? plain_lds_block_extra(plain_scored(a)) : 0;
  sh->spill = (size_t)device_info().max_lds_block < extra + sh->per_wave;
  if (sh->spill) {
    if (ext) return VSBPP_E_SIZE;
    sh->max_wpb = 8;
    return VSBPP_OK;
  }
  sh->max_wpb = (int)(((size_t)device_info().max_lds_block - extra) / sh->per_wave);
  if (sh->max_wpb < 1) return VSBPP_E_SIZE;
  if (sh->max_wpb > 8) sh->max_wpb = 8;
  return VSBPP_OK;
}

int h_nbslots(int heuristic, const BatchArgs& a) {
  return round_up(a.max_types + 2 * (heuristic == VSBPP_H1 ? a.s1 : a.s2), 4);
}

// the H2 kernel: the slim kernel (32-bit bin words plus a chunk of resolved
// positions), or 64-bit bins for wide batches.  At the largest subset (s2 =
// 6, 16 types: 28 slots) the slim kernel needs 95 KB of LDS per 768-thread
// workgroup, well inside gfx950's 160 KB; h_fit_block shrinks larger
// workgroups to fit.
H2Kernel h2_kernel(const BatchArgs& a, int /*block*/) {
  return is_wide(a) ? H2Kernel::kWide : H2Kernel::kSlim;
}

size_t h_lds(int heuristic, const BatchArgs& a, int block) {
  const bool wide = is_wide(a);
  const int nbs = h_nbslots(heuristic, a);
  return heuristic == VSBPP_H1 ? h1_lds_bytes(nbs, a.s1, block, wide, h1_learned(a))
                               : h2_lds_bytes(nbs, block, h2_group(a.s2), h2_kernel(a, block));
}

// largest workgroup of the given granularity that fits the LDS budget
int h_fit_block(int heuristic, const BatchArgs& a, int want) {
  const int gran = heuristic == VSBPP_H2 ? h2_group(a.s2) : 64;
  int b = want < gran ? gran : (want / gran) * gran;
  if (b > 1024) b = (1024 / gran) * gran;
  if (heuristic == VSBPP_H1 && h1_learned(a) && b > kH1LearnedMaxBlock) b = kH1LearnedMaxBlock;
  const size_t budget = (size_t)(device_info().max_lds_block - kStaticLdsReserve);
  while (b > gran && h_lds(heuristic, a, b) > budget) b -= gran;
  if (h_lds(heuristic, a, b) > budget) return 0;
  return b;
}

// LDS layout of the several-instances-per-wavefront kernel: bytes per
// segment, and the most wavefronts per workgroup (at most 4) that fit; 0 when
// not even one fits
struct SegShape {
  int slots;
  size_t stride;
  int max_wpb;
};

SegShape seg_shape(const BatchArgs& a, int seg) {
  SegShape sh;
  sh.slots = round_up(a.max_items, 4 * seg);
  sh.stride = plain_seg_stride(sh.slots, a.max_items);
  const size_t per_wave = sh.stride * (size_t)(64 / seg);
  const size_t fit = (size_t)device_info().max_lds_block / per_wave;
  sh.max_wpb = fit > 4 ? 4 : (int)fit;
  return sh;
}

}  // namespace

bool mw_eligible(const BatchArgs& a, int heuristic) {
  if (heuristic > VSBPP_WF || is_wide(a) || plain_ext(a) || a.active_limit != 0 ||
      a.max_items < 1)
    return false;
  const size_t lds = plain_mw_lds(round_up(a.max_items, 256), a.max_items);
  return lds + 256 <= (size_t)device_info().max_lds_block;
}

bool seg_eligible(const BatchArgs& a, int heuristic) {
  return heuristic <= VSBPP_WF && !is_wide(a) && !plain_ext(a) && a.active_limit == 0 &&
         a.max_items >= 1 && (seg_shape(a, 16).max_wpb >= 1 || seg_shape(a, 32).max_wpb >= 1);
}

int32_t check_cfg(const LaunchCfg& c, int heuristic, const BatchArgs& a) {
  if (c.mode < 0 || c.mode > 1 || c.lpt < 0 || c.lpt > 1) return VSBPP_E_OPTION;
  if (c.lpt && a.num > kLptMax) return VSBPP_E_OPTION;
  if (c.seg != 64 && c.seg != 32 && c.seg != 16) return VSBPP_E_OPTION;
  if (c.wpi != 1 && c.wpi != 2 && c.wpi != 4) return VSBPP_E_OPTION;
  if (c.wpi != 1 && (c.seg != 64 || !mw_eligible(a, heuristic))) return VSBPP_E_OPTION;
  if (heuristic <= VSBPP_WF) {
    if (c.wpb < 1 || c.wpb > 8) return VSBPP_E_OPTION;
    if (c.seg != 64) {
      if (c.wpb > 4 || !seg_eligible(a, heuristic) || seg_shape(a, c.seg).max_wpb < 1)
        return VSBPP_E_OPTION;
    }
  } else {
    if (c.seg != 64) return VSBPP_E_OPTION;
    if (heuristic == VSBPP_H1 && h1_learned(a) && c.block > kH1LearnedMaxBlock)
      return VSBPP_E_OPTION;
    if (c.block < 64 || c.block > 1024 || (c.block & 63)) return VSBPP_E_OPTION;
    if (heuristic == VSBPP_H2 && (c.block % h2_group(a.s2))) return VSBPP_E_OPTION;
  }
  return VSBPP_OK;
}

LaunchCfg default_cfg(int heuristic, const BatchArgs& a) {
  LaunchCfg c;
  if (heuristic == VSBPP_H1) {
    const int packers = (a.max_items + a.s1 - 1) / a.s1;
    int b = round_up(packers, 64);
    c.block = b > 256 ? 256 : b;
  } else if (heuristic == VSBPP_H2) {
    const int g = h2_group(a.s2);
    c.block = g >= 256 ? g : 256;
  }
  return c;
}

std::vector<LaunchCfg> candidate_cfgs(int heuristic, const BatchArgs& a) {
  std::vector<LaunchCfg> v;
  const bool lpt_ok = a.num <= kLptMax;
  for (int mode = 0; mode <= 1; ++mode) {
    for (int lpt = 0; lpt <= (lpt_ok ? 1 : 0); ++lpt) {
      if (heuristic <= VSBPP_WF) {
        for (int wpb : {1, 2, 4, 8}) {
          LaunchCfg c;
          c.mode = mode;
          c.lpt = lpt;
          c.wpb = wpb;
          v.push_back(c);
        }
        if (mw_eligible(a, heuristic)) {
          for (int wpi : {2, 4}) {
            LaunchCfg c;
            c.mode = mode;
            c.lpt = lpt;
            c.wpi = wpi;
            v.push_back(c);
          }
        }
        if (seg_eligible(a, heuristic)) {
          for (int seg : {16, 32}) {
            const int mw = seg_shape(a, seg).max_wpb;  // 0: this width does not fit
            for (int wpb : {1, 2, 4}) {
              if (wpb > mw) continue;
              LaunchCfg c;
              c.mode = mode;
              c.lpt = lpt;
              c.wpb = wpb;
              c.seg = seg;
              v.push_back(c);
            }
          }
        }
      } else {
        const int gran = heuristic == VSBPP_H2 ? h2_group(a.s2) : 64;
        const int bmax = (heuristic == VSBPP_H1 && h1_learned(a)) ? kH1LearnedMaxBlock : 1024;
        for (int b = gran; b <= bmax; b *= 2) {
          if (b % gran) continue;
          LaunchCfg c;
          c.mode = mode;
          c.lpt = lpt;
          c.block = b;
          v.push_back(c);
        }
      }
    }
  }
  return v;
}

thread_local char g_last_error[256] = "";

void set_last_error(const char* where, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorString(e),
                (int)e);
}

int64_t plain_spill_bytes(const BatchArgs& a, int heuristic) {
  if (heuristic > VSBPP_WF || a.num <= 0 || a.max_items < 1) return 0;
  PlainShape sh;
  if (plain_shape(a, &sh) != VSBPP_OK) return -1;
  return sh.spill ? (int64_t)sh.per_wave * (int64_t)a.num : 0;
}

BatchArgs batch_args(const vsbpp_batch& b, const vsbpp_options& o) {
  BatchArgs a{};
  a.w = b.weights;
  a.item_off = b.item_off;
  a.caps = b.capacities;
  a.cap_off = b.cap_off;
  a.order = b.order;
  a.seeds = b.seeds;
  a.seed = o.seed;
  a.assign = b.assignment;
  a.types = b.bin_types;
  a.nbins = b.nbins;
  a.cost = b.cost;
  a.num = b.num_instances;
  a.max_items = b.max_items;
  a.max_cap = b.max_capacity;
  a.max_types = b.max_types;
  a.type_rule = o.type_rule;
  a.force_crit = o.force_criterion;
  a.active_limit = o.active_limit;
  a.downsize = o.downsize;
  a.criterion_rule = o.criterion_rule;
  a.choice_rule = o.choice_rule;
  a.rule2_order = o.rule2_order;
  a.s1 = o.h1_items_per_sublist;
  a.s2 = o.h2_subset_size;
  return a;
}

int32_t check_batch(const vsbpp_batch* b, int32_t heuristic, const vsbpp_options& o) {
  if (!b) return VSBPP_E_NULL;
  if (b->num_instances < 0) return VSBPP_E_SIZE;
  if (b->num_instances > 0 &&
      (!b->weights || !b->item_off || !b->capacities || !b->cap_off || !b->assignment ||
       !b->bin_types || !b->nbins || !b->cost))
    return VSBPP_E_NULL;
  if (b->max_items < 1 || b->max_types < 1 || b->max_types > kMaxTypes || b->max_capacity < 1)
    return VSBPP_E_SIZE;
  if (heuristic < VSBPP_FF || heuristic > VSBPP_H2) return VSBPP_E_HEURISTIC;
  int32_t rc = check_options(o);
  if (rc == VSBPP_OK) rc = check_heuristic_options(o, heuristic);
  return rc;
}

int32_t enqueue_batch(BatchArgs a, int heuristic, const LaunchCfg& c, int32_t* queue,
                      int32_t* sched, hipStream_t s) {
  if (a.num <= 0) return VSBPP_OK;
  const DevInfo& d = device_info();
  const bool wide = is_wide(a);
  hipError_t e = hipSuccess;
  a.queue = nullptr;
  a.sched = nullptr;
  if ((c.mode == 1 && !queue) || (c.lpt && !sched)) return VSBPP_E_OPTION;
  if (c.lpt) {
    e = launch_lpt_schedule(a.item_off, a.num, sched, s);
    if (e != hipSuccess) goto fail;
    a.sched = sched;
  }
  if (c.mode == 1) {
    e = launch_queue_reset(queue, s);
    if (e != hipSuccess) goto fail;
    a.queue = queue;
  }
  if (heuristic <= VSBPP_WF && c.wpi != 1) {
    // several wavefronts per instance
    if (!mw_eligible(a, heuristic)) return VSBPP_E_OPTION;
    a.spill = nullptr;
    a.slots = round_up(a.max_items, 256);
    int grid = 0;
    if (c.mode == 1)
      grid = d.cus * plain_mw_blocks_per_cu(heuristic, c.wpi, plain_mw_lds(a.slots, a.max_items));
    e = launch_plain_mw(a, heuristic, c.wpi, grid, s);
  } else if (heuristic <= VSBPP_WF && c.seg != 64) {
    // several instances per wavefront
    if (!seg_eligible(a, heuristic)) return VSBPP_E_OPTION;
    const SegShape sh = seg_shape(a, c.seg);
    if (sh.max_wpb < 1) return VSBPP_E_OPTION;
    a.spill = nullptr;
    a.slots = sh.slots;
    const int wpb = c.wpb < sh.max_wpb ? c.wpb : sh.max_wpb;
    int grid = 0;
    if (c.mode == 1) grid = d.cus * plain_seg_blocks_per_cu(heuristic, c.seg, wpb, sh.stride);
    e = launch_plain_seg(a, heuristic, c.seg, wpb, sh.stride, grid, s);
  } else if (heuristic <= VSBPP_WF) {
    PlainShape sh;
    int32_t rc = plain_shape(a, &sh);
    if (rc != VSBPP_OK) return rc;
    // arrays beyond LDS need the caller's device region (plans and the
    // host-pointer calls provide one)
    if (sh.spill && !a.spill) return VSBPP_E_SIZE;
    if (!sh.spill) a.spill = nullptr;
    a.slots = sh.slots;
    const int wpb = c.wpb < sh.max_wpb ? c.wpb : sh.max_wpb;
    int grid = 0;
    if (c.mode == 1) grid = d.cus * plain_blocks_per_cu(a, heuristic, wide, wpb, sh.per_wave);
    e = launch_plain_grid(a, heuristic, wide, wpb, sh.per_wave, grid, s);
  } else {
    const int block = h_fit_block(heuristic, a, c.block);
    if (block == 0) return VSBPP_E_SIZE;
    const int nbs = h_nbslots(heuristic, a);
    int grid = 0;
    if (c.mode == 1) {
      const size_t lds = h_lds(heuristic, a, block);
      grid = d.cus * (heuristic == VSBPP_H1 ? h1_blocks_per_cu(wide, block, lds, h1_learned(a))
                                            : h2_blocks_per_cu(h2_kernel(a, block), block, lds));
    }
    e = heuristic == VSBPP_H1 ? launch_h1_grid(a, wide, nbs, block, grid, s)
                              : launch_h2_grid(a, h2_kernel(a, block), nbs, block, grid, s);
  }
  // (entries with a source instance sum their downsized cost in the kernel)
  if (e == hipSuccess && a.downsize && !a.src) {
    e = launch_downsize(a, s);
    if (e != hipSuccess) {
      set_last_error("downsize launch", e);
      (void)hipGetLastError();
      return VSBPP_E_DEVICE;
    }
  }
  if (e == hipSuccess) return VSBPP_OK;
fail:
  set_last_error(heuristic <= VSBPP_WF ? "plain launch" : heuristic == VSBPP_H1 ? "H1 launch"
                                                                               : "H2 launch",
                 e);
  (void)hipGetLastError();
  return VSBPP_E_DEVICE;
}

}  // namespace vsbpp

namespace {

bool device_ok_locked() { return vsbpp::device_info().ok; }

int32_t launch_batch(BatchArgs a, int32_t heuristic, hipStream_t s) {
  return vsbpp::enqueue_batch(a, heuristic, vsbpp::default_cfg(heuristic, a), nullptr, nullptr,
                              s);
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t n) { return hipMalloc(&p, sizeof(T) * (n ? n : 1)) == hipSuccess; }
};

}  // namespace

extern "C" {

void vsbpp_options_init(vsbpp_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(*opt);
  opt->seed = 0;
  opt->h1_items_per_sublist = 10;
  opt->h2_subset_size = 5;
  opt->type_rule = VSBPP_TYPE_SMALLEST_FIT;
  opt->force_criterion = -1;
  opt->order = nullptr;
  opt->active_limit = 0;
  opt->downsize = 0;
  opt->criterion_rule = 0;
  opt->choice_rule = 0;
  opt->rule2_order = 0;
}

const char* vsbpp_strerror(int32_t code) {
  switch (code) {
    case VSBPP_OK: return "ok";
    case VSBPP_E_NULL: return "null pointer argument";
    case VSBPP_E_SIZE: return "size out of range (m, n or a declared bound)";
    case VSBPP_E_CAPS: return "capacities must be positive and strictly decreasing";
    case VSBPP_E_WEIGHT: return "weights must lie in [1, B_1]";
    case VSBPP_E_HEURISTIC: return "unknown heuristic";
    case VSBPP_E_OPTION: return "invalid option";
    case VSBPP_E_DEVICE: return "no usable gfx950 device, or a HIP runtime error";
    case VSBPP_E_NOMEM: return "device memory allocation failed";
    case VSBPP_E_MODEL: return "learned type rule without a usable model";
    default: return code >= 0 ? "ok" : "unknown error";
  }
}

const char* vsbpp_last_error(void) { return vsbpp::g_last_error; }

int32_t vsbpp_device_ok(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device_ok_locked() ? 1 : 0;
}

int32_t vsbpp_pack_ex(const int32_t* weights, int32_t m, const int32_t* capacities, int32_t n,
                      int32_t heuristic, const vsbpp_options* opt, int32_t* out_assignment,
                      int32_t* out_bin_types, int64_t* out_cost) {
  const vsbpp_options o = resolve(opt);
  if (!out_assignment || !out_bin_types) return VSBPP_E_NULL;
  int32_t rc = check_instance(weights, m, capacities, n, heuristic, o, true);
  if (rc != VSBPP_OK) return rc;
  rc = check_options(o);
  if (rc == VSBPP_OK) rc = check_heuristic_options(o, heuristic);
  if (rc != VSBPP_OK) return rc;
  if (o.criterion_rule == 1 || o.choice_rule == 2) return VSBPP_E_MODEL;  // this call takes no model

  std::lock_guard<std::mutex> lk(g_mu);
  if (!device_ok_locked()) return VSBPP_E_DEVICE;

  DevBuf<int32_t> dw, dc, dord, dassign, dtypes, dnb, dcoff;
  DevBuf<int64_t> doff, dcost;
  if (!dw.alloc((size_t)m) || !dc.alloc((size_t)n) || !dassign.alloc((size_t)m) ||
      !dtypes.alloc((size_t)m) || !dnb.alloc(1) || !dcoff.alloc(2) || !doff.alloc(2) ||
      !dcost.alloc(1) || (o.order && !dord.alloc((size_t)m)))
    return VSBPP_E_NOMEM;
  const int64_t hoff[2] = {0, m};
  const int32_t hcoff[2] = {0, n};
  hipStream_t s = nullptr;
  bool ok = hipMemcpy(dw.p, weights, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(dc.p, capacities, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(doff.p, hoff, sizeof(hoff), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(dcoff.p, hcoff, sizeof(hcoff), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && o.order)
    ok = hipMemcpy(dord.p, o.order, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice) ==
         hipSuccess;
  if (!ok) return VSBPP_E_DEVICE;

  BatchArgs a{};
  a.w = dw.p;
  a.item_off = doff.p;
  a.caps = dc.p;
  a.cap_off = dcoff.p;
  a.order = o.order ? dord.p : nullptr;
  a.seeds = nullptr;
  a.seed = o.seed;
  a.assign = dassign.p;
  a.types = dtypes.p;
  a.nbins = dnb.p;
  a.cost = dcost.p;
  a.num = 1;
  a.max_items = m;
  a.max_cap = capacities[0];
  a.max_types = n;
  a.type_rule = o.type_rule;
  a.force_crit = o.force_criterion;
  a.active_limit = o.active_limit;
  a.downsize = o.downsize;
  a.rule2_order = o.rule2_order;
  a.s1 = o.h1_items_per_sublist;
  a.s2 = o.h2_subset_size;
  DevBuf<unsigned char> dspill;
  const int64_t spill = plain_spill_bytes(a, heuristic);
  if (spill < 0) return VSBPP_E_SIZE;
  if (spill > 0) {
    if (!dspill.alloc((size_t)spill)) return VSBPP_E_NOMEM;
    a.spill = dspill.p;
  }
  rc = launch_batch(a, heuristic, s);
  if (rc != VSBPP_OK) return rc;
  if (hipStreamSynchronize(s) != hipSuccess) return VSBPP_E_DEVICE;
  int32_t nb = 0;
  int64_t cost = 0;
  if (hipMemcpy(&nb, dnb.p, sizeof(nb), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&cost, dcost.p, sizeof(cost), hipMemcpyDeviceToHost) != hipSuccess)
    return VSBPP_E_DEVICE;
  if (nb < 0) return nb;
  std::vector<int32_t> ha((size_t)m), ht((size_t)nb);
  if (hipMemcpy(ha.data(), dassign.p, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(ht.data(), dtypes.p, sizeof(int32_t) * (size_t)nb, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return VSBPP_E_DEVICE;
  std::memcpy(out_assignment, ha.data(), sizeof(int32_t) * (size_t)m);
  std::memcpy(out_bin_types, ht.data(), sizeof(int32_t) * (size_t)nb);
  if (out_cost) *out_cost = cost;
  return nb;
}

int32_t vsbpp_pack(const int32_t* weights, int32_t m, const int32_t* capacities, int32_t n,
                   int32_t heuristic, int32_t* out_assignment, int32_t* out_bin_types) {
  return vsbpp_pack_ex(weights, m, capacities, n, heuristic, nullptr, out_assignment,
                       out_bin_types, nullptr);
}

int32_t vsbpp_pack_batch(int32_t num_instances, const int32_t* d_weights,
                         const int64_t* d_item_off, const int32_t* d_capacities,
                         const int32_t* d_cap_off, int32_t max_items, int32_t max_types,
                         int32_t max_capacity, int32_t heuristic, const vsbpp_options* opt,
                         const int32_t* d_order, const uint64_t* d_seeds,
                         int32_t* d_assignment, int32_t* d_bin_types, int32_t* d_nbins,
                         int64_t* d_cost, void* hip_stream) {
  const vsbpp_options o = resolve(opt);
  if (num_instances < 0) return VSBPP_E_SIZE;
  if (num_instances == 0) return VSBPP_OK;
  if (!d_weights || !d_item_off || !d_capacities || !d_cap_off || !d_assignment ||
      !d_bin_types || !d_nbins || !d_cost)
    return VSBPP_E_NULL;
  if (max_items < 1 || max_types < 1 || max_types > vsbpp::kMaxTypes || max_capacity < 1)
    return VSBPP_E_SIZE;
  if (heuristic < VSBPP_FF || heuristic > VSBPP_H2) return VSBPP_E_HEURISTIC;
  int32_t rc = check_options(o);
  if (rc == VSBPP_OK) rc = check_heuristic_options(o, heuristic);
  if (rc != VSBPP_OK) return rc;
  if (o.criterion_rule == 1 || o.choice_rule == 2) return VSBPP_E_MODEL;  // this call takes no model
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!device_ok_locked()) return VSBPP_E_DEVICE;
  }
  BatchArgs a{};
  a.w = d_weights;
  a.item_off = d_item_off;
  a.caps = d_capacities;
  a.cap_off = d_cap_off;
  a.order = d_order;
  a.seeds = d_seeds;
  a.seed = o.seed;
  a.assign = d_assignment;
  a.types = d_bin_types;
  a.nbins = d_nbins;
  a.cost = d_cost;
  a.num = num_instances;
  a.max_items = max_items;
  a.max_cap = max_capacity;
  a.max_types = max_types;
  a.type_rule = o.type_rule;
  a.force_crit = o.force_criterion;
  a.active_limit = o.active_limit;
  a.downsize = o.downsize;
  a.rule2_order = o.rule2_order;
  a.s1 = o.h1_items_per_sublist;
  a.s2 = o.h2_subset_size;
  return launch_batch(a, heuristic, (hipStream_t)hip_stream);
}

int32_t vsbpp_best_of(const int64_t* d_cost, int32_t num, int64_t* d_out, void* hip_stream) {
  if (!d_cost || !d_out) return VSBPP_E_NULL;
  if (num < 1) return VSBPP_E_SIZE;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!device_ok_locked()) return VSBPP_E_DEVICE;
  }
  if (vsbpp::launch_best_of(d_cost, num, d_out, (hipStream_t)hip_stream) != hipSuccess)
    return VSBPP_E_DEVICE;
  return VSBPP_OK;
}

int32_t vsbpp_exact_batch(const vsbpp_batch* b, void* hip_stream) {
  if (!b) return VSBPP_E_NULL;
  if (b->num_instances < 0) return VSBPP_E_SIZE;
  if (b->num_instances == 0) return VSBPP_OK;
  if (!b->weights || !b->item_off || !b->capacities || !b->cap_off || !b->assignment ||
      !b->bin_types || !b->nbins || !b->cost)
    return VSBPP_E_NULL;
  if (b->max_items < 1 || b->max_items > vsbpp::kExactMaxItems || b->max_types < 1 ||
      b->max_types > vsbpp::kMaxTypes || b->max_capacity < 1)
    return VSBPP_E_SIZE;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!device_ok_locked()) return VSBPP_E_DEVICE;
  }
  BatchArgs a{};
  a.w = b->weights;
  a.item_off = b->item_off;
  a.caps = b->capacities;
  a.cap_off = b->cap_off;
  a.assign = b->assignment;
  a.types = b->bin_types;
  a.nbins = b->nbins;
  a.cost = b->cost;
  a.num = b->num_instances;
  a.max_items = b->max_items;
  a.max_cap = b->max_capacity;
  a.max_types = b->max_types;
  constexpr int kBlock = 512;
  const int grid = vsbpp::exact_blocks_per_cu(a, kBlock) * vsbpp::device_info().cus;
  const hipError_t e = vsbpp::launch_exact(a, kBlock, grid, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    vsbpp::set_last_error("vsbpp_exact_batch", e);
    return VSBPP_E_DEVICE;
  }
  return VSBPP_OK;
}

}  // extern "C"

namespace vsbpp {
int32_t check_options_public(const vsbpp_options& o) { return check_options(o); }
int32_t check_heuristic_options_public(const vsbpp_options& o, int32_t heuristic) {
  return check_heuristic_options(o, heuristic);
}
vsbpp_options resolve_options(const vsbpp_options* opt) { return resolve(opt); }
}  // namespace vsbpp
