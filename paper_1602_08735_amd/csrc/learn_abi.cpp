// C-ABI entry points of the learned bin-type scorer: the plain batch with
// decision hooks and the scorer, rollout labels, and the trainer.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "../../include/vsbpp.h"
#include "host_internal.h"
#include "kernels.h"
#include "learn.h"

namespace vsbpp {
int32_t check_options_public(const vsbpp_options& o);
int32_t check_heuristic_options_public(const vsbpp_options& o, int32_t heuristic);
vsbpp_options resolve_options(const vsbpp_options* opt);
}  // namespace vsbpp

struct vsbpp_trainer {
  int nout = 0, np = 0, waves = 256, step = 0;
  float* master = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* grad = nullptr;
  float* partial = nullptr;
  float* loss_part = nullptr;
  vsbpp_model* d_model = nullptr;
};

namespace {

float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, sizeof f);
  return f;
}

// flat fp32 parameters (w1 b1 w2 b2 w3 b3) of a model
std::vector<float> flatten(const vsbpp_model& m) {
  std::vector<float> v;
  v.reserve((size_t)vsbpp::param_count(m.n_out));
  for (int i = 0; i < 64 * 16; ++i) v.push_back(bf16_value(m.w1[i]));
  for (int i = 0; i < 64; ++i) v.push_back(m.b1[i]);
  for (int i = 0; i < 64 * 64; ++i) v.push_back(bf16_value(m.w2[i]));
  for (int i = 0; i < 64; ++i) v.push_back(m.b2[i]);
  for (int i = 0; i < 64 * m.n_out; ++i) v.push_back(bf16_value(m.w3[i]));
  for (int i = 0; i < m.n_out; ++i) v.push_back(m.b3[i]);
  return v;
}

int32_t fail() {
  (void)hipGetLastError();
  return VSBPP_E_DEVICE;
}

// A trainer checkpoint: this header, the current bf16 model (vsbpp_model as
// laid out in memory), then the fp32 master weights and Adam's first and
// second moments, np floats each.
constexpr char kTrainerMagic[8] = {'V', 'S', 'B', 'P', 'T', 'R', 'N', '1'};
struct TrainerStateHeader {
  char magic[8];
  int32_t n_out;
  int32_t np;
  int32_t step;
  int32_t reserved;
};

}  // namespace

extern "C" {

int32_t vsbpp_pack_batch_ex(const vsbpp_batch* b, int32_t heuristic, const vsbpp_options* opt,
                            const vsbpp_model* d_model, const vsbpp_decisions* dec,
                            void* hip_stream) {
  if (!b) return VSBPP_E_NULL;
  if (b->num_instances < 0) return VSBPP_E_SIZE;
  if (b->num_instances == 0) return VSBPP_OK;
  const bool has_src = dec && dec->src;
  if (!b->weights || !b->item_off || !b->capacities || !b->cap_off || !b->nbins || !b->cost)
    return VSBPP_E_NULL;
  if (!has_src && (!b->assignment || !b->bin_types)) return VSBPP_E_NULL;
  if (b->max_items < 1 || b->max_types < 1 || b->max_types > vsbpp::kMaxTypes ||
      b->max_capacity < 1)
    return VSBPP_E_SIZE;
  if (heuristic < VSBPP_FF || heuristic > VSBPP_H2) return VSBPP_E_HEURISTIC;
  vsbpp_options o = vsbpp::resolve_options(opt);
  const bool learned = o.type_rule == VSBPP_TYPE_LEARNED;
  if (learned) o.type_rule = VSBPP_TYPE_SMALLEST_FIT;  // for the shared checks below
  {
    int32_t rc = vsbpp::check_options_public(o);
    if (rc == VSBPP_OK) rc = vsbpp::check_heuristic_options_public(o, heuristic);
    if (rc != VSBPP_OK) return rc;
  }
  if (learned) o.type_rule = VSBPP_TYPE_LEARNED;
  const bool hooks = dec && (dec->src || dec->force || dec->features || dec->info || dec->count);
  if (heuristic == VSBPP_H1) {
    // the first heuristic takes the learned criterion and the feature dump
    // of its contested placements; nothing else here
    if (learned || (dec && (dec->src || dec->force || dec->count))) return VSBPP_E_OPTION;
  } else if ((learned || hooks) && heuristic > VSBPP_WF) {
    return VSBPP_E_OPTION;
  }
  if ((learned || o.criterion_rule == 1 || o.choice_rule == 2) && !d_model)
    return VSBPP_E_MODEL;
  if (!vsbpp::device_info().ok) return VSBPP_E_DEVICE;
  vsbpp::BatchArgs a{};
  a.w = b->weights;
  a.item_off = b->item_off;
  a.caps = b->capacities;
  a.cap_off = b->cap_off;
  a.order = b->order;
  a.seeds = b->seeds;
  a.seed = o.seed;
  a.assign = b->assignment;
  a.types = b->bin_types;
  a.nbins = b->nbins;
  a.cost = b->cost;
  a.num = b->num_instances;
  a.max_items = b->max_items;
  a.max_cap = b->max_capacity;
  a.max_types = b->max_types;
  a.type_rule = o.type_rule;
  a.force_crit = o.force_criterion;
  a.active_limit = o.active_limit;
  a.downsize = o.downsize;
  a.criterion_rule = o.criterion_rule;
  a.choice_rule = o.choice_rule;
  a.rule2_order = o.rule2_order;
  a.s1 = o.h1_items_per_sublist;
  a.s2 = o.h2_subset_size;
  if (dec) {
    a.src = dec->src;
    a.force = dec->force;
    a.feat_out = dec->features;
    a.info_out = dec->info;
    a.count_out = dec->count;
  }
  a.model = (o.type_rule == VSBPP_TYPE_LEARNED || o.criterion_rule == 1 || o.choice_rule == 2)
                ? d_model
                : nullptr;
  return vsbpp::enqueue_batch(a, heuristic, vsbpp::default_cfg(heuristic, a), nullptr, nullptr,
                              (hipStream_t)hip_stream);
}

int32_t vsbpp_rollout_labels(const int64_t* d_cost, const int32_t* d_info, int32_t num,
                             int32_t n_types, int32_t* d_labels, int64_t* d_values,
                             void* hip_stream) {
  if (!d_cost || !d_info || !d_labels) return VSBPP_E_NULL;
  if (num < 0 || n_types < 1 || n_types > vsbpp::kMaxTypes) return VSBPP_E_SIZE;
  if (num == 0) return VSBPP_OK;
  if (!vsbpp::device_info().ok) return VSBPP_E_DEVICE;
  if (vsbpp::launch_labels(d_cost, d_info, num, n_types, d_labels, d_values,
                           (hipStream_t)hip_stream) != hipSuccess)
    return fail();
  return VSBPP_OK;
}

int32_t vsbpp_lower_bounds(int32_t num, const int32_t* d_weights, const int64_t* d_item_off,
                           const int32_t* d_capacities, const int32_t* d_cap_off, int64_t* d_out,
                           void* hip_stream) {
  if (num < 0) return VSBPP_E_SIZE;
  if (num == 0) return VSBPP_OK;
  if (!d_weights || !d_item_off || !d_capacities || !d_cap_off || !d_out) return VSBPP_E_NULL;
  if (!vsbpp::device_info().ok) return VSBPP_E_DEVICE;
  if (vsbpp::launch_bounds(num, d_weights, d_item_off, d_capacities, d_cap_off, d_out,
                           (hipStream_t)hip_stream) != hipSuccess)
    return fail();
  return VSBPP_OK;
}

void vsbpp_trainer_destroy(vsbpp_trainer* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  for (float* p : {t->master, t->m1, t->m2, t->grad, t->partial, t->loss_part})
    if (p) (void)hipFree(p);
  if (t->d_model) (void)hipFree(t->d_model);
  delete t;
}

int32_t vsbpp_trainer_create(const vsbpp_model* init, vsbpp_trainer** out) {
  if (!out) return VSBPP_E_NULL;
  *out = nullptr;
  if (!init) return VSBPP_E_NULL;
  if (init->n_out < 1 || init->n_out > VSBPP_MAX_OUT) return VSBPP_E_SIZE;
  if (!vsbpp::device_info().ok) return VSBPP_E_DEVICE;
  vsbpp_trainer* t = new vsbpp_trainer;
  t->nout = init->n_out;
  t->np = vsbpp::param_count(t->nout);
  const size_t pb = sizeof(float) * (size_t)t->np;
  bool ok = hipMalloc(&t->master, pb) == hipSuccess && hipMalloc(&t->m1, pb) == hipSuccess &&
            hipMalloc(&t->m2, pb) == hipSuccess && hipMalloc(&t->grad, pb) == hipSuccess &&
            hipMalloc(&t->partial, pb * (size_t)t->waves) == hipSuccess &&
            hipMalloc(&t->loss_part, sizeof(float) * (size_t)t->waves) == hipSuccess &&
            hipMalloc(&t->d_model, sizeof(vsbpp_model)) == hipSuccess;
  if (!ok) {
    vsbpp_trainer_destroy(t);
    return VSBPP_E_NOMEM;
  }
  const std::vector<float> flat = flatten(*init);
  ok = hipMemcpy(t->master, flat.data(), pb, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(t->m1, 0, pb) == hipSuccess && hipMemset(t->m2, 0, pb) == hipSuccess &&
       hipMemcpy(t->d_model, init, sizeof(vsbpp_model), hipMemcpyHostToDevice) == hipSuccess &&
       hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    vsbpp_trainer_destroy(t);
    return fail();
  }
  *out = t;
  return VSBPP_OK;
}

int32_t vsbpp_trainer_step(vsbpp_trainer* t, const float* d_x, const int32_t* d_mask,
                           const int32_t* d_label, const int32_t* d_idx, int32_t batch, float lr,
                           float beta1, float beta2, float eps, float* out_loss,
                           void* hip_stream) {
  if (!t || !d_x || !d_mask || !d_label || !d_idx) return VSBPP_E_NULL;
  if (batch < 1) return VSBPP_E_SIZE;
  hipStream_t s = (hipStream_t)hip_stream;
  if (vsbpp::launch_train(t->d_model, d_x, d_mask, d_label, d_idx, batch, t->waves, t->nout,
                          t->partial, t->loss_part, t->grad, s) != hipSuccess)
    return fail();
  t->step += 1;
  if (vsbpp::launch_adam(t->master, t->m1, t->m2, t->grad, t->np, lr, beta1, beta2, eps, t->step,
                         t->d_model, s) != hipSuccess)
    return fail();
  if (out_loss) {
    std::vector<float> lp((size_t)t->waves);
    if (hipMemcpyAsync(lp.data(), t->loss_part, sizeof(float) * lp.size(),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail();
    double sum = 0.0;
    for (float v : lp) sum += v;
    *out_loss = (float)(sum / batch);
  }
  return VSBPP_OK;
}

int32_t vsbpp_trainer_gradient(vsbpp_trainer* t, const float* d_x, const int32_t* d_mask,
                               const int32_t* d_label, const int32_t* d_idx, int32_t batch,
                               float* out, int32_t out_cap) {
  if (!t || !d_x || !d_mask || !d_label || !d_idx || !out) return VSBPP_E_NULL;
  if (batch < 1 || out_cap < t->np) return VSBPP_E_SIZE;
  if (vsbpp::launch_train(t->d_model, d_x, d_mask, d_label, d_idx, batch, t->waves, t->nout,
                          t->partial, t->loss_part, t->grad, nullptr) != hipSuccess)
    return fail();
  if (hipMemcpy(out, t->grad, sizeof(float) * (size_t)t->np, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return fail();
  return t->np;
}

const vsbpp_model* vsbpp_trainer_device_model(const vsbpp_trainer* t) {
  return t ? t->d_model : nullptr;
}

int32_t vsbpp_trainer_export(const vsbpp_trainer* t, vsbpp_model* out) {
  if (!t || !out) return VSBPP_E_NULL;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(out, t->d_model, sizeof(vsbpp_model), hipMemcpyDeviceToHost) != hipSuccess)
    return fail();
  return VSBPP_OK;
}

int64_t vsbpp_trainer_state_bytes(const vsbpp_trainer* t) {
  if (!t) return VSBPP_E_NULL;
  return (int64_t)(sizeof(TrainerStateHeader) + sizeof(vsbpp_model) +
                   3 * sizeof(float) * (size_t)t->np);
}

int32_t vsbpp_trainer_save(const vsbpp_trainer* t, void* buf, int64_t cap) {
  if (!t || !buf) return VSBPP_E_NULL;
  const int64_t need = vsbpp_trainer_state_bytes(t);
  if (cap < need) return VSBPP_E_SIZE;
  unsigned char* p = static_cast<unsigned char*>(buf);
  TrainerStateHeader h{};
  std::memcpy(h.magic, kTrainerMagic, sizeof h.magic);
  h.n_out = t->nout;
  h.np = t->np;
  h.step = t->step;
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  const size_t pb = sizeof(float) * (size_t)t->np;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(p, t->d_model, sizeof(vsbpp_model), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(p + sizeof(vsbpp_model), t->master, pb, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(p + sizeof(vsbpp_model) + pb, t->m1, pb, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(p + sizeof(vsbpp_model) + 2 * pb, t->m2, pb, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return fail();
  return VSBPP_OK;
}

int32_t vsbpp_trainer_restore(vsbpp_trainer* t, const void* buf, int64_t size) {
  if (!t || !buf) return VSBPP_E_NULL;
  if (size < (int64_t)sizeof(TrainerStateHeader)) return VSBPP_E_SIZE;
  const unsigned char* p = static_cast<const unsigned char*>(buf);
  TrainerStateHeader h;
  std::memcpy(&h, p, sizeof h);
  if (std::memcmp(h.magic, kTrainerMagic, sizeof h.magic) != 0) return VSBPP_E_MODEL;
  if (h.n_out != t->nout || h.np != t->np || h.step < 0) return VSBPP_E_SIZE;
  if (size != vsbpp_trainer_state_bytes(t)) return VSBPP_E_SIZE;
  p += sizeof h;
  vsbpp_model m;
  std::memcpy(&m, p, sizeof m);
  if (m.n_out != t->nout) return VSBPP_E_MODEL;
  const size_t pb = sizeof(float) * (size_t)t->np;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(t->d_model, p, sizeof(vsbpp_model), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->master, p + sizeof(vsbpp_model), pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->m1, p + sizeof(vsbpp_model) + pb, pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->m2, p + sizeof(vsbpp_model) + 2 * pb, pb, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return fail();
  t->step = h.step;
  return VSBPP_OK;
}

}  // extern "C"
