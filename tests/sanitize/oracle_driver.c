/* Drives every entry point of the CPU oracle over seeded random instances
 * (all heuristics, type rules, bounded and downsized runs, forced and traced
 * decisions, the learned rules with a random model, lookahead labels, lower
 * bounds and both exact solvers) so that an AddressSanitizer /
 * UndefinedBehaviorSanitizer build can check its memory and integer use.
 * Exits 0 when every call returns a sane code. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/vsbpp_oracle.h"

static uint64_t g_state = 12345;
static uint32_t next_u32(void) {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(g_state >> 33);
}
static int32_t uni(int32_t lo, int32_t hi) { return lo + (int32_t)(next_u32() % (uint32_t)(hi - lo + 1)); }

static void random_model(orc_model* m, int32_t n_out) {
  memset(m, 0, sizeof *m);
  m->n_out = n_out;
  for (int i = 0; i < ORC_HIDDEN * ORC_NFEAT; ++i) m->w1[i] = (uint16_t)(0x3c00 + (next_u32() & 0x3ff)) ^ (uint16_t)((next_u32() & 1) << 15);
  for (int i = 0; i < ORC_HIDDEN * ORC_HIDDEN; ++i) m->w2[i] = (uint16_t)(0x3c00 + (next_u32() & 0x3ff)) ^ (uint16_t)((next_u32() & 1) << 15);
  for (int i = 0; i < ORC_MAX_OUT * ORC_HIDDEN; ++i) m->w3[i] = (uint16_t)(0x3c00 + (next_u32() & 0x3ff)) ^ (uint16_t)((next_u32() & 1) << 15);
  for (int i = 0; i < ORC_HIDDEN; ++i) { m->b1[i] = 0.01f * (float)uni(-10, 10); m->b2[i] = 0.01f * (float)uni(-10, 10); }
  for (int i = 0; i < ORC_MAX_OUT; ++i) m->b3[i] = 0.01f * (float)uni(-10, 10);
}

int main(void) {
  int32_t bad = 0;
  orc_model model3, model2;
  random_model(&model3, 5);
  random_model(&model2, 2);
  for (int it = 0; it < 400; ++it) {
    const int32_t n = uni(1, 7);
    const int32_t m = it % 50 == 0 ? uni(1, 3) : uni(1, 300);
    int32_t caps[16];
    caps[0] = uni(n + 1, it % 7 == 0 ? 70000 : 1000);
    for (int32_t k = 1; k < n; ++k) caps[k] = caps[k - 1] - uni(1, caps[k - 1] / (n - k + 1) > 1 ? caps[k - 1] / (n - k + 1) : 1);
    int32_t nn = n;
    for (int32_t k = 1; k < n; ++k)
      if (caps[k] <= 0 || caps[k] >= caps[k - 1]) { nn = k; break; }
    int32_t* w = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* t = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    orc_decision* tr = (orc_decision*)malloc(sizeof(orc_decision) * (size_t)m);
    for (int32_t j = 0; j < m; ++j) { w[j] = uni(1, caps[0]); order[j] = m - 1 - j; }
    int64_t cost = 0;
    int32_t count = 0;
    orc_stats st;
    for (int32_t h = ORC_FF; h <= ORC_H2; ++h) {
      for (int32_t rule = 0; rule < 2; ++rule) {
        orc_opts o;
        memset(&o, 0, sizeof o);
        o.seed = (uint64_t)it * 7919u;
        o.s1 = uni(1, 16);
        o.s2 = uni(1, 6);
        o.type_rule = rule;
        o.force_crit = h >= ORC_H1 ? uni(-1, 2) : -1;
        o.order = (it & 1) ? order : NULL;
        o.force_event = uni(-1, 5);
        o.force_t1 = uni(0, nn - 1);
        o.force_t2 = uni(0, nn - 1);
        o.trace = tr;
        o.trace_cap = m;
        o.trace_count = &count;
        o.active_limit = h <= ORC_WF ? uni(0, 4) : 0;
        o.downsize = uni(0, 1);
        int32_t rc = orc_pack(w, m, caps, nn, h, &o, a, t, &cost, &st);
        if (rc < 1 || cost < 0) bad++;
        if (h <= ORC_WF) {
          o.active_limit = 0;
          o.type_rule = ORC_TYPE_LEARNED;
          o.model = &model3;
          o.downsize = 0;
          if (orc_pack(w, m, caps, nn, h, &o, a, t, &cost, NULL) < 1) bad++;
          o.type_rule = ORC_TYPE_LARGEST;
          o.downsize = 1;
          o.choice_rule = 2;
          o.model = &model2;
          if (orc_pack(w, m, caps, nn, h, &o, a, t, &cost, NULL) < 1) bad++;
        } else if (h == ORC_H1) {
          o.force_crit = -1;
          o.criterion_rule = 1;
          o.model = &model3;
          if (orc_pack(w, m, caps, nn, h, &o, a, t, &cost, NULL) < 1) bad++;
        }
      }
    }
    if (m <= 60) {
      int64_t vals[16];
      for (int32_t c = 0; c < 3; ++c) {
        if (orc_rollout_label_ex(w, m, caps, nn, c, uni(0, 3), uni(0, 1), uni(0, 1), vals) < -6) bad++;
        if (orc_choice_label(w, m, caps, nn, c, uni(0, 3), vals) < -6) bad++;
      }
    }
    if (orc_lb_cap(w, m, caps, nn) < orc_lb_sum(w, m)) bad++;
    (void)orc_lb_big(w, m, caps, nn);
    if (m <= 9 && orc_opt_partitions(w, m, caps, nn) != orc_opt_subset_dp(w, m, caps, nn)) bad++;
    /* error paths: every code, nothing written */
    int32_t bw = 0;
    if (orc_pack(&bw, 1, caps, nn, ORC_FF, NULL, a, t, &cost, NULL) != ORC_E_WEIGHT) bad++;
    if (orc_pack(w, 0, caps, nn, ORC_BF, NULL, a, t, &cost, NULL) != ORC_E_SIZE) bad++;
    if (orc_pack(w, m, caps, nn, 9, NULL, a, t, &cost, NULL) != ORC_E_HEURISTIC) bad++;
    free(w);
    free(a);
    free(t);
    free(order);
    free(tr);
  }
  printf("oracle driver: %d failures\n", bad);
  return bad ? 1 : 0;
}
