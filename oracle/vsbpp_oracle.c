/*
 * Sequential CPU oracle for the VSBPP placement heuristics (Alenezi et al.).
 *
 * TEST INFRASTRUCTURE ONLY: it checks the HIP path and shares no code with
 * it.  Every function is the plain, slow statement of what the paper (and the
 * readings listed with it) computes; there is no blocking, fusion or pruning.
 *
 * Citations name the paper's sections, rules and tables.
 */
#include "vsbpp_oracle.h"

#include <stdlib.h>
#include <math.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Counter-based generator.                                                */
/* ---------------------------------------------------------------------- */

/* SplitMix64 as published by Steele, Lea & Flood (OOPSLA 2014): the state
 * advances by the golden-gamma 0x9e3779b97f4a7c15 and each output is the
 * state passed through the 64-bit finaliser (shift-xor 30, multiply,
 * shift-xor 27, multiply, shift-xor 31).  Output k uses state seed+(k+1)*g. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

uint64_t orc_stream_key(uint64_t seed, uint64_t stream) {
  return orc_splitmix64(seed, stream);
}

/* Rule 3 (Section 6.3): the item leaving its sublist is tagged with FF, BF
 * or WF "with equal probabilities".  The draw maps the high 32 bits x of a
 * generator output to floor(3x / 2^32) (multiply-shift range reduction). */
int32_t orc_criterion(uint64_t stream_key, uint64_t counter) {
  uint64_t hi = orc_splitmix64(stream_key, counter) >> 32;
  return (int32_t)((hi * 3u) >> 32);
}

/* Rule 3 for the second heuristic (Section 6.4): each permutation packing
 * takes one generator output, counter I*S! + r, and its t-th placement the
 * (t+1)-th base-3 digit of h/2^32, h = the output's high 32 bits:
 * floor(3^(t+1) * h / 2^32) mod 3.  For t < 6, 3^(t+1) * h < 2^64.  Every
 * tuple of the first k <= 6 digits has probability 3^-k up to 3^k/2^32. */
int32_t orc_criterion_digit(uint64_t stream_key, uint64_t counter, int32_t t) {
  uint64_t h = orc_splitmix64(stream_key, counter) >> 32;
  uint64_t p = 3;
  for (int32_t i = 0; i < t; ++i) p *= 3;
  return (int32_t)(((p * h) >> 32) % 3u);
}

/* purposes of the generator streams */
#define STREAM_RULE1 1u
#define STREAM_H1 2u
#define STREAM_H2 3u

/* Rule 1 (Section 6.2/6.3 step 1) distributes the items "randomly" into the
 * sublists.  Reading: a keyed pseudo-random permutation pi of [0,m) assigns
 * item pi(q) to position q, and sublists are consecutive runs of positions.
 * pi is a 4-round balanced Feistel network over 2h bits (2^(2h) >= m) whose
 * round function is the generator, restricted to [0,m) by cycle walking
 * (Black & Rogaway, "Ciphers with arbitrary finite domains", CT-RSA 2002). */
static uint32_t feistel(uint64_t key, uint32_t h, uint32_t x) {
  uint32_t mask = (1u << h) - 1u;
  uint32_t left = x >> h, right = x & mask;
  for (uint32_t r = 0; r < 4; ++r) {
    uint32_t f = (uint32_t)(orc_splitmix64(key, ((uint64_t)r << 32) | right)) & mask;
    uint32_t nl = right;
    right = left ^ f;
    left = nl;
  }
  return (left << h) | right;
}

int32_t orc_perm(uint64_t seed, int32_t m, int32_t q) {
  if (m <= 1) return 0;
  uint32_t bits = 0;
  while ((1ull << bits) < (uint64_t)m) ++bits;
  uint32_t h = (bits + 1) / 2;
  uint64_t key = orc_stream_key(seed, STREAM_RULE1);
  uint32_t y = feistel(key, h, (uint32_t)q);
  while (y >= (uint32_t)m) y = feistel(key, h, y);
  return (int32_t)y;
}

/* ---------------------------------------------------------------------- */
/* Packer: an ordered list of bins (creation order = bin index).           */
/* ---------------------------------------------------------------------- */

typedef struct {
  int32_t type;
  int64_t load;
  int32_t divided;
  int32_t closed;  /* bounded plain runs: the bin takes no more items */
} obin;

typedef struct {
  obin* b;
  int32_t nb, capn;
} opacker;

static void pk_init(opacker* p) { p->b = NULL; p->nb = 0; p->capn = 0; }
static void pk_free(opacker* p) { free(p->b); pk_init(p); }
static void pk_push(opacker* p, int32_t type) {
  if (p->nb == p->capn) {
    p->capn = p->capn ? 2 * p->capn : 16;
    p->b = (obin*)realloc(p->b, sizeof(obin) * (size_t)p->capn);
  }
  p->b[p->nb].type = type;
  p->b[p->nb].load = 0;
  p->b[p->nb].divided = 0;
  p->b[p->nb].closed = 0;
  p->nb++;
}

/* Rule 2 (Section 6.3): a packer starts with one empty bin of every type.
 * The paper gives no order for them; it matters to First Fit (lowest index)
 * and to ties.  order 0 creates them in type order (B_1 first), order 1 in
 * increasing capacity (B_n first). */
static void rule2_bins(opacker* p, int32_t n, int32_t order) {
  for (int32_t ty = 0; ty < n; ++ty) pk_push(p, order ? n - 1 - ty : ty);
}

/* Type of a bin opened when no open bin can take the item.  The paper says
 * extra rules are needed to choose among bin types (Section 1) but gives
 * none.  SMALLEST_FIT takes the smallest capacity >= w; LARGEST takes B_1. */
static int32_t open_type(const int32_t* caps, int32_t n, int32_t w, int32_t rule) {
  if (rule == ORC_TYPE_LARGEST) return 0;
  for (int32_t k = n - 1; k >= 0; --k)
    if (caps[k] >= w) return k;
  return 0; /* unreachable for valid input: w <= B_1 */
}

/* Rule 4 (Section 6.3) with the FF/BF/WF choices of Section 1.
 * Candidate set: bins whose load plus w stays within capacity.
 *   FF: the candidate with the lowest index.
 *   BF: least room left after placing; ties -> lowest index.
 *   WF: most room left after placing; ties -> lowest index.
 * No candidate: open a bin (type per open_type).
 * Bounded runs (active_limit > 0, plain heuristics only): only bins that are
 * not closed are candidates, and a bin about to open while active_limit bins
 * are open first closes the fullest open bin (least room; lowest index on
 * ties).  Section 1 says Best Fit keeps a fixed number of bins active but
 * gives no closing rule; this one is the Best-k-Fit rule of bounded-space
 * bin packing (Csirik & Johnson, Algorithmica 2001).
 * Rule 5 (when enabled): a bin whose load reaches half its capacity and that
 * has not divided yet divides once, adding an empty bin of its type.
 * `suffix_min` is the smallest weight among this item and all later items of
 * the same packer; it only feeds the work counters. */
typedef int32_t (*type_chooser)(void* ctx, int32_t w);
/* plain runs under a choice rule: given the criterion's bin, 1 opens a new
 * bin instead */
typedef int32_t (*bin_chooser)(void* ctx, const obin* b, int32_t w);

static int32_t place(opacker* p, const int32_t* caps, int32_t n, int32_t w,
                     int32_t crit, int32_t rule5, int32_t type_rule, int32_t active_limit,
                     int64_t suffix_min, orc_stats* st, type_chooser choose, void* cctx,
                     bin_chooser choose_bin) {
  int32_t best = -1;
  int64_t best_after = 0;
  for (int32_t b = 0; b < p->nb; ++b) {
    if (p->b[b].closed) continue;
    int64_t room = (int64_t)caps[p->b[b].type] - p->b[b].load;
    if (st) {
      st->bin_tests++;
      if (room >= suffix_min) st->live_tests++;
    }
    if (room < w) continue;
    int64_t after = room - w;
    if (crit == ORC_FF) {
      best = b;
      break;
    }
    if (best < 0 || (crit == ORC_BF ? after < best_after : after > best_after)) {
      best = b;
      best_after = after;
    }
  }
  if (best >= 0 && choose_bin && choose_bin(cctx, &p->b[best], w)) best = -1;
  if (best < 0) {
    if (active_limit > 0) {
      int32_t open = 0, fullest = -1;
      int64_t least = 0;
      for (int32_t b = 0; b < p->nb; ++b) {
        if (p->b[b].closed) continue;
        ++open;
        const int64_t room = (int64_t)caps[p->b[b].type] - p->b[b].load;
        if (fullest < 0 || room < least) {
          fullest = b;
          least = room;
        }
      }
      if (open >= active_limit) p->b[fullest].closed = 1;
    }
    pk_push(p, choose ? choose(cctx, w) : open_type(caps, n, w, type_rule));
    best = p->nb - 1;
    if (st) st->new_bins++;
  }
  obin* bb = &p->b[best];
  bb->load += w;
  if (rule5 && !bb->divided && 2 * bb->load >= (int64_t)caps[bb->type]) {
    int32_t t = bb->type;
    bb->divided = 1;
    pk_push(p, t); /* may move p->b */
    if (st) st->divisions++;
  }
  if (st) st->placements++;
  return best;
}

/* Canonical output of one packer: bins with load > 0 keep creation order and
 * get consecutive ids starting at `base`; empty bins (Rule 2 / Rule 5 bins
 * that never received an item) are not used and cost nothing. */
static int32_t emit_packer(const opacker* p, const int32_t* caps, const int32_t* items,
                           const int32_t* local, int32_t k, int32_t base,
                           int32_t* assign, int32_t* types, int64_t* cost) {
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)(p->nb ? p->nb : 1));
  int32_t used = 0;
  for (int32_t b = 0; b < p->nb; ++b) {
    if (p->b[b].load > 0) {
      rank[b] = used;
      types[base + used] = p->b[b].type;
      *cost += caps[p->b[b].type];
      used++;
    } else {
      rank[b] = -1;
    }
  }
  for (int32_t t = 0; t < k; ++t) assign[items[t]] = base + rank[local[t]];
  free(rank);
  return used;
}

static int64_t packer_cost(const opacker* p, const int32_t* caps) {
  int64_t c = 0;
  for (int32_t b = 0; b < p->nb; ++b)
    if (p->b[b].load > 0) c += caps[p->b[b].type];
  return c;
}

/* ---------------------------------------------------------------------- */
/* Validation.                                                             */
/* ---------------------------------------------------------------------- */

static int32_t validate(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                        int32_t heuristic, const orc_opts* o) {
  if (!w || !caps) return ORC_E_NULL;
  if (m < 1 || n < 1 || n > 16) return ORC_E_SIZE;
  for (int32_t k = 0; k < n; ++k) {
    if (caps[k] <= 0) return ORC_E_CAPS;
    if (k > 0 && caps[k] >= caps[k - 1]) return ORC_E_CAPS;
  }
  for (int32_t j = 0; j < m; ++j)
    if (w[j] < 1 || w[j] > caps[0]) return ORC_E_WEIGHT;
  if (heuristic < ORC_FF || heuristic > ORC_H2) return ORC_E_HEURISTIC;
  if (o) {
    if (o->s1 < 1 || o->s2 < 1 || o->s2 > 6) return ORC_E_OPTION;
    if (o->type_rule != ORC_TYPE_SMALLEST_FIT && o->type_rule != ORC_TYPE_LARGEST &&
        o->type_rule != ORC_TYPE_LEARNED)
      return ORC_E_OPTION;
    if (o->type_rule == ORC_TYPE_LEARNED &&
        (!o->model || o->model->n_out < 1 || o->model->n_out > ORC_MAX_OUT ||
         heuristic > ORC_WF))
      return ORC_E_OPTION;
    if (o->force_crit < -1 || o->force_crit > ORC_WF) return ORC_E_OPTION;
    if (o->active_limit < 0 || (o->active_limit > 0 && heuristic > ORC_WF)) return ORC_E_OPTION;
    if (o->downsize != 0 && o->downsize != 1) return ORC_E_OPTION;
    if (o->criterion_rule != 0 && o->criterion_rule != 1) return ORC_E_OPTION;
    if (o->choice_rule < 0 || o->choice_rule > 2) return ORC_E_OPTION;
    if (o->rule2_order < 0 || o->rule2_order > 1 || (o->rule2_order == 1 && heuristic <= ORC_WF))
      return ORC_E_OPTION;
    if (o->choice_rule > 0 &&
        (heuristic > ORC_WF || o->type_rule != ORC_TYPE_LARGEST || o->downsize != 1 ||
         o->active_limit != 0))
      return ORC_E_OPTION;
    if (o->choice_rule == 2 &&
        (!o->model || o->model->n_out < 2 || o->model->n_out > ORC_MAX_OUT))
      return ORC_E_OPTION;
    if (o->criterion_rule == 1 &&
        (heuristic != ORC_H1 || o->force_crit != -1 || !o->model || o->model->n_out < 3 ||
         o->model->n_out > ORC_MAX_OUT))
      return ORC_E_OPTION;
    if (o->order) {
      /* must be a permutation of [0,m) */
      char* seen = (char*)calloc((size_t)m, 1);
      for (int32_t q = 0; q < m; ++q) {
        int32_t j = o->order[q];
        if (j < 0 || j >= m || seen[j]) { free(seen); return ORC_E_OPTION; }
        seen[j] = 1;
      }
      free(seen);
    }
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Heuristics.                                                             */
/* ---------------------------------------------------------------------- */

static int32_t item_at(const orc_opts* o, int32_t m, int32_t q, int32_t heuristic) {
  if (o->order) return o->order[q];
  if (heuristic == ORC_H1 || heuristic == ORC_H2) return orc_perm(o->seed, m, q);
  return q; /* plain heuristics: input order */
}

/* ---------------------------------------------------------------------- */
/* Learned bin-type scorer (decision = an item that fits no open bin).     */
/* ---------------------------------------------------------------------- */

static float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, sizeof f);
  return f;
}

static float relu(float v) { return v > 0.0f ? v : 0.0f; }

/* Every unit -- hidden or output -- is its bias followed by a chain of fused
 * multiply-adds over its inputs in index order (fp32); hidden units then
 * take ReLU.  This fixes the rounding of each score, so the scores, and the
 * integer decisions they drive, are reproducible bit for bit. */
void orc_mlp_forward(const orc_model* mdl, const float* x, float* z) {
  float h1[ORC_HIDDEN], h2[ORC_HIDDEN];
  for (int l = 0; l < ORC_HIDDEN; ++l) {
    float acc = mdl->b1[l];
    for (int i = 0; i < ORC_NFEAT; ++i) acc = fmaf(bf16_to_f32(mdl->w1[l * ORC_NFEAT + i]), x[i], acc);
    h1[l] = relu(acc);
  }
  for (int l = 0; l < ORC_HIDDEN; ++l) {
    float acc = mdl->b2[l];
    for (int j = 0; j < ORC_HIDDEN; ++j) acc = fmaf(bf16_to_f32(mdl->w2[l * ORC_HIDDEN + j]), h1[j], acc);
    h2[l] = relu(acc);
  }
  for (int k = 0; k < mdl->n_out; ++k) {
    float acc = mdl->b3[k];
    for (int j = 0; j < ORC_HIDDEN; ++j) acc = fmaf(bf16_to_f32(mdl->w3[k * ORC_HIDDEN + j]), h2[j], acc);
    z[k] = acc;
  }
}

/* state of a plain run that the decision features read */
typedef struct {
  const int32_t* caps;
  int32_t n, m, q, w;
  int64_t total, placed;     /* weight of all items; of positions < q        */
  int64_t smin_after;        /* smallest weight at positions > q, or -1      */
  int32_t nb;                /* bins opened so far                           */
  int32_t hist[6];           /* bins by room bucket                          */
  int32_t event;             /* decisions so far                             */
  const orc_opts* o;
} plain_ctx;

/* room bucket of the histogram: floor(6 r / (B_1 + 1)) in 0..5 */
static int32_t room_bucket(int64_t r, int32_t b1) {
  int64_t k = (6 * r) / ((int64_t)b1 + 1);
  return (int32_t)(k > 5 ? 5 : k);
}

/* The 16 decision features (fp32; "* (1/a)" multiplies by the fp32
 * reciprocal 1.0f/a):
 *  0  w * (1/B_1)
 *  1  (items after this one) * (1/m)
 *  2  ((weight of the items after this one) / (their count)) * (1/B_1), 0 if none
 *  3  (smallest weight after this one) * (1/B_1), 1 if none
 *  4  (bins opened so far) * (1/m)
 *  5..10  (bins so far in room bucket floor(6r/(B_1+1))) * (1/max(bins, 1))
 *  11..14 B_2..B_5 * (1/B_1) (0 beyond n)
 *  15 w * (1/(smallest capacity >= w)) */
static void decision_features(const plain_ctx* c, float* x) {
  const float inv_b1 = 1.0f / (float)c->caps[0];
  const float inv_m = 1.0f / (float)c->m;
  const int32_t rem = c->m - c->q - 1;
  const int64_t rsum = c->total - c->placed - c->w;
  x[0] = (float)c->w * inv_b1;
  x[1] = (float)rem * inv_m;
  x[2] = rem > 0 ? ((float)rsum / (float)rem) * inv_b1 : 0.0f;
  x[3] = rem > 0 ? (float)c->smin_after * inv_b1 : 1.0f;
  x[4] = (float)c->nb * inv_m;
  const float inv_den = 1.0f / (float)(c->nb > 0 ? c->nb : 1);
  for (int k = 0; k < 6; ++k) x[5 + k] = (float)c->hist[k] * inv_den;
  for (int k = 1; k <= 4; ++k) x[10 + k] = k < c->n ? (float)c->caps[k] * inv_b1 : 0.0f;
  x[15] = (float)c->w *
          (1.0f / (float)c->caps[open_type(c->caps, c->n, c->w, ORC_TYPE_SMALLEST_FIT)]);
}

static int32_t plain_choose(void* vc, int32_t w) {
  plain_ctx* c = (plain_ctx*)vc;
  const orc_opts* o = c->o;
  const int32_t base_rule = o->type_rule == ORC_TYPE_LEARNED ? ORC_TYPE_SMALLEST_FIT : o->type_rule;
  const int32_t base = open_type(c->caps, c->n, w, base_rule);
  const int32_t d = c->event++;
  uint32_t feasible = 0;
  for (int32_t k = 0; k < c->n; ++k)
    if (c->caps[k] >= w) feasible |= 1u << k;
  int32_t chosen = base;
  float x[ORC_NFEAT];
  const int need_feat = (o->type_rule == ORC_TYPE_LEARNED) || (o->trace && d < o->trace_cap);
  if (need_feat) decision_features(c, x);
  if (o->type_rule == ORC_TYPE_LEARNED) {
    float z[ORC_MAX_OUT];
    orc_mlp_forward(o->model, x, z);
    const int32_t kmax = c->n < o->model->n_out ? c->n : o->model->n_out;
    int32_t best = 0; /* type 0 always holds the item */
    int finite = 1;
    for (int32_t k = 0; k < kmax; ++k) finite &= isfinite(z[k]) ? 1 : 0;
    for (int32_t k = 1; k < kmax; ++k)
      if ((feasible >> k) & 1u)
        if (z[k] > z[best]) best = k;
    /* the scorer only proposes: a non-finite output falls back to the base rule */
    chosen = finite ? best : base;
  }
  if (o->force_event >= 0) {
    int32_t t = -1;
    if (d == o->force_event) t = o->force_t1;
    else if (d == o->force_event + 1) t = o->force_t2;
    if (t >= 0 && t < c->n && ((feasible >> t) & 1u)) chosen = t;
  }
  if (o->trace && d < o->trace_cap) {
    orc_decision* r = &o->trace[d];
    r->position = c->q;
    r->weight = w;
    r->plain_type = base;
    r->chosen = chosen;
    r->feasible = feasible;
    memcpy(r->feat, x, sizeof x);
  }
  return chosen;
}

/* Learned bin choice (plain FF/BF/WF under the largest type rule with
 * downsizing).  Section 1 leaves open how bins and their types are chosen
 * beyond the three rules; with downsizing a bin of load L costs c(L), the
 * smallest capacity >= L, whatever type it was opened with.  A placement of
 * w into the criterion's bin (load L) is contested when c(L + w) > c(L):
 * the bin becomes costlier.  At a contested placement the alternative is a
 * new bin (of type B_1, the largest type rule's).  The scores decide: output
 * 1 (new bin) must be strictly larger than output 0 (the criterion's bin)
 * and both finite; elsewhere, and on ties, the criterion's bin is kept. */
static int64_t holding_cap(const int32_t* caps, int32_t n, int64_t load) {
  int64_t c = caps[0];
  for (int32_t k = 0; k < n; ++k)
    if (caps[k] >= load) c = caps[k];
  return c;
}

/* The 16 features of a contested placement (fp32; "* (1/a)" multiplies by
 * the fp32 reciprocal 1.0f/a): 0..10 as for a type decision (item, the items
 * after it, bins so far and their room histogram), then, for the criterion's
 * bin b with load L and capacity C:
 *  11 (C - L - w) * (1/B_1)          room left in b after the item
 *  12 (c(L + w) - c(L)) * (1/B_1)    what placing the item in b adds
 *  13 c(w) * (1/B_1)                 the cost of a new bin holding the item
 *  14 (c(L + w) - L - w) * (1/B_1)   b's slack after the item
 *  15 (c(L) - L) * (1/B_1)           b's slack before it */
static void choice_features(const plain_ctx* c, const obin* b, float* x) {
  decision_features(c, x);
  const float inv_b1 = 1.0f / (float)c->caps[0];
  const int64_t L = b->load, w = c->w;
  const int64_t before = holding_cap(c->caps, c->n, L);
  const int64_t after = holding_cap(c->caps, c->n, L + w);
  x[11] = (float)((int64_t)c->caps[b->type] - L - w) * inv_b1;
  x[12] = (float)(after - before) * inv_b1;
  x[13] = (float)holding_cap(c->caps, c->n, w) * inv_b1;
  x[14] = (float)(after - L - w) * inv_b1;
  x[15] = (float)(before - L) * inv_b1;
}

static int32_t plain_choice(void* vc, const obin* b, int32_t w) {
  plain_ctx* c = (plain_ctx*)vc;
  const orc_opts* o = c->o;
  if (holding_cap(c->caps, c->n, b->load + w) == holding_cap(c->caps, c->n, b->load))
    return 0; /* not contested */
  const int32_t d = c->event++;
  int32_t open = 0;
  float x[ORC_NFEAT];
  const int need_feat = o->choice_rule == 2 || (o->trace && d < o->trace_cap);
  if (need_feat) choice_features(c, b, x);
  if (o->choice_rule == 2) {
    float z[ORC_MAX_OUT];
    orc_mlp_forward(o->model, x, z);
    open = (isfinite(z[0]) && isfinite(z[1]) && z[1] > z[0]) ? 1 : 0;
  }
  if (o->force_event >= 0) {
    int32_t t = -1;
    if (d == o->force_event) t = o->force_t1;
    else if (d == o->force_event + 1) t = o->force_t2;
    if (t == 0 || t == 1) open = t;
  }
  if (o->trace && d < o->trace_cap) {
    orc_decision* r = &o->trace[d];
    r->position = c->q;
    r->weight = w;
    r->plain_type = 0;
    r->chosen = open;
    r->feasible = 3u;
    memcpy(r->feat, x, sizeof x);
  }
  return open;
}

/* Plain FF/BF/WF (Section 1): one packer over the whole list, starting with
 * no bins, one fixed criterion, no Rule 2 and no Rule 5.  The type of a bin
 * opened when nothing fits follows the type rule, the scorer, or a forced
 * choice at one decision and the next. */
static int32_t run_plain(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                         int32_t crit, const orc_opts* o, int32_t* assign,
                         int32_t* types, int64_t* cost, orc_stats* st) {
  int32_t* items = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t* local = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int64_t* smin = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
  for (int32_t q = 0; q < m; ++q) items[q] = item_at(o, m, q, crit);
  for (int32_t q = m - 1; q >= 0; --q) {
    int64_t v = w[items[q]];
    smin[q] = (q == m - 1 || v < smin[q + 1]) ? v : smin[q + 1];
  }
  plain_ctx c;
  memset(&c, 0, sizeof c);
  c.caps = caps;
  c.n = n;
  c.m = m;
  c.o = o;
  for (int32_t q = 0; q < m; ++q) c.total += w[items[q]];
  opacker p;
  pk_init(&p);
  for (int32_t q = 0; q < m; ++q) {
    const int32_t wq = w[items[q]];
    c.q = q;
    c.w = wq;
    c.smin_after = q + 1 < m ? smin[q + 1] : -1;
    c.nb = p.nb;
    const int32_t nb_before = p.nb;
    const int32_t b = place(&p, caps, n, wq, crit, 0, o->type_rule, o->active_limit, smin[q], st,
                            o->choice_rule ? NULL : plain_choose, &c,
                            o->choice_rule ? plain_choice : NULL);
    local[q] = b;
    const int64_t room = (int64_t)caps[p.b[b].type] - p.b[b].load;
    if (b != nb_before) c.hist[room_bucket(room + wq, caps[0])]--;
    c.hist[room_bucket(room, caps[0])]++;
    c.placed += wq;
  }
  if (o->trace_count) *o->trace_count = c.event;
  *cost = 0;
  int32_t nb = emit_packer(&p, caps, items, local, m, 0, assign, types, cost);
  if (st) st->packers += 1;
  pk_free(&p);
  free(items);
  free(local);
  free(smin);
  return nb;
}

int32_t orc_rollout_label(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                          int32_t crit, int32_t d, int64_t* values) {
  return orc_rollout_label_ex(w, m, caps, n, crit, d, ORC_TYPE_SMALLEST_FIT, 0, values);
}

int32_t orc_rollout_label_ex(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                             int32_t crit, int32_t d, int32_t type_rule, int32_t downsize,
                             int64_t* values) {
  if (!w || !caps || !values) return ORC_E_NULL;
  if (crit < ORC_FF || crit > ORC_WF || d < 0) return ORC_E_OPTION;
  if (type_rule != ORC_TYPE_SMALLEST_FIT && type_rule != ORC_TYPE_LARGEST) return ORC_E_OPTION;
  int32_t* assign = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t* types = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  orc_decision* tr = (orc_decision*)malloc(sizeof(orc_decision) * (size_t)(d + 1));
  int32_t count = 0;
  int64_t cost = 0;
  orc_opts o = {0, 10, 5, type_rule, -1, NULL, NULL, -1, 0, 0, tr, d + 1, &count, 0, downsize, 0, 0, 0};
  int32_t rc = orc_pack(w, m, caps, n, crit, &o, assign, types, &cost, NULL);
  int32_t label = -1;
  if (rc >= 0 && d < count) {
    const uint32_t feasible = tr[d].feasible;
    const int32_t base = tr[d].plain_type;
    int64_t best = -1;
    for (int32_t k1 = 0; k1 < n; ++k1) {
      values[k1] = -1;
      if (!((feasible >> k1) & 1u)) continue;
      int64_t v = -1;
      for (int32_t k2 = 0; k2 < n; ++k2) {
        orc_opts f = {0, 10, 5, type_rule, -1, NULL, NULL, d, k1, k2, NULL, 0, NULL, 0, downsize, 0, 0, 0};
        orc_pack(w, m, caps, n, crit, &f, assign, types, &cost, NULL);
        if (v < 0 || cost < v) v = cost;
      }
      values[k1] = v;
      if (best < 0 || v < best) best = v;
    }
    if (values[base] == best) label = base;
    else
      for (int32_t k1 = 0; k1 < n && label < 0; ++k1)
        if (values[k1] == best) label = k1;
  } else if (rc >= 0) {
    label = ORC_E_OPTION; /* the run has fewer than d+1 decisions */
  } else {
    label = rc;
  }
  free(assign);
  free(types);
  free(tr);
  return label;
}

int32_t orc_choice_label(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                         int32_t crit, int32_t d, int64_t* values) {
  if (!w || !caps || !values) return ORC_E_NULL;
  if (crit < ORC_FF || crit > ORC_WF || d < 0) return ORC_E_OPTION;
  int32_t* assign = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t* types = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t count = 0;
  int64_t cost = 0;
  orc_opts o = {0, 10, 5, ORC_TYPE_LARGEST, -1, NULL, NULL, -1, 0, 0, NULL, 0, &count, 0, 1, 0, 1, 0};
  int32_t rc = orc_pack(w, m, caps, n, crit, &o, assign, types, &cost, NULL);
  int32_t label;
  if (rc >= 0 && d < count) {
    for (int32_t k1 = 0; k1 < 2; ++k1) {
      int64_t v = -1;
      for (int32_t k2 = 0; k2 < 2; ++k2) {
        orc_opts f = {0, 10, 5, ORC_TYPE_LARGEST, -1, NULL, NULL, d, k1, k2, NULL, 0, NULL, 0, 1, 0, 1, 0};
        orc_pack(w, m, caps, n, crit, &f, assign, types, &cost, NULL);
        if (v < 0 || cost < v) v = cost;
      }
      values[k1] = v;
    }
    label = values[1] < values[0] ? 1 : 0;
  } else {
    label = rc >= 0 ? ORC_E_OPTION : rc;
  }
  free(assign);
  free(types);
  return label;
}

/* Learned criterion for the first heuristic (an alternative to Rule 3's
 * equal-probability draw, Section 6.3): where First, Best and Worst Fit would
 * put the item into different bins of the packer, a network scores the three
 * criteria from features of the placement and the best score wins (lowest
 * criterion on ties).  Where they agree, or nothing fits, the criterion does
 * not change the placement and the draw `drawn` stands; a non-finite score
 * also falls back to the draw.  Features (fp32; "a / b" is a times the fp32
 * reciprocal of b), the rest zero:
 *   0  w / B_1            1  t / k (position t of a sublist of k items)
 *   2  room left in First Fit's bin after the item / B_1
 *   3  the same for Best Fit's bin    4  the same for Worst Fit's bin
 *   5  bins the item fits / 16        6  bins in the packer / 32        */
static int32_t h1_learned_criterion(const opacker* p, const int32_t* caps, int32_t w,
                                    int32_t t, int32_t k, int32_t q, int32_t drawn,
                                    const orc_opts* o) {
  int32_t bff = -1, bbf = -1, bwf = -1, nfit = 0;
  int64_t abf = 0, awf = 0;
  for (int32_t b = 0; b < p->nb; ++b) {
    const int64_t room = (int64_t)caps[p->b[b].type] - p->b[b].load;
    if (room < w) continue;
    const int64_t after = room - w;
    ++nfit;
    if (bff < 0) bff = b;
    if (bbf < 0 || after < abf) { bbf = b; abf = after; }
    if (bwf < 0 || after > awf) { bwf = b; awf = after; }
  }
  if (bff < 0 || (bff == bbf && bbf == bwf)) return drawn;
  const float inv_b1 = 1.0f / (float)caps[0];
  float x[ORC_NFEAT];
  memset(x, 0, sizeof x);
  const int64_t aff = (int64_t)caps[p->b[bff].type] - p->b[bff].load - w;
  x[0] = (float)w * inv_b1;
  x[1] = (float)t * (1.0f / (float)k);
  x[2] = (float)aff * inv_b1;
  x[3] = (float)abf * inv_b1;
  x[4] = (float)awf * inv_b1;
  x[5] = (float)nfit * (1.0f / 16.0f);
  x[6] = (float)p->nb * (1.0f / 32.0f);
  float z[ORC_MAX_OUT];
  orc_mlp_forward(o->model, x, z);
  int32_t c = drawn;
  if (isfinite(z[0]) && isfinite(z[1]) && isfinite(z[2])) {
    c = 0;
    if (z[1] > z[c]) c = 1;
    if (z[2] > z[c]) c = 2;
  }
  if (o->trace && o->trace_count && *o->trace_count < o->trace_cap) {
    orc_decision* d = &o->trace[(*o->trace_count)++];
    d->position = q;
    d->weight = w;
    d->plain_type = drawn;
    d->chosen = c;
    d->feasible = 7u;
    memcpy(d->feat, x, sizeof x);
  }
  return c;
}

/* First heuristic (Section 6.3).  Sublist I holds positions
 * [I*s1, min((I+1)*s1, m)); every sublist is its own packer that starts with
 * one empty bin of each type (Rule 2), takes its items in position order
 * (Rule 3, criterion drawn per position), places them (Rule 4) and divides
 * half-full bins (Rule 5). */
static int32_t run_h1(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                      const orc_opts* o, int32_t* assign, int32_t* types,
                      int64_t* cost, orc_stats* st) {
  int32_t s1 = o->s1;
  int32_t l = (m + s1 - 1) / s1;
  uint64_t ck = orc_stream_key(o->seed, STREAM_H1);
  int32_t* items = (int32_t*)malloc(sizeof(int32_t) * (size_t)s1);
  int32_t* local = (int32_t*)malloc(sizeof(int32_t) * (size_t)s1);
  int64_t* smin = (int64_t*)malloc(sizeof(int64_t) * (size_t)s1);
  int32_t base = 0;
  *cost = 0;
  if (o->criterion_rule == 1 && o->trace_count) *o->trace_count = 0;
  for (int32_t I = 0; I < l; ++I) {
    int32_t q0 = I * s1;
    int32_t k = (m - q0 < s1) ? m - q0 : s1;
    for (int32_t t = 0; t < k; ++t) items[t] = item_at(o, m, q0 + t, ORC_H1);
    for (int32_t t = k - 1; t >= 0; --t) {
      int64_t v = w[items[t]];
      smin[t] = (t == k - 1 || v < smin[t + 1]) ? v : smin[t + 1];
    }
    opacker p;
    pk_init(&p);
    rule2_bins(&p, n, o->rule2_order);
    for (int32_t t = 0; t < k; ++t) {
      int32_t c = o->force_crit >= 0 ? o->force_crit
                                     : orc_criterion(ck, (uint64_t)(q0 + t));
      if (o->criterion_rule == 1)
        c = h1_learned_criterion(&p, caps, w[items[t]], t, k, q0 + t, c, o);
      local[t] = place(&p, caps, n, w[items[t]], c, 1, o->type_rule, 0, smin[t], st, NULL, NULL,
                       NULL);
    }
    base += emit_packer(&p, caps, items, local, k, base, assign, types, cost);
    pk_free(&p);
    if (st) st->packers += 1;
  }
  free(items);
  free(local);
  free(smin);
  return base;
}

static int64_t factorial(int32_t k) {
  int64_t f = 1;
  for (int32_t i = 2; i <= k; ++i) f *= i;
  return f;
}

/* r-th permutation of 0..k-1 in lexicographic order (factorial-base digits
 * of r select, one after another, among the values not yet used). */
static void nth_permutation(int64_t r, int32_t k, int32_t* out) {
  int32_t avail[8];
  for (int32_t i = 0; i < k; ++i) avail[i] = i;
  int32_t left = k;
  for (int32_t t = 0; t < k; ++t) {
    int64_t f = factorial(k - 1 - t);
    int32_t d = (int32_t)(r / f);
    r %= f;
    out[t] = avail[d];
    for (int32_t i = d; i < left - 1; ++i) avail[i] = avail[i + 1];
    left--;
  }
}

/* Second heuristic (Section 6.4).  Subsets of S = min(s2, m) consecutive
 * positions; for each subset every permutation of its k items (lexicographic
 * rank r) is packed by its own packer with Rules 2-6; the subset keeps the
 * permutation of least cost, the lowest rank on ties; the instance cost is
 * the sum over subsets.  Criterion of placement t of permutation r of subset
 * I: digit t of output I*S! + r of the H2 stream (orc_criterion_digit). */
static int32_t run_h2(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                      const orc_opts* o, int32_t* assign, int32_t* types,
                      int64_t* cost, orc_stats* st) {
  int32_t S = o->s2 < m ? o->s2 : m;
  int64_t P = factorial(S);
  int32_t l = (m + S - 1) / S;
  uint64_t ck = orc_stream_key(o->seed, STREAM_H2);
  int32_t items[8], order[8], placed_items[8], local[8];
  int64_t smin[8];
  int32_t base = 0;
  *cost = 0;
  for (int32_t I = 0; I < l; ++I) {
    int32_t q0 = I * S;
    int32_t k = (m - q0 < S) ? m - q0 : S;
    for (int32_t t = 0; t < k; ++t) items[t] = item_at(o, m, q0 + t, ORC_H2);
    int64_t kf = factorial(k);
    int64_t best_cost = -1, best_r = -1;
    for (int64_t r = 0; r < kf; ++r) {
      nth_permutation(r, k, order);
      for (int32_t t = k - 1; t >= 0; --t) {
        int64_t v = w[items[order[t]]];
        smin[t] = (t == k - 1 || v < smin[t + 1]) ? v : smin[t + 1];
      }
      opacker p;
      pk_init(&p);
      rule2_bins(&p, n, o->rule2_order);
      for (int32_t t = 0; t < k; ++t) {
        int32_t c = o->force_crit >= 0
                        ? o->force_crit
                        : orc_criterion_digit(ck, (uint64_t)((int64_t)I * P + r), t);
        place(&p, caps, n, w[items[order[t]]], c, 1, o->type_rule, 0, smin[t], st, NULL, NULL,
              NULL);
      }
      int64_t c = packer_cost(&p, caps);
      if (best_r < 0 || c < best_cost) {
        best_cost = c;
        best_r = r;
      }
      pk_free(&p);
      if (st) st->perm_packings++;
    }
    /* re-run the winning permutation to emit its packing */
    nth_permutation(best_r, k, order);
    opacker p;
    pk_init(&p);
    rule2_bins(&p, n, o->rule2_order);
    for (int32_t t = 0; t < k; ++t) {
      int32_t c = o->force_crit >= 0
                      ? o->force_crit
                      : orc_criterion_digit(ck, (uint64_t)((int64_t)I * P + best_r), t);
      placed_items[t] = items[order[t]];
      local[t] = place(&p, caps, n, w[placed_items[t]], c, 1, o->type_rule, 0, 0, NULL, NULL, NULL,
                       NULL);
    }
    base += emit_packer(&p, caps, placed_items, local, k, base, assign, types, cost);
    pk_free(&p);
    if (st) st->packers += 1;
  }
  return base;
}

static int32_t orc_pack_run(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                            int32_t heuristic, const orc_opts* opt, int32_t* assign,
                            int32_t* types, int64_t* cost, orc_stats* stats);

/* Downsizing (with the LARGEST type rule, a pass the paper's Section 1 open
 * type choice invites): a bin's cost is its capacity, so once the packing
 * is fixed every bin can take the smallest type whose capacity holds its
 * load.  Bins, ids and the item assignment are unchanged; types and the
 * cost are recomputed. */
static void downsize_bins(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                          const int32_t* assign, int32_t nb, int32_t* types, int64_t* cost) {
  int64_t* load = (int64_t*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
  for (int32_t j = 0; j < m; ++j) load[assign[j]] += w[j];
  *cost = 0;
  for (int32_t b = 0; b < nb; ++b) {
    int32_t t = 0;
    for (int32_t k = 0; k < n; ++k)
      if (caps[k] >= load[b]) t = k;
    types[b] = t;
    *cost += caps[t];
  }
  free(load);
}

int32_t orc_pack(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                 int32_t heuristic, const orc_opts* opt, int32_t* assign,
                 int32_t* types, int64_t* cost, orc_stats* stats) {
  const int32_t nb = orc_pack_run(w, m, caps, n, heuristic, opt, assign, types, cost, stats);
  if (nb > 0 && opt && opt->downsize) downsize_bins(w, m, caps, n, assign, nb, types, cost);
  return nb;
}

static int32_t orc_pack_run(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                            int32_t heuristic, const orc_opts* opt, int32_t* assign,
                            int32_t* types, int64_t* cost, orc_stats* stats) {
  orc_opts def = {0, 10, 5, ORC_TYPE_SMALLEST_FIT, -1, NULL, NULL, -1, 0, 0, NULL, 0, NULL, 0, 0, 0, 0, 0};
  const orc_opts* o = opt ? opt : &def;
  if (!assign || !types || !cost) return ORC_E_NULL;
  int32_t rc = validate(w, m, caps, n, heuristic, o);
  if (rc != ORC_OK) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  switch (heuristic) {
    case ORC_FF:
    case ORC_BF:
    case ORC_WF:
      return run_plain(w, m, caps, n, heuristic, o, assign, types, cost, stats);
    case ORC_H1:
      return run_h1(w, m, caps, n, o, assign, types, cost, stats);
    default:
      return run_h2(w, m, caps, n, o, assign, types, cost, stats);
  }
}

int32_t orc_pack_packer(const int32_t* w, int32_t m, const int32_t* caps,
                        int32_t n, const int32_t* crit, int32_t rule2,
                        int32_t rule5, int32_t type_rule, int32_t* assign,
                        int32_t* types, int64_t* cost) {
  if (!w || !caps || !crit || !assign || !types || !cost) return ORC_E_NULL;
  int32_t rc = validate(w, m, caps, n, ORC_FF, NULL);
  if (rc != ORC_OK) return rc;
  for (int32_t t = 0; t < m; ++t)
    if (crit[t] < ORC_FF || crit[t] > ORC_WF) return ORC_E_OPTION;
  int32_t* items = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t* local = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  opacker p;
  pk_init(&p);
  if (rule2 < 0 || rule2 > 2) {
    free(items);
    free(local);
    return ORC_E_OPTION;
  }
  if (rule2) rule2_bins(&p, n, rule2 - 1);
  for (int32_t t = 0; t < m; ++t) {
    items[t] = t;
    local[t] = place(&p, caps, n, w[t], crit[t], rule5, type_rule, 0, 0, NULL, NULL, NULL, NULL);
  }
  *cost = 0;
  int32_t nb = emit_packer(&p, caps, items, local, m, 0, assign, types, cost);
  pk_free(&p);
  free(items);
  free(local);
  return nb;
}

/* ---------------------------------------------------------------------- */
/* Lower bounds.                                                           */
/* ---------------------------------------------------------------------- */

int64_t orc_lb_sum(const int32_t* w, int32_t m) {
  int64_t s = 0;
  for (int32_t j = 0; j < m; ++j) s += w[j];
  return s;
}

/* The used bins' capacities must add up to at least the total weight, and
 * any such total is a non-negative integer combination of B_1..B_n: the least
 * reachable total >= sum(w) (unbounded reachability table). */
int64_t orc_lb_cap(const int32_t* w, int32_t m, const int32_t* caps, int32_t n) {
  int64_t total = orc_lb_sum(w, m);
  int64_t top = total + caps[0];
  char* reach = (char*)calloc((size_t)top + 1, 1);
  reach[0] = 1;
  for (int64_t v = 1; v <= top; ++v)
    for (int32_t k = 0; k < n; ++k)
      if (v >= caps[k] && reach[v - caps[k]]) { reach[v] = 1; break; }
  int64_t lb = top;
  for (int64_t v = total; v <= top; ++v)
    if (reach[v]) { lb = v; break; }
  free(reach);
  return lb;
}

/* Two items heavier than B_1/2 never share a bin, so each needs a bin of its
 * own whose capacity is at least its weight. */
int64_t orc_lb_big(const int32_t* w, int32_t m, const int32_t* caps, int32_t n) {
  int64_t lb = 0;
  for (int32_t j = 0; j < m; ++j) {
    if (2 * (int64_t)w[j] > caps[0]) {
      int32_t k = n - 1;
      while (caps[k] < w[j]) --k;
      lb += caps[k];
    }
  }
  return lb;
}

/* ---------------------------------------------------------------------- */
/* Exact optimum for tiny instances.                                       */
/* ---------------------------------------------------------------------- */

/* cheapest single bin holding total s, or -1 */
static int64_t cheapest_bin(int64_t s, const int32_t* caps, int32_t n) {
  if (s > caps[0]) return -1;
  for (int32_t k = n - 1; k >= 0; --k)
    if (caps[k] >= s) return caps[k];
  return -1;
}

/* Method 1: enumerate every set partition of the items (restricted growth
 * strings); a block costs the smallest capacity that holds its total. */
typedef struct {
  const int32_t* w;
  int32_t m;
  const int32_t* caps;
  int32_t n;
  int64_t sums[16];
  int64_t best;
} part_ctx;

static void part_rec(part_ctx* c, int32_t j, int32_t nblocks) {
  if (j == c->m) {
    int64_t tot = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
      int64_t cb = cheapest_bin(c->sums[b], c->caps, c->n);
      if (cb < 0) return;
      tot += cb;
    }
    if (c->best < 0 || tot < c->best) c->best = tot;
    return;
  }
  for (int32_t b = 0; b <= nblocks; ++b) {
    c->sums[b] += c->w[j];
    if (c->sums[b] <= c->caps[0]) part_rec(c, j + 1, b == nblocks ? nblocks + 1 : nblocks);
    c->sums[b] -= c->w[j];
  }
}

int64_t orc_opt_partitions(const int32_t* w, int32_t m, const int32_t* caps, int32_t n) {
  if (m < 1 || m > 12) return -1;
  part_ctx c;
  c.w = w; c.m = m; c.caps = caps; c.n = n; c.best = -1;
  memset(c.sums, 0, sizeof(c.sums));
  part_rec(&c, 0, 0);
  return c.best;
}

/* Method 2: dynamic programme over subsets; best[S] = min over blocks T of S
 * that contain the lowest item of S of cost(T) + best[S \ T]. */
int64_t orc_opt_subset_dp(const int32_t* w, int32_t m, const int32_t* caps, int32_t n) {
  if (m < 1 || m > 12) return -1;
  uint32_t full = (1u << m) - 1u;
  int64_t* blk = (int64_t*)malloc(sizeof(int64_t) * ((size_t)full + 1));
  int64_t* best = (int64_t*)malloc(sizeof(int64_t) * ((size_t)full + 1));
  for (uint32_t s = 0; s <= full; ++s) {
    int64_t tot = 0;
    for (int32_t j = 0; j < m; ++j)
      if (s & (1u << j)) tot += w[j];
    blk[s] = cheapest_bin(tot, caps, n);
  }
  best[0] = 0;
  for (uint32_t s = 1; s <= full; ++s) {
    uint32_t low = s & (~s + 1u);
    uint32_t rest = s ^ low;
    int64_t bs = -1;
    /* every subset t of rest; the block is t | low */
    uint32_t t = rest;
    for (;;) {
      uint32_t blkset = t | low;
      if (blk[blkset] >= 0 && best[s ^ blkset] >= 0) {
        int64_t v = blk[blkset] + best[s ^ blkset];
        if (bs < 0 || v < bs) bs = v;
      }
      if (t == 0) break;
      t = (t - 1) & rest;
    }
    best[s] = bs;
  }
  int64_t r = best[full];
  free(blk);
  free(best);
  return r;
}
