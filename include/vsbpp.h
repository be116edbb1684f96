/*
 * vsbpp.h -- C ABI of the MI355X (gfx950) implementation of the placement
 * hot path of the Variable Sized Bin Packing heuristics of Alenezi,
 * Aboelfotoh, Albdaiwi & Almulla, "Heuristics for the Variable Sized Bin
 * Packing Problem Using a Hybrid P System and CUDA Architecture".
 *
 * Problem (paper Section 1, "Formal Definition of VSBPP", and Section 6.1):
 * n bin types with capacities B_1 > B_2 > ... > B_n > 0, unlimited supply of
 * each; m indivisible items with integer weights 1 <= w_j <= B_1; a packing
 * puts every item in one bin without exceeding any bin's capacity; its cost
 * is the sum of the capacities of the bins that hold at least one item.
 *
 * Heuristics:
 *   VSBPP_FF / VSBPP_BF / VSBPP_WF -- First, Best and Worst Fit (Section 1)
 *       over the whole list in order: the item goes to the lowest-index open
 *       bin it fits (FF), to the fitting bin with least room left after it
 *       (BF) or most room left after it (WF); ties go to the lowest index.
 *       When no open bin fits, a bin is opened.
 *   VSBPP_H1 -- the first hybrid-P-system heuristic (Section 6.3): the items
 *       are distributed into sublists of s1 items (Rule 1), each sublist is
 *       packed independently starting from one empty bin of every type
 *       (Rule 2), every item is tagged FF, BF or WF with equal probability
 *       (Rule 3) and placed by that criterion (Rule 4), and a bin whose load
 *       reaches half its capacity divides once into a new empty bin of its
 *       type (Rule 5).
 *   VSBPP_H2 -- the second heuristic (Section 6.4): subsets of s2 items; every
 *       permutation of a subset is packed with Rules 2-6; each subset keeps
 *       its cheapest permutation (lowest permutation rank on ties); the
 *       instance cost is the sum over subsets.
 *
 * Readings where the paper leaves a choice open (fixed here so results are
 * reproducible bit for bit):
 *   - an item fits a bin when load + w <= capacity;
 *   - a bin opened because nothing fits has type max{k : B_k >= w} (the
 *     smallest capacity that holds the item) unless options say otherwise;
 *   - Rule 1's random distribution is the keyed permutation pi of [0,m): a
 *     4-round balanced Feistel network whose round function is SplitMix64,
 *     restricted to [0,m) by cycle walking; position q holds item pi(q) and
 *     sublists/subsets are consecutive runs of positions;
 *   - Rule 3's equal-probability draw uses SplitMix64 (Steele, Lea & Flood,
 *     2014) with one key per purpose derived from the seed.  H1: position q
 *     takes the output x for counter q and criterion floor(3*hi32(x)/2^32).
 *     H2: the packing of permutation rank r of subset I (S items) takes one
 *     output for counter I*S! + r; with h its high 32 bits, placement t
 *     (0-based) takes base-3 digit t+1 of h/2^32, i.e.
 *     floor(3^(t+1)*h/2^32) mod 3;
 *   - Rule 5 is checked right after every placement, at most once per bin;
 *   - output bin ids: bins holding items, in creation order, packer after
 *     packer (sublist or subset order); empty Rule-2/Rule-5 bins cost nothing
 *     and are not output.
 *
 * Type indices are 0-based: type 0 is B_1.  Every packing computation is
 * integer.  Memory: the caller owns every buffer; the library keeps no
 * pointer after a call returns.  Errors never leave partial results in the
 * output buffers of the host-pointer calls.
 */
#ifndef VSBPP_H
#define VSBPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VSBPP_FF = 0, VSBPP_BF = 1, VSBPP_WF = 2, VSBPP_H1 = 3, VSBPP_H2 = 4 };

/* type of a bin opened when no open bin fits; LEARNED asks the scorer
 * (plain FF/BF/WF only, see vsbpp_pack_batch_ex) */
enum { VSBPP_TYPE_SMALLEST_FIT = 0, VSBPP_TYPE_LARGEST = 1, VSBPP_TYPE_LEARNED = 2 };

enum {
  VSBPP_OK = 0,
  VSBPP_E_NULL = -1,      /* a required pointer is NULL                       */
  VSBPP_E_SIZE = -2,      /* m < 1, n < 1, n > 16, or a declared bound is
                             exceeded, or the instance is beyond the device
                             limits (see vsbpp_pack_batch)                    */
  VSBPP_E_CAPS = -3,      /* capacities not > 0 or not strictly decreasing    */
  VSBPP_E_WEIGHT = -4,    /* a weight < 1 or > B_1                            */
  VSBPP_E_HEURISTIC = -5, /* unknown heuristic                                */
  VSBPP_E_OPTION = -6,    /* bad option (s1, s2, type rule, criterion, order) */
  VSBPP_E_DEVICE = -7,    /* no usable gfx950 device or a HIP runtime error   */
  VSBPP_E_NOMEM = -8,     /* device allocation failed                          */
  VSBPP_E_MODEL = -9      /* the learned type rule without a model, a model
                             file that is missing, of the wrong size, with
                             n_out outside 1..16 or a non-finite parameter,
                             or a buffer that is not a trainer checkpoint     */
};
/* Argument checks run in this order and the first failure is returned:
 * NULL, SIZE, CAPS, WEIGHT, HEURISTIC, OPTION, MODEL. */

/* Options.  Fill with vsbpp_options_init() first. */
typedef struct vsbpp_options {
  uint32_t struct_size;     /* sizeof(vsbpp_options)                           */
  uint64_t seed;            /* generator key for Rules 1 and 3 (default 0)     */
  int32_t h1_items_per_sublist; /* s1, 1..16 (default 10, paper Table 1)       */
  int32_t h2_subset_size;   /* s2, 1..6 with s2! <= 1024 (default 5, Tables 1,
                               4 and 6)                                        */
  int32_t type_rule;        /* VSBPP_TYPE_* (default SMALLEST_FIT)             */
  int32_t force_criterion;  /* -1: Rule 3 draws per placement (default);
                               0/1/2: every H1/H2 placement uses FF/BF/WF      */
  const int32_t* order;     /* optional item order: order[q] is the item at
                               position q (a permutation of 0..m-1).  Plain
                               heuristics pack in this order; H1/H2 use it in
                               place of Rule 1's drawn permutation.  Host
                               pointer for vsbpp_pack_ex; ignored by
                               vsbpp_pack_batch (which takes d_order).         */
  int32_t active_limit;     /* plain FF/BF/WF: at most this many bins open at
                               once (0, the default: no limit).  Section 1
                               has Best Fit keep a fixed number of bins
                               active; when a bin must open while this many
                               are open, the fullest open bin (least room,
                               lowest index on ties) closes and takes no more
                               items.  Nonzero with H1/H2: VSBPP_E_OPTION.
                               (Appended last: callers built against the
                               shorter struct keep working through
                               struct_size.)                                   */
  int32_t downsize;         /* 1: after packing, every bin takes the smallest
                               type whose capacity holds its load, and the cost
                               is recomputed (bins and the assignment are
                               kept).  With VSBPP_TYPE_LARGEST this is the
                               "largest type, then shrink" rule.  A pass over
                               the outputs, so it does not change the choices
                               the heuristic made (H2's permutation minimum
                               included).  0 (default) or 1, else
                               VSBPP_E_OPTION; not with decision-hook entries
                               that name a source instance.                   */
  int32_t criterion_rule;   /* H1 only: 0 (default) Rule 3 draws FF/BF/WF with
                               equal probability; 1 a trained network picks
                               the criterion wherever FF, BF and WF would put
                               the item into different bins (see the learned
                               criterion below).  1 needs a model, so only
                               vsbpp_pack_batch_ex and vsbpp_plan_create_ex
                               take it (the other calls: VSBPP_E_MODEL);
                               with another heuristic or a forced criterion:
                               VSBPP_E_OPTION.                                */
  int32_t choice_rule;      /* plain FF/BF/WF under VSBPP_TYPE_LARGEST with
                               downsize 1 and no bound on the open bins (else
                               VSBPP_E_OPTION): 0 (default) the criterion's
                               bin always; 1 the same, but the decisions of
                               the run (decision hooks) are its contested
                               placements; 2 a trained network chooses at
                               each contested placement between the
                               criterion's bin and a new bin (see the learned
                               bin choice below).  2 needs a model, so only
                               vsbpp_pack_batch_ex and vsbpp_plan_create_ex
                               take it (the other calls: VSBPP_E_MODEL).     */
  int32_t rule2_order;      /* H1/H2: the order in which Rule 2 creates a
                               packer's empty bins (Section 6.3 gives none; it
                               decides First Fit's lowest index and ties):
                               0 (default) type order, B_1 first; 1
                               increasing capacity, B_n first.  Nonzero with
                               plain FF/BF/WF: VSBPP_E_OPTION.                */
} vsbpp_options;

void vsbpp_options_init(vsbpp_options* opt);

/* Packs one instance (host pointers, synchronous, default options).
 *   weights[m]          item weights, 1 <= w <= capacities[0]
 *   capacities[n]       B_1 > ... > B_n > 0, 1 <= n <= 16
 *   out_assignment[m]   receives the bin id of every item, in [0, nbins)
 *   out_bin_types[m]    receives the type index of bins 0..nbins-1 (room for
 *                       m entries; nbins <= m)
 * Returns nbins >= 1, or a negative VSBPP_E_* code (outputs untouched). */
int32_t vsbpp_pack(const int32_t* weights, int32_t m, const int32_t* capacities, int32_t n,
                   int32_t heuristic, int32_t* out_assignment, int32_t* out_bin_types);

/* As vsbpp_pack with options (opt may be NULL for the defaults) and the
 * packing cost written to *out_cost (may be NULL). */
int32_t vsbpp_pack_ex(const int32_t* weights, int32_t m, const int32_t* capacities, int32_t n,
                      int32_t heuristic, const vsbpp_options* opt, int32_t* out_assignment,
                      int32_t* out_bin_types, int64_t* out_cost);

/* Packs a batch of independent instances held in device memory, in one
 * launch, asynchronously on `hip_stream` (a hipStream_t; NULL = the default
 * stream).  No host synchronisation, no device allocation: the call can be
 * captured into a HIP graph.
 *
 * Layout (CSR, all device pointers):
 *   d_weights[sum m]         weights of instance i at [d_item_off[i], d_item_off[i+1])
 *   d_item_off[N+1]          int64 offsets, d_item_off[0] = 0
 *   d_capacities[sum n]      capacities of instance i at [d_cap_off[i], d_cap_off[i+1])
 *   d_cap_off[N+1]           int32 offsets
 *   d_order[sum m] or NULL   per-instance item order (local ids 0..m_i-1),
 *                            same offsets as the weights
 *   d_seeds[N] or NULL       per-instance generator keys (else opt->seed)
 * Bounds the caller guarantees (they size the launch):
 *   max_items     >= every m_i     (plain FF/BF/WF: this call keeps the
 *                                   bins of an instance in LDS, which limits
 *                                   max_items to about 26000, or 13000 when
 *                                   max_capacity > 32767 or max_items >
 *                                   65535; beyond that it returns
 *                                   VSBPP_E_SIZE, while plans and the
 *                                   host-pointer calls keep the bins in a
 *                                   device region they allocate instead.
 *                                   The scorer and the decision hooks need
 *                                   the bins in LDS.)
 *   max_types     >= every n_i, <= 16
 *   max_capacity  >= every B_1 of the batch
 * Outputs (device):
 *   d_assignment[sum m]  bin id of every item, local to its instance
 *   d_bin_types[sum m]   type of bins 0..nbins_i-1 of instance i, at the
 *                        instance's item offset
 *   d_nbins[N]           nbins_i >= 1, or a negative VSBPP_E_* code for an
 *                        instance that fails the checks (its other outputs
 *                        are then unspecified)
 *   d_cost[N]            packing cost of every instance (0 on error)
 * Returns VSBPP_OK or a negative code for errors detectable on the host
 * (nothing is launched then).  d_order must be a permutation per instance;
 * an entry outside [0, m_i) gives VSBPP_E_OPTION for that instance. */
int32_t vsbpp_pack_batch(int32_t num_instances, const int32_t* d_weights,
                         const int64_t* d_item_off, const int32_t* d_capacities,
                         const int32_t* d_cap_off, int32_t max_items, int32_t max_types,
                         int32_t max_capacity, int32_t heuristic, const vsbpp_options* opt,
                         const int32_t* d_order, const uint64_t* d_seeds,
                         int32_t* d_assignment, int32_t* d_bin_types, int32_t* d_nbins,
                         int64_t* d_cost, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Plans: a batch bound to its buffers, a heuristic and a launch shape, run   */
/* any number of times.  A plan owns a device workspace (a work counter, an  */
/* instance schedule and, for plain FF/BF/WF instances whose bins do not fit */
/* LDS, max_items-sized arrays per instance) allocated when it is created,   */
/* so runs allocate nothing and may be captured into, or replayed from, a    */
/* HIP graph.                                                                */
/* ------------------------------------------------------------------------ */

/* A device-resident batch: the same CSR layout, bounds and outputs as the
 * arguments of vsbpp_pack_batch (see there). */
typedef struct vsbpp_batch {
  int32_t num_instances;
  const int32_t* weights;
  const int64_t* item_off;
  const int32_t* capacities;
  const int32_t* cap_off;
  const int32_t* order;   /* or NULL */
  const uint64_t* seeds;  /* or NULL */
  int32_t max_items, max_types, max_capacity;
  int32_t* assignment;
  int32_t* bin_types;
  int32_t* nbins;
  int64_t* cost;
} vsbpp_batch;

/* Launch shape.  mode 0: one wavefront (FF/BF/WF) or one workgroup (H1/H2)
 * per instance, in a grid covering the batch; mode 1: persistent grid of
 * resident workgroups taking instances from a device work counter.  lpt = 1
 * processes instances by decreasing item count (largest first, for uneven
 * batches; batches up to 8192 instances).  waves_per_block: FF/BF/WF
 * wavefronts per workgroup, 1..8 (1..4 with fewer than 64 lanes per
 * instance).  block_threads: H1/H2 workgroup size (H2: a multiple of
 * roundup(s2!, 64)).  lanes_per_instance: FF/BF/WF lanes that test one
 * instance's bins, 64 (one instance per wavefront; 0 means 64), 32 or 16
 * (two or four instances per wavefront, stepping through their items
 * together; only for runs with B_1 <= 32767, m <= 65535, no scorer, hooks
 * or bound on the open bins, whose bins fit LDS, else VSBPP_E_OPTION). */
typedef struct vsbpp_launch {
  int32_t mode;
  int32_t lpt;
  int32_t waves_per_block;
  int32_t block_threads;
  int32_t lanes_per_instance;
  int32_t waves_per_instance;  /* FF/BF/WF: 1 (0 means 1), or 2 or 4
                                  wavefronts of one workgroup sharing one
                                  instance's bins (its groups of 256 bin
                                  positions dealt out among them; one barrier
                                  per item), for instances of thousands of
                                  items; only for runs with B_1 <= 32767, m <=
                                  65535, no scorer, hooks or bound on the
                                  open bins, whose bins fit one workgroup's
                                  LDS, and with lanes_per_instance 64, else
                                  VSBPP_E_OPTION.  waves_per_block is then
                                  ignored. (Appended last.)                   */
} vsbpp_launch;

enum {
  VSBPP_PLAN_GRAPH = 1,     /* capture the launch sequence into a hipGraph    */
  VSBPP_PLAN_AUTOTUNE = 2   /* time the candidate launch shapes on the batch
                               (running it several times) and keep the
                               fastest; results are cached per process and,
                               when the environment variable VSBPP_TUNE_CACHE
                               names a file, in that file                    */
};

typedef struct vsbpp_plan vsbpp_plan;

/* Creates a plan.  `launch` (may be NULL) forces a launch shape; otherwise
 * the shape comes from the tuning cache, from tuning (VSBPP_PLAN_AUTOTUNE)
 * or from defaults.  Autotuning runs the batch on the device, synchronously.
 * Returns VSBPP_OK or a negative code; *out is NULL on error. */
int32_t vsbpp_plan_create(const vsbpp_batch* batch, int32_t heuristic, const vsbpp_options* opt,
                          const vsbpp_launch* launch, uint32_t flags, vsbpp_plan** out);
/* As vsbpp_plan_create with a scorer: opt->type_rule VSBPP_TYPE_LEARNED and
 * d_model (a device pointer to a vsbpp_model, e.g. from vsbpp_model_load,
 * which must stay valid while the plan is used; VSBPP_E_MODEL when it is
 * NULL); plain FF/BF/WF only.  Declared with the scorer below. */
struct vsbpp_model;
int32_t vsbpp_plan_create_ex(const vsbpp_batch* batch, int32_t heuristic,
                             const vsbpp_options* opt, const struct vsbpp_model* d_model,
                             const vsbpp_launch* launch, uint32_t flags, vsbpp_plan** out);
/* Enqueues one run on hip_stream (graph replay when captured). */
int32_t vsbpp_plan_run(vsbpp_plan* plan, void* hip_stream);
/* Launch shape the plan uses. */
int32_t vsbpp_plan_launch(const vsbpp_plan* plan, vsbpp_launch* out);
/* Releases the plan, its workspace and graph (after outstanding runs). */
void vsbpp_plan_destroy(vsbpp_plan* plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one run of
 * a device batch with a chosen launch shape, as a plan created with that
 * shape would run it, but with no plan and no allocation of any kind.  The
 * work counter of persistent launches (mode 1) and the largest-first
 * schedule (lpt 1) live in one device array inside the library, a copy per
 * GPU held until the process ends: 1 + 8192 int32 (32 KiB + 4 B), so lpt 1
 * takes at most 8192 instances (more: VSBPP_E_SIZE).  Plain FF/BF/WF runs
 * whose bins do not fit LDS need a plan's device region and return
 * VSBPP_E_SIZE here, as from vsbpp_pack_batch.  `launch` may be NULL (the
 * default shape).  The learned rules take a model and are not run here
 * (VSBPP_E_MODEL).  Every call on one GPU uses that GPU's array: the counter
 * is reset by a kernel on hip_stream before each run, and calls that overlap
 * on one GPU (other streams or threads) race.  Asynchronous on hip_stream;
 * returns VSBPP_OK or the codes of vsbpp_plan_create in its order of checks
 * (nothing is launched on error). */
int32_t vsbpp_pack_batch_static(const vsbpp_batch* batch, int32_t heuristic,
                                const vsbpp_options* opt, const vsbpp_launch* launch,
                                void* hip_stream);

/* Exact optimum of every instance of a device-resident batch with at most
 * 12 items per instance (batch->max_items <= 12), for measuring heuristic
 * and learned packings against the optimum.  The cost of a packing is the
 * sum of the capacities of its bins (Section 1, formal definition), so a bin holding a set of
 * items costs the smallest capacity that holds their total and the optimum
 * is the cheapest partition of the items into such sets.  The call evaluates
 * it exactly, by dynamic programming over the subsets of the items.
 *   batch    the CSR inputs and bounds of vsbpp_pack_batch (order and seeds
 *            are ignored); every instance needs 1 <= m_i <= 12
 *   outputs  d_cost[i]   the optimum cost;
 *            d_nbins[i]  the bins of one optimal packing, or a negative
 *                        VSBPP_E_* code for an instance that fails the checks
 *                        of vsbpp_pack_batch or has more than max_items or
 *                        12 items (its other outputs are then unspecified);
 *            d_assignment / d_bin_types  that packing, in the layout of
 *                        vsbpp_pack_batch.  Its bins are ordered by their
 *                        lowest item and each has the smallest type that
 *                        holds its load.  Where several packings are optimal
 *                        it is the one whose first bin, as a bit mask of
 *                        items, is smallest, then the same rule for the
 *                        items left.
 * Asynchronous on hip_stream, no device allocation (graph-capturable).
 * Returns VSBPP_OK, VSBPP_E_NULL, VSBPP_E_SIZE (max_items outside 1..12,
 * max_types outside 1..16, max_capacity < 1) or VSBPP_E_DEVICE. */
int32_t vsbpp_exact_batch(const vsbpp_batch* batch, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Learned bin-type scorer.                                                  */
/*                                                                            */
/* A decision is an item that fits no open bin in a plain FF/BF/WF run; the  */
/* scorer proposes the type of the bin it opens, among the types that hold   */
/* the item.  Capacity checks stay exact integer; a non-finite score falls   */
/* back to the smallest fitting type, and that plain rule is the baseline    */
/* the scorer's cost is judged against.                                      */
/*                                                                            */
/* Decision features (fp32), for item w at position q of m, before the bin  */
/* opens:                                                                     */
/*   0  w / B_1                                                               */
/*   1  (m - q - 1) / m                                                       */
/*   2  mean weight of the items after q / B_1 (0 if none)                    */
/*   3  smallest weight after q / B_1 (1 if none)                             */
/*   4  bins opened so far / m                                                */
/*   5..10  share of the bins opened so far whose room r falls in bucket     */
/*          floor(6 r / (B_1 + 1)) = 0..5                                     */
/*   11..14 B_2 .. B_5 over B_1 (0 beyond n)                                  */
/*   15 w / (smallest capacity >= w)                                          */
/* Arithmetic: integers convert to fp32 first; "a / b" with b one of B_1, m, */
/* the bins opened so far (at least 1) or a capacity is a * (1.0f / b), the */
/* product with the fp32 reciprocal; the mean in feature 2 is the fp32      */
/* quotient (sum / count), then times 1/B_1.                                */
/* Network: h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64),           */
/* z = W3 h2 + b3 (n_out).  Every unit, hidden or output, is its bias       */
/* followed by a chain of fp32 fused multiply-adds over its inputs in index  */
/* order, so results are reproducible bit for bit.                           */
/* Decision: the type k < min(n, n_out) holding                              */
/* the item with the largest z, lowest k on ties; decisions where only B_1   */
/* holds the item are not scored.                                            */
/* ------------------------------------------------------------------------ */

#define VSBPP_NFEAT 16
#define VSBPP_HIDDEN 64
#define VSBPP_MAX_OUT 16

/* Weights as bfloat16 bit patterns, biases fp32, row-major [out][in]. */
typedef struct vsbpp_model {
  int32_t n_out;
  uint16_t w1[VSBPP_HIDDEN * VSBPP_NFEAT];
  float b1[VSBPP_HIDDEN];
  uint16_t w2[VSBPP_HIDDEN * VSBPP_HIDDEN];
  float b2[VSBPP_HIDDEN];
  uint16_t w3[VSBPP_MAX_OUT * VSBPP_HIDDEN];
  float b3[VSBPP_MAX_OUT];
} vsbpp_model;

/* Decision hooks of a plain FF/BF/WF batch (all device pointers, each may be
 * NULL).  Entry e of the batch reads the inputs of instance src[e] (the
 * batch's CSR arrays, weights/capacities/order/seed) -- so one instance can
 * be packed by many entries -- and writes d_nbins[e] and d_cost[e].  With
 * src set, the assignment and bin-type outputs are not written (they may be
 * NULL).  force[3e..3e+2] = (d, t1, t2): the bin opened at decision d of
 * entry e gets type t1 and the one at decision d+1 type t2 (a type that does
 * not hold the item is ignored; d = -1 forces nothing).  At decision d,
 * features[16e..16e+15] receive the decision features and info[2e] the mask
 * of types holding the item (bit k for B_k >= w), info[2e+1] the smallest
 * fitting type; entries whose run has no decision d leave them untouched.
 * count[e] receives the number of decisions of entry e's run (plain
 * FF/BF/WF; appended last, so a caller that zero-fills the struct before
 * setting the fields it knows keeps working). */
typedef struct vsbpp_decisions {
  const int32_t* src;
  const int32_t* force;
  float* features;
  int32_t* info;
  int32_t* count;
} vsbpp_decisions;

/* Learned criterion of the first heuristic (opt->criterion_rule = 1, Section
 * 6.3's Rule 3 replaced where it matters).  At a placement where First, Best
 * and Worst Fit would choose different bins of the packer, the network
 * (n_out >= 3; outputs 0, 1, 2 score FF, BF, WF) is evaluated on these fp32
 * features, the rest 0 ("a / b" is a times the fp32 reciprocal of b):
 *   0  w / B_1                 1  t / k (position t of a sublist of k items)
 *   2  room left in FF's bin after the item / B_1
 *   3  the same for BF's bin   4  the same for WF's bin
 *   5  bins the item fits / 16 6  bins in the packer (Rule 2 and 5 bins
 *                                 included) / 32
 * and the criterion with the largest score is used, lowest on ties.  Where
 * the three agree or nothing fits, the criterion does not change the
 * placement and Rule 3's draw stands; non-finite scores also keep the draw.
 * The network's arithmetic is that of the bin-type scorer.  A model with
 * fewer than 3 outputs gives VSBPP_E_MODEL in every instance's d_nbins. */

/* Learned bin choice (opt->choice_rule = 2; plain FF/BF/WF, largest type
 * rule, downsizing; Section 1 leaves the choice of bins and types beyond the
 * three rules open).  After downsizing a bin of load L costs c(L), the
 * smallest capacity >= L.  Placing item w into the criterion's bin (load L)
 * is contested when c(L + w) > c(L).  There the network (n_out >= 2;
 * outputs 0 = keep the criterion's bin, 1 = open a new bin of type B_1)
 * is evaluated on these fp32 features ("a / b" is a times the fp32
 * reciprocal of b): 0..10 as features 0..10 of a bin-type decision (the
 * histogram over all bins, every bin with capacity B_1), then
 *   11 (B_1 - L - w) / B_1     12 (c(L + w) - c(L)) / B_1
 *   13 c(w) / B_1              14 (c(L + w) - L - w) / B_1
 *   15 (c(L) - L) / B_1
 * A new bin opens only when output 1 is strictly larger and both are
 * finite.  Bins opened because nothing fits are not decisions.  The
 * decision hooks then index contested placements: force t1/t2 are 0 (keep)
 * or 1 (open), info[2e] = 3 (both allowed) and info[2e+1] = 0 (the plain
 * choice).  A model with fewer than 2 outputs gives VSBPP_E_MODEL in every
 * instance's d_nbins.  The network's arithmetic is that of the bin-type
 * scorer. */

/* vsbpp_pack_batch with a scorer (d_model: device pointer to a vsbpp_model,
 * e.g. from vsbpp_model_load, required when opt->type_rule is
 * VSBPP_TYPE_LEARNED, opt->criterion_rule is 1 or opt->choice_rule is 2 --
 * VSBPP_E_MODEL when it is NULL -- else ignored) and decision hooks (dec may
 * be NULL).  The bin-type
 * scorer and the hooks above are for plain FF/BF/WF.  With H1, dec may carry
 * features and info only (src and force: VSBPP_E_OPTION), in another
 * layout: for the item at position q of instance i (offset off_i of its
 * items), info[off_i + q] = 1 when the placement was contested (the three
 * criteria choose different bins) and 0 otherwise, and a contested
 * placement's 16 features go to features[16*(off_i + q) ..].  Asynchronous
 * on hip_stream, no allocation. */
int32_t vsbpp_pack_batch_ex(const vsbpp_batch* batch, int32_t heuristic,
                            const vsbpp_options* opt, const vsbpp_model* d_model,
                            const vsbpp_decisions* dec, void* hip_stream);

/* Depth-2 lookahead labels from rollout costs.  d_cost holds, for decision
 * i, k1 and k2 in [0, n_types), the cost of the run with k1 forced at the
 * decision and k2 at the next one, at index (i*n_types + k1)*n_types + k2;
 * d_info holds the (feasible mask, smallest fitting type) pair of each
 * decision.  V(k1) = min over k2; the label is argmin over feasible k1 of V,
 * ties to the smallest fitting type when it is among them, else the lowest
 * type.  Writes d_labels[num_decisions] (and d_values[num*n_types] with -1
 * for infeasible types, when not NULL). */
int32_t vsbpp_rollout_labels(const int64_t* d_cost, const int32_t* d_info,
                             int32_t num_decisions, int32_t n_types, int32_t* d_labels,
                             int64_t* d_values, void* hip_stream);

/* Training of the scorer on the GPU: fp32 master weights, bfloat16 working
 * weights (round to nearest even after every step), forward and backward
 * with fp32 accumulation, masked softmax cross-entropy over the feasible
 * types, Adam.  Gradients are summed over the minibatch (mean over its
 * samples) in a fixed order, so training is deterministic. */
typedef struct vsbpp_trainer vsbpp_trainer;

/* init: host model holding the initial weights (their fp32 values are the
 * bf16 ones); n_out in 1..16. */
int32_t vsbpp_trainer_create(const vsbpp_model* init, vsbpp_trainer** out);
/* One step on the minibatch d_idx[batch] of the training set d_x[N*16]
 * (features), d_mask[N] (feasible types), d_label[N]; lr, beta1, beta2, eps
 * as in Adam.  *out_loss (host, may be NULL) receives the minibatch mean
 * loss after the step's forward pass (this synchronises).  Asynchronous
 * otherwise. */
int32_t vsbpp_trainer_step(vsbpp_trainer* tr, const float* d_x, const int32_t* d_mask,
                           const int32_t* d_label, const int32_t* d_idx, int32_t batch,
                           float lr, float beta1, float beta2, float eps, float* out_loss,
                           void* hip_stream);
/* Gradient of the mean loss over the minibatch at the current weights,
 * without an update: host out[] in the order w1, b1, w2, b2, w3 (n_out rows),
 * b3 (n_out); returns the number of values written.  Synchronous. */
int32_t vsbpp_trainer_gradient(vsbpp_trainer* tr, const float* d_x, const int32_t* d_mask,
                               const int32_t* d_label, const int32_t* d_idx, int32_t batch,
                               float* out, int32_t out_cap);
/* Device pointer to the current bf16 model (for vsbpp_pack_batch_ex). */
const vsbpp_model* vsbpp_trainer_device_model(const vsbpp_trainer* tr);
/* Copies the current bf16 model to host memory (synchronous). */
int32_t vsbpp_trainer_export(const vsbpp_trainer* tr, vsbpp_model* out);
/* Checkpoint and resume (for callers that train in several sessions): the
 * trainer's whole state -- its step count (Adam's bias correction), current
 * bf16 model, fp32 master weights and both Adam moments -- as one host byte
 * buffer of vsbpp_trainer_state_bytes(tr) bytes (negative: VSBPP_E_NULL).
 * vsbpp_trainer_save writes it into buf (cap bytes; VSBPP_E_SIZE when
 * smaller); vsbpp_trainer_restore loads one into a trainer created with the
 * same n_out (VSBPP_E_SIZE on a size or n_out mismatch, VSBPP_E_MODEL when
 * buf is not a trainer checkpoint), after which steps continue exactly as
 * they would have in the saved trainer.  Both synchronise the device; the
 * caller owns buf. */
int64_t vsbpp_trainer_state_bytes(const vsbpp_trainer* tr);
int32_t vsbpp_trainer_save(const vsbpp_trainer* tr, void* buf, int64_t cap);
int32_t vsbpp_trainer_restore(vsbpp_trainer* tr, const void* buf, int64_t size);
void vsbpp_trainer_destroy(vsbpp_trainer* tr);

/* Lower bounds of the optimum of every instance of a device CSR batch (the
 * denominator of the cost/LB quality figure): d_out[3i] = total weight,
 * d_out[3i+1] = LB_cap, the least total >= the weight that is a sum of
 * capacities with repetition (exact when the smallest capacity is <= 8192,
 * else the total weight), d_out[3i+2] = LB_big, the sum over items heavier
 * than B_1/2 of the smallest capacity holding them.  LB = max(LB_cap, LB_big).
 * An instance with m < 1 or n outside 1..16 gets -1s.  Asynchronous. */
int32_t vsbpp_lower_bounds(int32_t num, const int32_t* d_weights, const int64_t* d_item_off,
                           const int32_t* d_capacities, const int32_t* d_cap_off, int64_t* d_out,
                           void* hip_stream);

/* Cost of a packing (Section 1, formal definition; Section 6.1): the sum of
 * the capacities of its bins, sum over b < nbins of capacities[bin_types[b]]
 * (host pointers; bin_types may be NULL when nbins is 0).  Returns the cost
 * (>= 0) or a negative VSBPP_E_* code: NULL, SIZE (nbins < 0, n outside
 * 1..16, or a type index outside [0, n)), CAPS. */
int64_t vsbpp_cost(const int32_t* bin_types, int32_t nbins, const int32_t* capacities,
                   int32_t n);

/* Lower bound on the optimum cost of one instance (host pointers,
 * synchronous, no device use): max(LB_cap, LB_big).  The bins of any packing
 * hold the total weight W, and their capacities are a sum of B_1..B_n with
 * repetition, so the cost is at least LB_cap, the least such sum >= W
 * (exact when B_n <= 2^20; above that W itself is returned for LB_cap).
 * Items heavier than B_1/2 pairwise cannot share a bin, so the cost is also
 * at least LB_big, the sum over those items of the smallest capacity
 * holding each.  The same bounds as vsbpp_lower_bounds computes per
 * instance on the device (whose LB_cap is exact only when B_n <= 8192).
 * Returns the bound or a negative code: NULL, SIZE (m < 1, n outside
 * 1..16), CAPS, WEIGHT. */
int64_t vsbpp_lower_bound(const int32_t* weights, int32_t m, const int32_t* capacities,
                          int32_t n);

/* Loads a trained scorer: the file holds one vsbpp_model exactly as laid
 * out above (little-endian, sizeof(vsbpp_model) bytes; the layout the
 * trainer exports).  Checks the size, 1 <= n_out <= 16 and that every weight
 * and bias in use is finite, then copies the model to device memory of the
 * current device; *out receives that device pointer, ready for
 * vsbpp_pack_batch_ex and vsbpp_plan_create_ex.  The caller releases it with
 * vsbpp_model_free.  Returns VSBPP_OK, VSBPP_E_NULL, VSBPP_E_MODEL (file
 * missing or unreadable, or a failed check), VSBPP_E_DEVICE or
 * VSBPP_E_NOMEM; *out is NULL on error. */
int32_t vsbpp_model_load(const char* path, vsbpp_model** out);
/* Frees a model returned by vsbpp_model_load (NULL is ignored). */
void vsbpp_model_free(vsbpp_model* d_model);

/* Best of a batch: writes d_out[0] = min cost and d_out[1] = the lowest index
 * reaching it over d_cost[0..num-1] (device pointers, asynchronous on
 * hip_stream).  Used to keep the best of several orderings of one instance. */
int32_t vsbpp_best_of(const int64_t* d_cost, int32_t num, int64_t* d_out, void* hip_stream);

/* Achievable on-chip peaks of the current device, measured now by two
 * stream kernels (synchronous, a few milliseconds): out[0] = LDS read
 * bandwidth in bytes/s (16-byte reads at unit lane stride, no bank
 * conflicts, 16 workgroups of 256 threads per compute unit), out[1] = 32-bit
 * integer VALU lane-operations/s (independent add/xor/min chains).
 * The packing kernels' roofline fractions are taken against these next to
 * the published peaks.  Returns VSBPP_OK, VSBPP_E_NULL, VSBPP_E_DEVICE or
 * VSBPP_E_NOMEM. */
int32_t vsbpp_measure_peaks(double* out);

/* Text of an error code (static storage). */
const char* vsbpp_strerror(int32_t code);

/* Detail of the last HIP runtime failure reported as VSBPP_E_DEVICE by this
 * thread (empty if none); static thread-local storage. */
const char* vsbpp_last_error(void);

/* 1 if a gfx950 device is visible and usable, else 0. */
int32_t vsbpp_device_ok(void);

#ifdef __cplusplus
}
#endif
#endif /* VSBPP_H */
