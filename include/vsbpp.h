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
 *   - Rule 3 draws criterion floor(3*hi32(x)/2^32) from the SplitMix64 output
 *     x for counter q (H1, position q) or (I*S! + r)*S + t (H2, subset I,
 *     permutation rank r, placement t), with per-purpose keys derived from
 *     the seed;
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

/* type of a bin opened when no open bin fits */
enum { VSBPP_TYPE_SMALLEST_FIT = 0, VSBPP_TYPE_LARGEST = 1 };

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
  VSBPP_E_NOMEM = -8      /* device allocation failed                          */
};

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
 *   max_items     >= every m_i     (plain FF/BF/WF: the bins of one instance
 *                                   must fit in LDS, which limits max_items
 *                                   to about 26000, or 16000 when
 *                                   max_capacity > 32767)
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
/* any number of times.  A plan owns a small device workspace (a work        */
/* counter and an instance schedule) allocated when it is created, so runs   */
/* allocate nothing and may be captured into, or replayed from, a HIP graph. */
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
 * wavefronts (one instance each) per workgroup, 1..4.  block_threads: H1/H2
 * workgroup size (H2: a multiple of roundup(s2!, 64)). */
typedef struct vsbpp_launch {
  int32_t mode;
  int32_t lpt;
  int32_t waves_per_block;
  int32_t block_threads;
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
/* Enqueues one run on hip_stream (graph replay when captured). */
int32_t vsbpp_plan_run(vsbpp_plan* plan, void* hip_stream);
/* Launch shape the plan uses. */
int32_t vsbpp_plan_launch(const vsbpp_plan* plan, vsbpp_launch* out);
/* Releases the plan, its workspace and graph (after outstanding runs). */
void vsbpp_plan_destroy(vsbpp_plan* plan);

/* Best of a batch: writes d_out[0] = min cost and d_out[1] = the lowest index
 * reaching it over d_cost[0..num-1] (device pointers, asynchronous on
 * hip_stream).  Used to keep the best of several orderings of one instance. */
int32_t vsbpp_best_of(const int64_t* d_cost, int32_t num, int64_t* d_out, void* hip_stream);

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
