/*
 * Sequential CPU oracle for the VSBPP placement heuristics of
 * "Heuristics for the Variable Sized Bin Packing Problem Using a Hybrid
 * P System and CUDA Architecture" (Alenezi, Aboelfotoh, Albdaiwi, Almulla).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; it
 * shares no source, header or table with it.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Problem (Section 1, "Formal Definition of VSBPP"; Section 6.1): n bin types
 * with capacities B_1 > ... > B_n > 0 in unlimited supply, indivisible items
 * w_1..w_m with max w <= B_1; minimise the total capacity of the used bins.
 * All packing arithmetic is integer.
 *
 * Type indices are 0-based: type 0 is B_1 (the largest capacity).
 */
#ifndef VSBPP_ORACLE_H
#define VSBPP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* heuristics: plain First/Best/Worst Fit (Section 1) and the two hybrid
 * P-system heuristics (Sections 6.3 and 6.4) */
enum { ORC_FF = 0, ORC_BF = 1, ORC_WF = 2, ORC_H1 = 3, ORC_H2 = 4 };
/* rule for the type of a newly opened bin when no open bin fits */
enum { ORC_TYPE_SMALLEST_FIT = 0, ORC_TYPE_LARGEST = 1, ORC_TYPE_LEARNED = 2 };

/* Learned bin-type scorer: MLP 16 -> 64 -> 64 -> n_out with ReLU, weights in
 * bfloat16 (raw 16-bit patterns), biases in fp32, row-major [out][in]. */
#define ORC_NFEAT 16
#define ORC_HIDDEN 64
#define ORC_MAX_OUT 16
typedef struct {
  int32_t n_out;
  uint16_t w1[ORC_HIDDEN * ORC_NFEAT];
  float b1[ORC_HIDDEN];
  uint16_t w2[ORC_HIDDEN * ORC_HIDDEN];
  float b2[ORC_HIDDEN];
  uint16_t w3[ORC_MAX_OUT * ORC_HIDDEN];
  float b3[ORC_MAX_OUT];
} orc_model;

/* one decision of a run: an item that fits no open bin in a plain FF/BF/WF
 * run (chosen = type opened, plain_type = the base rule's type, feasible =
 * types holding the item), or a placement of the first heuristic where the
 * three criteria pick different bins under the learned criterion rule
 * (chosen = criterion used, plain_type = Rule 3's draw, feasible = 7), or a
 * contested placement of a plain run under a choice rule (chosen = 1 when a
 * new bin opened, else 0; plain_type = 0; feasible = 3) */
typedef struct {
  int32_t position;   /* position of the item in processing order      */
  int32_t weight;
  int32_t plain_type; /* type the base rule would open                  */
  int32_t chosen;     /* type actually opened                           */
  uint32_t feasible;  /* bit k set when B_k >= weight                   */
  float feat[ORC_NFEAT];
} orc_decision;
enum { ORC_OK = 0, ORC_E_NULL = -1, ORC_E_SIZE = -2, ORC_E_CAPS = -3,
       ORC_E_WEIGHT = -4, ORC_E_HEURISTIC = -5, ORC_E_OPTION = -6 };

typedef struct {
  uint64_t seed;          /* key of the counter-based generator            */
  int32_t s1;             /* H1 items per sublist (Table 1: 10)            */
  int32_t s2;             /* H2 subset size (Tables 1, 4, 6: 5)            */
  int32_t type_rule;      /* ORC_TYPE_*                                    */
  int32_t force_crit;     /* -1: drawn per placement; else ORC_FF/BF/WF    */
  const int32_t* order;   /* optional: order[q] = item at position q       */
  const orc_model* model; /* ORC_TYPE_LEARNED: the scorer                  */
  int32_t force_event;    /* plain heuristics: decision number d whose type
                             is forced (-1: none)                          */
  int32_t force_t1;       /* type forced at decision d                     */
  int32_t force_t2;       /* type forced at decision d + 1                 */
  orc_decision* trace;    /* optional: receives the run's decisions        */
  int32_t trace_cap;      /* capacity of trace                             */
  int32_t* trace_count;   /* number of decisions of the run                */
  int32_t active_limit;   /* plain FF/BF/WF: at most this many bins open at
                             once (0: no limit); see run_plain               */
  int32_t downsize;       /* 1: after packing, every bin takes the smallest
                             type that holds its load (see downsize_bins)   */
  int32_t criterion_rule; /* H1 only: 0 = Rule 3's draw; 1 = the model (n_out
                             >= 3) picks FF/BF/WF where they differ (see
                             h1_learned_criterion); needs force_crit = -1  */
  int32_t choice_rule;    /* plain FF/BF/WF with type_rule LARGEST and
                             downsize 1 only (see plain_choice): 0 = the
                             criterion's bin always; 1 = the same, but the
                             run's decisions are its contested placements
                             (forcing and the trace index those); 2 = the
                             model (n_out >= 2) chooses at each contested
                             placement between the criterion's bin (output
                             0) and a new bin (output 1)                    */
  int32_t rule2_order;    /* H1/H2: order of Rule 2's empty bins in the
                             packer, 0 = B_1 first (type order), 1 = B_n
                             first (increasing capacity); plain: must be 0  */
} orc_opts;

typedef struct {
  int64_t packers;        /* H1 sublists / H2 subsets / 1 for plain        */
  int64_t perm_packings;  /* H2: permutations packed (sum of k!)           */
  int64_t placements;     /* item placements performed                     */
  int64_t bin_tests;      /* open bins visited by fit tests                */
  int64_t live_tests;     /* open bins that could still take any item      */
  int64_t new_bins;       /* bins opened because nothing fitted            */
  int64_t divisions;      /* Rule-5 divisions                              */
} orc_stats;

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the k-th output (k >= 0)
 * of the generator whose state starts at `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);
/* derived per-purpose key: output `stream` of the generator at `seed` */
uint64_t orc_stream_key(uint64_t seed, uint64_t stream);
/* criterion draw in {0,1,2} = {FF,BF,WF} with equal probabilities */
int32_t orc_criterion(uint64_t stream_key, uint64_t counter);
int32_t orc_criterion_digit(uint64_t stream_key, uint64_t counter, int32_t t);
/* pseudo-random permutation of [0,m): the item at position q (Rule 1) */
int32_t orc_perm(uint64_t seed, int32_t m, int32_t q);

/* Runs one heuristic on one instance.  assign[m] receives a bin id per item,
 * types[m] the type index of bins 0..nbins-1.  Returns nbins (>= 1) or a
 * negative ORC_E_* code; nothing is written on error.  stats may be NULL. */
int32_t orc_pack(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                 int32_t heuristic, const orc_opts* opt, int32_t* assign,
                 int32_t* types, int64_t* cost, orc_stats* stats);

/* One packer of the hybrid P system with explicit per-placement criteria:
 * Rule-2 bins (one empty bin per type: B_1 first when rule2 == 1, B_n first
 * when rule2 == 2) when rule2 != 0, Rule-5 division when rule5 != 0.  Items are placed in the given order.  Same outputs as
 * orc_pack (used bins only, creation order). */
int32_t orc_pack_packer(const int32_t* w, int32_t m, const int32_t* caps,
                        int32_t n, const int32_t* crit, int32_t rule2,
                        int32_t rule5, int32_t type_rule, int32_t* assign,
                        int32_t* types, int64_t* cost);

/* Scorer forward pass: z[0..n_out) from x[16] (fp32, fused multiply-add
 * chains in index order). */
void orc_mlp_forward(const orc_model* mdl, const float* x, float* z);

/* Depth-2 lookahead label of decision d of a plain run with criterion crit:
 * for every feasible type k1 at d, V(k1) = min over k2 of the cost of the
 * run with k1 forced at d and k2 at d+1 (the base rule elsewhere); the label
 * is argmin V, ties to the base rule's own choice, else the lowest type.
 * values[n] receives V (-1 for infeasible types).  Returns the label or a
 * negative code. */
int32_t orc_rollout_label(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                          int32_t crit, int32_t d, int64_t* values);
/* The same with the base rule's type rule (ORC_TYPE_SMALLEST_FIT or
 * ORC_TYPE_LARGEST) and every run's cost taken after the downsizing pass
 * when downsize is 1. */
int32_t orc_rollout_label_ex(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                             int32_t crit, int32_t d, int32_t type_rule, int32_t downsize,
                             int64_t* values);

/* Depth-2 lookahead label of contested placement d of a plain run with
 * criterion crit under the largest type rule with downsizing: for k1 in
 * {0 = the criterion's bin, 1 = a new bin}, V(k1) = min over k2 of the
 * downsized cost of the run with k1 at d and k2 at d+1 (the criterion's bin
 * elsewhere); the label is argmin V, 0 on ties.  values[2] receives V.
 * Returns the label, ORC_E_OPTION when the run has fewer than d+1 contested
 * placements, or another negative code. */
int32_t orc_choice_label(const int32_t* w, int32_t m, const int32_t* caps, int32_t n,
                         int32_t crit, int32_t d, int64_t* values);

/* lower bounds on the optimum */
int64_t orc_lb_sum(const int32_t* w, int32_t m);
int64_t orc_lb_cap(const int32_t* w, int32_t m, const int32_t* caps, int32_t n);
int64_t orc_lb_big(const int32_t* w, int32_t m, const int32_t* caps, int32_t n);

/* exact optimum, two independent methods (m <= 12) */
int64_t orc_opt_partitions(const int32_t* w, int32_t m, const int32_t* caps, int32_t n);
int64_t orc_opt_subset_dp(const int32_t* w, int32_t m, const int32_t* caps, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
