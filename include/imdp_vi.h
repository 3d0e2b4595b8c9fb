/*
 * imdp_vi.h -- C ABI of robust value iteration for interval Markov decision
 * processes (IMDPs) on one MI355X.
 *
 * Problem (the paper's section 2): an IMDP has states S, actions A(s) per
 * state, and for every state-action pair (s, a) and destination s' an
 * interval [lower(s,a,s'), upper(s,a,s')] for the transition probability,
 * with sum lower <= 1 <= sum upper.  Robust value iteration (its Eq. 2)
 * computes, for k = 1 .. K,
 *
 *     V_k(s) = opt_a  opt_{p in Gamma_{s,a}}  sum_{s'} p(s') V_{k-1}(s'),
 *
 * with the goal states held at 1 (reachability), or V_k = r + gamma * (...)
 * (discounted reward).  The inner problem (its Eq. 3) is solved by
 * O-maximization (its section 4): order the destinations by V_{k-1}
 * (ascending when the adversary minimises, descending when it maximises),
 * start from the lower bounds and hand the remaining mass 1 - sum lower to
 * the destinations in that order, each up to its upper bound.
 *
 * The value of that distribution depends on the ordering only through the
 * destination at which the remaining mass runs out (the threshold): every
 * destination before it gets its full gap, the threshold gets the rest.  The
 * GPU finds the threshold by bisection over order-preserving keys of V,
 * starting from the previous iteration's threshold, instead of sorting.
 *
 * Conventions: functions return 0 (IMDP_OK) or a negative IMDP_E* code;
 * nothing throws or aborts across this boundary.  Not thread-safe per
 * handle: one caller at a time.
 */
#ifndef IMDP_VI_H
#define IMDP_VI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IMDP_OK            0
#define IMDP_EINVAL      (-1)  /* bad argument: NULL, sizes, indices, bounds  */
#define IMDP_EDEVICE     (-5)  /* HIP error                                    */
#define IMDP_ENOMEM      (-6)  /* host or device allocation failed             */
#define IMDP_EUNSUPPORTED (-7) /* more than 2^31 - 1 transitions or columns   */

/* imdp_spec.property */
#define IMDP_REACH        0   /* reach the target set                          */
#define IMDP_REACH_AVOID  1   /* reach the targets, never entering avoid states */
#define IMDP_REWARD       2   /* discounted cumulative reward                   */

/* The model, in compressed sparse columns with one column per state-action
 * pair (host memory; copied by imdp_vi_create, which the caller may free
 * afterwards).  The columns of state s are stateptr[s] .. stateptr[s+1]-1
 * (the action index of column j is j - stateptr[s]); column j holds the
 * destinations rowval[colptr[j] .. colptr[j+1]-1] with bounds lower[.] and
 * upper[.].  Requirements: stateptr and colptr non-decreasing from 0 to
 * n_columns and nnz; 0 <= rowval < n_states; 0 <= lower <= upper <= 1,
 * finite.  A state with no column gets value 0 (reward: r(s)). */
typedef struct imdp_model {
  int32_t n_states;
  int32_t n_columns;
  int64_t nnz;
  const int32_t* stateptr;  /* n_states + 1  */
  const int32_t* colptr;    /* n_columns + 1 */
  const int32_t* rowval;    /* nnz           */
  const double* lower;      /* nnz           */
  const double* upper;      /* nnz           */
} imdp_model;

/* What to compute (the paper's section 3.2). */
typedef struct imdp_spec {
  int32_t property;        /* IMDP_REACH, IMDP_REACH_AVOID, IMDP_REWARD           */
  int32_t horizon;         /* > 0: K iterations; 0: until the residual < eps     */
  double  eps;             /* infinite horizon: max_s |V_k - V_{k-1}| < eps      */
  int32_t max_iterations;  /* infinite horizon bound; <= 0 selects 100000        */
  int32_t pessimistic;     /* 1: the adversary minimises; 0: it maximises        */
  int32_t maximize;        /* 1: the strategy maximises; 0: it minimises         */
  const int32_t* targets;  /* reachability goal states (host memory)             */
  int32_t n_targets;
  const int32_t* avoid;    /* IMDP_REACH_AVOID: states held at 0 (a state in both
                              sets counts as a target)                          */
  int32_t n_avoid;
  const double* reward;    /* IMDP_REWARD: r(s), n_states entries; V_0 = r       */
  double  discount;        /* IMDP_REWARD: gamma in [0, 1]                        */
} imdp_spec;

typedef struct imdp_result {
  int32_t iterations;      /* iterations performed                                 */
  double  residual;        /* max_s |V_k - V_{k-1}| of the last iteration          */
  double  kernel_ms;       /* device time of the iterations (HIP events)           */
} imdp_result;

typedef struct imdp_vi imdp_vi;

/* Validate the model and copy it to `device` (rowval, lower and the gaps
 * upper - lower, plus per-column 1 - sum lower and sum of gaps).  Returns
 * IMDP_OK and *out, IMDP_EINVAL, IMDP_EUNSUPPORTED, IMDP_ENOMEM or
 * IMDP_EDEVICE. */
int imdp_vi_create(int32_t device, const imdp_model* model, imdp_vi** out);

/* Run value iteration (blocking).  V_out (host, n_states doubles) receives
 * V_K.  policy_out (host, optional): for a finite horizon n_states * horizon
 * int32 entries, policy_out[s * horizon + t] = the action to take in state s
 * at time t = 0 .. K-1 (the optimiser of iteration K - t); for an infinite
 * horizon n_states entries, the optimiser of the last iteration.  Ties
 * between actions go to the lowest action index.  out (optional) receives
 * the iteration count and last residual.
 * Returns IMDP_OK, IMDP_EINVAL (bad spec) or IMDP_EDEVICE. */
int imdp_vi_run(imdp_vi* h, const imdp_spec* spec, double* V_out, int32_t* policy_out, imdp_result* out);

/* Release the device copy of the model. */
int imdp_vi_destroy(imdp_vi* h);

#ifdef __cplusplus
}
#endif
#endif /* IMDP_VI_H */
