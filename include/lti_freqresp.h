/*
 * lti_freqresp.h -- C ABI of the MI355X frequency-response engine.
 *
 * Problem (the definition every entry point follows): for a continuous-time
 * LTI state-space model  x' = A x + B u,  y = C x + D u  with nx states,
 * nu inputs and ny outputs, evaluate the transfer matrix on the imaginary
 * axis
 *
 *        G(j w_k) = C (j w_k I - A)^{-1} B + D ,   k = 0 .. n_omega-1 ,
 *
 * (Kailath, *Linear Systems*, 1980, ch. 2).  The method: one Householder
 * reduction H = Q^T A Q to upper Hessenberg form per model (Golub & Van
 * Loan, *Matrix Computations*, 4th ed., sec. 7.4.3), after which every
 * frequency costs one shifted Hessenberg solve (Laub, "Efficient
 * multivariable frequency response computations", IEEE TAC 26(2), 1981):
 *
 *        G(j w) = (C Q) (j w I - H)^{-1} (Q^T B) + D .
 *
 * The shifted solve is done with Givens rotations (one unitary column
 * rotation per subdiagonal entry) fused with column back-substitution.
 * Two precisions exist: plain float64, and complex-float32 solves with
 * float64 residual-based iterative refinement (Higham, *Accuracy and
 * Stability of Numerical Algorithms*, 2nd ed., ch. 12).  Points whose
 * refinement stalls, and float64 points whose estimated error exceeds the
 * request's tolerance, are refined once more with the residual of the
 * original (A, B) in double-double arithmetic (Higham, sec. 12.1), since
 * near an eigenvalue the rounding of the reduction itself dominates.
 * With fewer outputs than inputs the transposed system (A^T, C^T, B^T, D^T)
 * is solved (G^T = B^T (s I - A^T)^{-1} C^T + D^T), so every solve has
 * min(nu, ny) right-hand sides.  The same solves evaluate G at any complex
 * point s (request.points), including the discrete-time z = exp(j theta).
 *
 * Serving model: a context owns a scheduler thread.  submit() copies a
 * request's host inputs and returns at once; the scheduler admits requests
 * as arena memory allows, reduces each model once (reduced models with a
 * nonzero model_key stay resident for repeat queries), and batches the
 * per-frequency solves of all live requests into shared kernel launches.
 * poll() collects a finished request.
 *
 * Conventions for every entry point:
 *   - All matrices are float64, row-major, densely packed.
 *   - Complex outputs are interleaved (re, im) float64 pairs.
 *   - Functions return 0 (LTI_OK) on success, LTI_PENDING (> 0) where
 *     documented, and a negative LTI_E* code on error.  Nothing throws or
 *     aborts across this boundary.
 *   - One internal mutex per context; every call may come from any thread.
 */
#ifndef LTI_FREQRESP_H
#define LTI_FREQRESP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LTI_ABI_VERSION 4u

/* ---------------------------------------------------------------- codes */
#define LTI_OK            0
#define LTI_PENDING       1   /* poll(): request not finished yet          */
#define LTI_EINVAL      (-1)  /* bad argument: NULL, dims <= 0, non-finite  */
#define LTI_ENOSPC      (-2)  /* request can never fit in the arena budget  */
#define LTI_EAGAIN      (-3)  /* pending queue full; retry after a poll()   */
#define LTI_ENOENT      (-4)  /* unknown or already collected id / key      */
#define LTI_EDEVICE     (-5)  /* HIP error; the context is unusable         */
#define LTI_ENOMEM      (-6)  /* host allocation failed                     */
#define LTI_EUNSUPPORTED (-7) /* dimensions outside what the kernels cover  */

/* request.precision */
#define LTI_PREC_FP64     0   /* float64 Givens solve per frequency          */
#define LTI_PREC_REFINED  1   /* complex-float32 solves + float64 refinement */

/* request.mem */
#define LTI_MEM_HOST      0   /* A,B,C,D,omega,G_out,info_out are host memory   */
#define LTI_MEM_DEVICE    1   /* ... are device memory on the context's device */

/* lti_point_info.path */
#define LTI_PATH_FP64      0  /* plain float64 solve                          */
#define LTI_PATH_REFINED   1  /* float32 solves, float64 refinement converged  */
#define LTI_PATH_FALLBACK  2  /* refinement stalled; float64 solve used        */
#define LTI_PATH_SINGULAR  3  /* j w I - A singular to working precision       */
#define LTI_PATH_FP64_DD   4  /* float64 solve, then double-double residual
                                 refinement against A (estimated error
                                 > rtol / 4)                                  */

/* request.points: what omega holds */
#define LTI_POINTS_JW     0   /* real frequencies w_k in rad/s: s_k = j w_k            */
#define LTI_POINTS_S      1   /* complex points: omega[2k] + j omega[2k+1] = s_k       */
#define LTI_POINTS_Z      2   /* discrete time: theta_k = w_k T in rad/sample,
                                 z_k = exp(j theta_k); the solves use s_k = z_k     */

/* config.flags */
#define LTI_CFG_KERNEL_TIMING 1u  /* bracket every kernel launch with HIP events */
#define LTI_CFG_FORCE_DD      2u  /* testing: every point takes the double-double
                                     refinement (path FALLBACK / FP64_DD)        */
#define LTI_CFG_NO_TRANSPOSE  4u  /* never solve the transposed system           */

/* Per-frequency result information, 8 bytes. */
typedef struct lti_point_info {
  float   est_rel_err;  /* estimated relative error of G(j w_k) (see below) */
  uint8_t iters;        /* float32 solves used (refined path); 1 for fp64   */
  uint8_t path;         /* LTI_PATH_*                                        */
  uint16_t reserved;
} lti_point_info;
/* est_rel_err: for LTI_PATH_REFINED the predicted error after the last
 * correction, min(||dX|| / ||X||, (||dX|| / ||X||) * contraction); for
 * LTI_PATH_FP64 (u/2) sqrt(nx) max|R(k,k)| / min|R(k,k)|, u the float64
 * unit roundoff and R the triangular factor of the shifted solve (the
 * diagonal spread alone underestimates kappa by about sqrt(nx) on isolated
 * resonances); for LTI_PATH_FALLBACK / _FP64_DD the last
 * correction norm ||dx|| / ||x|| of the double-double refinement.
 * iters: float32 solves (refined), plus float64 solves for _FALLBACK and
 * _FP64_DD.  With the columns of one point split over several kernel tiles,
 * the record is merged: the largest estimate and the worst path. */

/* Create-time configuration. */
typedef struct lti_config {
  uint32_t abi_version;   /* must equal LTI_ABI_VERSION                          */
  int32_t  device;        /* HIP device ordinal                                  */
  void*    arena;         /* caller-owned device memory, 256-byte aligned; the
                             library sub-allocates inside it and never frees it */
  size_t   arena_bytes;   /* size of the arena = the HBM budget                  */
  void*    stream;        /* hipStream_t to launch on (must stay valid until
                             destroy); NULL: the library creates its own        */
  int32_t  max_pending;   /* bound on submitted, not yet collected requests;
                             <= 0 selects 8192                                   */
  uint32_t flags;         /* LTI_CFG_*                                            */
  int32_t  tile_points;   /* frequencies per wave tile; 0 = automatic            */
  int32_t  max_batch_tiles; /* tiles per kernel launch; 0 = automatic            */
  size_t   host_staging_bytes; /* pinned host staging for host-memory requests;
                                  0 selects 256 MiB.  Requests that do not fit
                                  fall back to (slower) pageable copies         */
} lti_config;

/* One request: one model evaluated on one frequency grid. */
typedef struct lti_request {
  int32_t nx, nu, ny;     /* n >= 1, m >= 1, p >= 1                              */
  int32_t mem;            /* LTI_MEM_HOST or LTI_MEM_DEVICE                      */
  const double* A;        /* nx*nx                                               */
  const double* B;        /* nx*nu                                               */
  const double* C;        /* ny*nx                                               */
  const double* D;        /* ny*nu; NULL means D = 0                             */
  const double* omega;    /* n_omega frequencies in rad/s, any finite value      */
  int64_t  n_omega;       /* >= 1                                                */
  int32_t  precision;     /* LTI_PREC_*                                          */
  int32_t  points;        /* LTI_POINTS_*: how omega is read (n_omega points;
                             LTI_POINTS_S: 2 * n_omega doubles)                  */
  double   rtol;          /* error target, <= 0 selects 1e-10.  Refined path:
                             stop when the predicted ||dX||/||X|| <= rtol / 10.
                             Float64 path: points whose estimated error exceeds
                             rtol / 4 are refined against A in double-double  */
  uint64_t model_key;     /* 0: no reuse.  Otherwise the reduced model stays
                             resident and later requests with the same key,
                             dimensions and (host memory) content reuse it     */
  double*  G_out;         /* n_omega*ny*nu complex = 2*n_omega*ny*nu doubles,
                             layout [k][i][j] (re, im)                           */
  lti_point_info* info_out; /* optional, n_omega entries                          */
  double*  dG_out;        /* optional: the derivative dG/ds = -C (s I - A)^{-2} B
                             at each point, same layout as G_out (on the
                             imaginary axis dG/dw = j dG/ds).  A request with
                             dG_out runs the float64 path whatever its
                             precision says                                     */
  const double* E;        /* optional: a descriptor system E x' = A x + B u
                             (nx*nx, may be singular); then
                             G(s) = C (s E - A)^{-1} B + D, computed by a
                             Hessenberg-triangular reduction Q^T A Z = H,
                             Q^T E Z = T (Golub & Van Loan, 4th ed., Alg.
                             7.7.1) and one solve with s T - H per point, on
                             the float64 path (no double-double refinement;
                             est_rel_err states the estimate).  nx <= 256, no
                             dG_out.  NULL: E = I                               */
} lti_request;
/* Ownership: with LTI_MEM_HOST, submit() copies A, B, C, D and omega before
 * it returns; G_out and info_out must stay valid until poll() reports the
 * request done (or until destroy()).  With LTI_MEM_DEVICE nothing is copied:
 * every pointer must stay valid and unmodified until the request is done,
 * and inputs are not checked for finiteness. */

/* Result of a finished request (filled by poll()). */
typedef struct lti_result {
  int32_t status;           /* LTI_OK, or the error that ended the request   */
  int32_t reduction_reused; /* 1 when a resident reduced model was reused    */
  int64_t n_points;
  int64_t n_refined, n_fallback, n_singular, n_fp64_dd;  /* points per path  */
  double  max_est_rel_err;
  double  t_submit_us;      /* microseconds since the context was created    */
  double  t_admit_us;
  double  t_first_launch_us;
  double  t_done_us;        /* results visible to poll()                     */
} lti_result;

/* Kernel families, for the per-family timing of lti_stats. */
#define LTI_KF_SWEEP4     0  /* four frequencies per wavefront (nx <= 64)       */
#define LTI_KF_SWEEP1     1  /* one frequency per wavefront (nx <= 256)          */
#define LTI_KF_SWEEPWG    2  /* one frequency per workgroup (nx <= 1024)         */
#define LTI_KF_REFINE_DD  3  /* double-double refinement of queued points       */
#define LTI_KF_SWEEPDESC  4  /* descriptor systems (one frequency per wavefront) */
#define LTI_KF_SWEEP2     5  /* two frequencies per wavefront (64 < nx <= 128)   */
#define LTI_KF_COUNT      6

/* Counters of one context. */
typedef struct lti_stats {
  uint64_t requests_submitted, requests_done, requests_failed;
  uint64_t reductions, reduction_cache_hits;
  uint64_t sweep_launches, tiles_launched, points_done;
  uint64_t arena_bytes_in_use, arena_peak_bytes;
  /* with LTI_CFG_KERNEL_TIMING: summed HIP-event durations (events on the
     stream the kernels run on).  sweep_kernel_ms covers the sweep families
     of every batch (timed_sweep_launches batches); family_ms[f] the
     launches of family f, bracketed per batch (family_launches[f]). */
  double   sweep_kernel_ms;
  double   reduce_kernel_ms;
  uint64_t timed_sweep_launches, timed_reduce_launches;
  double   family_ms[LTI_KF_COUNT];
  uint64_t family_launches[LTI_KF_COUNT];
} lti_stats;

typedef struct lti_ctx lti_ctx;

/* Create a context on config->device.  Validates the config (abi_version,
 * non-NULL arena of at least 1 MiB, 256-byte alignment), creates the stream
 * if none is given, and starts the scheduler thread.
 * Returns LTI_OK and *out, or LTI_EINVAL / LTI_EDEVICE / LTI_ENOMEM. */
int lti_freqresp_create(const lti_config* config, lti_ctx** out);

/* Queue one request and return without waiting for the GPU.  When the
 * request can start at once, its first kernels are launched from the calling
 * thread (on the context's stream) before submit returns.
 * LTI_EINVAL: NULL pointers, dims <= 0, n_omega <= 0, unknown precision or
 *             mem, non-finite host input.
 * LTI_EUNSUPPORTED: nx > 1024, or nu or ny > 16, or n_omega * nu > 2^32 - 1.
 * LTI_ENOSPC: the request alone needs more than the whole arena.
 * LTI_EAGAIN: max_pending requests are outstanding.
 * LTI_EDEVICE: the context saw a HIP error.
 * On LTI_OK, *out_id identifies the request for poll(). */
int lti_freqresp_submit(lti_ctx* ctx, const lti_request* req, uint64_t* out_id);

/* Wait up to timeout_us microseconds (< 0: forever, 0: do not wait) for
 * request id.  Returns LTI_OK with *out filled once the request is done (the
 * id is then collected: a second poll gives LTI_ENOENT), LTI_PENDING if it is
 * still running, LTI_ENOENT for an unknown id, or the request's own error
 * (also reported in out->status) if it failed.  A waiting poll drives the
 * scheduling itself (retire, admit, launch) for up to 2 ms before it sleeps
 * on the completion signal. */
int lti_freqresp_poll(lti_ctx* ctx, uint64_t id, int32_t timeout_us, lti_result* out);

/* Stop the scheduler, wait for the device work already launched, release
 * every sub-allocation and the context.  Requests not yet collected are
 * dropped; their output buffers may be partly written.  The arena itself is
 * not freed (it belongs to the caller). */
int lti_freqresp_destroy(lti_ctx* ctx);

/* Copy the resident reduced model of (model_key, nx, nu, ny) to host memory:
 * H (nx*nx, upper Hessenberg, zeros below the subdiagonal), Bt = Q^T B
 * (nx*nu) and Ct = C Q (ny*nx), all row-major float64.  Any of the three
 * pointers may be NULL.  Waits for the reduction to finish.
 * Returns LTI_ENOENT if no such model is resident. */
int lti_freqresp_get_reduced(lti_ctx* ctx, uint64_t model_key, int32_t nx, int32_t nu,
                             int32_t ny, double* H, double* Bt, double* Ct);

/* A resonance peak: frequency (rad/s) and gain sigma_max(G(j w)). */
typedef struct lti_peak {
  double w;
  double gain;
} lti_peak;

typedef struct lti_hinf_result {
  double  hinf;         /* estimate of ||G||_inf = sup_w sigma_max(G(j w))     */
  double  w_hinf;       /* where it is attained (INFINITY: the D term)         */
  int32_t n_peaks;      /* refined local maxima written to peaks_out            */
  int32_t evaluations;  /* frequency points evaluated in all                    */
} lti_hinf_result;

/* Resonance peaks and the H-infinity norm estimate of the model in `req`
 * (LTI_MEM_HOST, LTI_POINTS_JW; omega is the starting grid, any order).
 * sigma(w) = sigma_max(G(j w)) and d sigma / d w = Re(u1^H (dG/dw) v1) (a
 * simple largest singular value's first-order perturbation) come from G and
 * dG/ds evaluated through `ctx` on the float64 path; every interior local
 * maximum of sigma on the grid (the max_peaks largest) is bracketed by its
 * grid neighbours and refined by a safeguarded secant iteration on
 * d sigma / d w = 0 until the bracket is below wtol (relative; <= 0 selects
 * 1e-12).  hinf is the largest of the refined peaks, the grid values and
 * sigma_max(D) (w -> infinity).  Blocks until done (it submits and polls
 * requests itself; the reduced model stays resident between them).  peaks_out
 * receives n_peaks entries, largest gain first.
 * Returns LTI_OK, LTI_EINVAL, or the error of an underlying submit/poll. */
int lti_freqresp_peaks(lti_ctx* ctx, const lti_request* req, int32_t max_peaks, double wtol,
                       lti_peak* peaks_out, lti_hinf_result* out);

/* Evaluation without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid
 * hipMalloc): the work of submit() + poll() for one LTI_MEM_DEVICE request,
 * enqueued on `stream` (a hipStream_t of `device`; NULL = the null stream)
 * with no context.  Nothing is allocated: the reduced model, the reduction's
 * working matrix, the refinement queue and (when info_out is NULL) the point
 * records live in one fixed device array of 8 MiB inside the library, one
 * copy per device, held until the process ends.  The same kernels as the
 * context path run, tiled as an idle context would tile the request, so G
 * equals a context's result for the same request alone.
 * Limits: nx <= 256, nu, ny <= 16, n_omega <= 2^18 and
 * n_omega * min(nu, ny) <= 2^18, no descriptor E; beyond them
 * LTI_EUNSUPPORTED.  Returns
 * LTI_OK once the work is enqueued: G_out, info_out and dG_out are written
 * when the stream reaches it (synchronise the stream before reading them);
 * nothing is reduced or kept for reuse.  LTI_EINVAL for a host-memory
 * request or bad arguments, LTI_EDEVICE for a HIP error.  Calls that overlap
 * on one device -- on different streams or threads, or before an earlier
 * call's work has finished on another stream -- race on the shared array:
 * serialise them (one stream per device). */
int lti_freqresp_eval_noalloc(int32_t device, const lti_request* req, void* stream);

/* Snapshot of the context's counters. */
int lti_freqresp_stats(lti_ctx* ctx, lti_stats* out);

/* Static description of a return code; never NULL. */
const char* lti_freqresp_strerror(int code);

/* LTI_ABI_VERSION of the loaded library. */
uint32_t lti_freqresp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LTI_FREQRESP_H */
