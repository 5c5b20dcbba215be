/*
 * parapn -- parallel-in-time probabilistic numerical ODE solver (ParaIEKS)
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Bosch, Corenflos, Yaghoobi, Tronarp, Hennig, Saerkkae,
 * "Parallel-in-Time Probabilistic Numerical ODE Solvers", JMLR 25 (2024).
 *
 * Plain C ABI.  Pointers marked "device" are HIP device pointers (any memory
 * the GPU can address, e.g. torch tensor storage); pointers marked "host" are
 * ordinary host memory read during the call.  Matrices are dense row-major.
 * The state ordering is the Kronecker order of Sec. 2.1: index
 * k = i*(q+1) + j holds derivative j of ODE component i, D = d*(q+1).
 * Square-root factors are lower-triangular ("left square roots", Sec. 3.1.2).
 * Floating-point device buffers have the element type of the precision
 * argument: double for PARAPN_FP64, float for PARAPN_FP32_SQRT.
 *
 * Every function returns a status code (PARAPN_OK = 0 on success).  A
 * negative status leaves a message in parapn_last_error() (thread-local);
 * output buffers are then unspecified.  No exception crosses the boundary.
 * All GPU work is queued on the caller's stream (a hipStream_t passed as
 * void*, NULL = the default stream).
 */
#ifndef PARAPN_H
#define PARAPN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PARAPN_OK 0          /* done; for a solve: the stopping criterion was met   */
#define PARAPN_MAXITER 1     /* solve hit max_iter; the returned result is valid     */
#define PARAPN_EINVAL (-1)   /* bad argument (unknown field, d/q/N out of range, ..) */
#define PARAPN_ENOMEM (-2)   /* device memory or the context budget is exhausted    */
#define PARAPN_EDEVICE (-3)  /* HIP runtime error                                   */
#define PARAPN_ENONFINITE (-4) /* NaN/Inf in the iterate; outputs hold the last one  */

/* priors */
#define PARAPN_PRIOR_IWP 0
#define PARAPN_PRIOR_IOUP 1
#define PARAPN_PRIOR_MATERN 2

/* starting trajectory (parapn_problem.init_mode; a given init_traj overrides it) */
#define PARAPN_INIT_CONSTANT 0 /* eta_n = mu0 for every n (Alg. 2)                         */
#define PARAPN_INIT_COARSE 1   /* sequential extended Kalman smoother on a coarse grid,
                                * bridged to the fine grid by the prior (the alternative
                                * start of the remark on initial trajectories, Sec. 3.2.2) */

/* which start a solve used (parapn_info.start) */
#define PARAPN_START_CONSTANT 0
#define PARAPN_START_COARSE 1
#define PARAPN_START_GIVEN 2
#define PARAPN_START_COARSE_FAILED 3 /* the coarse smoother produced a non-finite value; the
                                      * solve ran from the constant start instead          */

/* Jacobian used by the linearisation (parapn_problem.linearization; the
 * remark on linearizing with approximate Jacobians, Sec. 3.2.1) */
#define PARAPN_LIN_EK1 0      /* the exact Jacobian F_y (first-order Taylor)           */
#define PARAPN_LIN_EK0 1      /* F_y ~ 0                                               */
#define PARAPN_LIN_DIAG_EK1 2 /* F_y ~ diag(F_y)                                       */

/* stopping criteria (parapn_problem.stop_rule) */
#define PARAPN_STOP_TRAJECTORY 1
#define PARAPN_STOP_OBJECTIVE 2

/* arithmetic of the path */
#define PARAPN_FP64 0      /* every step in double                                  */
#define PARAPN_FP32_SQRT 1 /* elements, scans and linearisation in float; the prior
                            * constants, the output unscaling and the convergence
                            * test in double (Sec. 2.4 preconditioned form)         */

/* Vector-field registry.  f is autonomous in every entry.
 * PARAPN_LOGISTIC        d=1  y' = y(1-y)                                     no params
 * PARAPN_FHN             d=2  V' = c(V - V^3/3 + R), R' = -(V - a + bR)/c     params a,b,c
 * PARAPN_LORENZ63        d=3  x' = s(y-x), y' = x(r-z)-y, z' = xy - b z      params s,r,b
 * PARAPN_LOTKA_VOLTERRA  d=2  x' = al x - be x y, y' = de x y - ga y          params al,be,ga,de
 * PARAPN_AFFINE          d    y' = L y + c                                    params L (d*d, row-major), c (d)
 * PARAPN_RIGID_BODY      d=3  y' = (-2 y2 y3, 1.25 y1 y3, -0.5 y1 y2)         no params
 * PARAPN_VAN_DER_POL     d=2  y' = (y2, mu((1-y1^2) y2 - y1))                 params mu
 * PARAPN_MOL_HEAT_REACTION  d>=3  method of lines for u_t = nu u_xx + u(1-u) on
 *                        d periodic grid points x_i = i/d:
 *                        y_i' = nu d^2 (y_{i-1} - 2 y_i + y_{i+1}) + y_i (1 - y_i)  params nu
 * The first three, the rigid body and Van der Pol follow the problems of the
 * experiments section and the workload list; the affine field is the exactly
 * solvable case of Sec. 3.1. */
#define PARAPN_LOGISTIC 0
#define PARAPN_FHN 1
#define PARAPN_LORENZ63 2
#define PARAPN_MOL_HEAT_REACTION 4
#define PARAPN_LOTKA_VOLTERRA 3
#define PARAPN_AFFINE 5
#define PARAPN_RIGID_BODY 6
#define PARAPN_VAN_DER_POL 7

/* limits of this build: 1 <= q <= 4; the fixed-size fields have 1 <= d <= 3,
 * D = d(q+1) <= 15 (one group of lanes per scan element); the method-of-lines
 * field has d >= 3 and D <= 256 (one workgroup per element, matrix-core
 * products and triangularisations) */
#define PARAPN_MAX_D 15
#define PARAPN_MAX_DENSE_D 256
#define PARAPN_MAX_PARAMS 16

typedef struct parapn_ctx parapn_ctx;

/* One initial value problem (eq. ivp) on the uniform grid t_n = t0 + n h,
 * h = (t1 - t0)/N, n = 0..N, solved with an IWP(q) prior (Sec. 2.1), exact
 * Taylor initialisation mu0 and Sigma0 = 0 (eq. mu0), EK1 linearisation
 * (Sec. 3.2.1) and the iterated smoother of Alg. 2. */
typedef struct {
    int32_t field;         /* PARAPN_* field id                                        */
    int32_t d;             /* ODE dimension (must match the field; free for AFFINE)    */
    const double *params;  /* host, n_params values (may be NULL when n_params == 0)   */
    int32_t n_params;
    const double *y0;      /* host, d values                                           */
    double t0, t1;         /* time span, t1 > t0                                       */
    int32_t q;             /* prior order, 1..4                                        */
    int64_t N;             /* number of steps, >= 1                                    */
    double tol;            /* stop when delta_k < tol (see parapn_solve)               */
    int32_t max_iter;      /* iteration cap, >= 1                                      */
    int32_t fixed_iters;   /* > 0: run exactly this many iterations, ignore tol        */
    int32_t precision;     /* PARAPN_FP64 or PARAPN_FP32_SQRT                          */
    const double *init_traj; /* [N+1][D] starting trajectory in original coordinates
                              * (row 0 is replaced by mu0), or NULL for the constant
                              * mu0 of Alg. 2                                       */
    int32_t init_on_device;  /* 0: init_traj is host memory; 1: device memory on the
                              * context's device (read on the solve's stream)       */
    double lm_sigma;         /* >= 0.  > 0: Levenberg-Marquardt damping of each Gauss-
                              * Newton step (the globalisation the paper leaves to
                              * future work): every step n >= 1 gets the pseudo-
                              * observation E0 Y_n = E0 (current iterate)_n with
                              * standard deviation lm_sigma / sqrt(h) in the units of
                              * y.  The fixed point is unchanged; the scans stay well
                              * conditioned at unstable iterates.  Factors
                              * (sqrtcov_out) then come from one more, undamped pass
                              * at the final iterate.  0: plain Alg. 2.             */
    int32_t prior;           /* PARAPN_PRIOR_IWP (0, Sec. 2.1), or one of the
                              * alternative Gauss-Markov priors of Sec. 2.1:
                              * PARAPN_PRIOR_IOUP, the q-th derivative an Ornstein-
                              * Uhlenbeck process dX_q = -prior_theta X_q dt + dW;
                              * PARAPN_PRIOR_MATERN, the Matern process of
                              * smoothness q + 1/2 and length scale prior_theta
                              * (drift polynomial (s + lambda)^(q+1), lambda =
                              * sqrt(2q+1) / prior_theta, unit diffusion).  Both are
                              * discretised in FP64 on the host (Van Loan).  Served
                              * requests must use the IWP prior.                   */
    double prior_theta;      /* IOUP: rate, finite and >= 0 (0 gives the IWP);
                              * Matern: length scale, finite and > 0              */
    int32_t init_mode;       /* PARAPN_INIT_CONSTANT or PARAPN_INIT_COARSE; used only
                              * when init_traj is NULL.  COARSE: a sequential EK1
                              * filter (linearised at each predicted mean) and RTS
                              * smoother on a grid of M coarse steps of s fine steps
                              * each, s = ceil(N / coarse_points), M = ceil(N / s)
                              * (the last coarse node may lie past t1), with the
                              * IWP(q) prior whatever `prior` says; every fine row is
                              * the prior's mean between its two smoothed coarse
                              * nodes.  Runs on the device in the path's precision
                              * (means in FP64).                                     */
    int32_t coarse_points;   /* target M of the coarse grid; 0 = max(1024, 64
                              * ceil(log2 N)); values above N mean N (s = 1: the
                              * sequential smoother on the fine grid itself)         */
    int32_t stop_rule;       /* stopping criteria of Sec. 3.2.2 (not with fixed_iters):
                              * PARAPN_STOP_TRAJECTORY (bit 0): delta_k below the
                              * threshold of parapn_solve; PARAPN_STOP_OBJECTIVE
                              * (bit 1): the change of the objective value
                              * V (eq. objective-value) since the previous iterate
                              * (the start for k = 1) at most obj_atol + obj_rtol |V_k|;
                              * with both bits either criterion stops.  0 = bit 0. */
    double obj_atol, obj_rtol; /* >= 0; the paper's experiments use 1e-9 and 1e-6  */
    int32_t calibrate;       /* 1: scale the returned factors (sqrtcov_out) by the
                              * quasi-maximum-likelihood diffusion sigma-hat of the
                              * final linearisation (Sec. 2.4); 0: sigma = 1        */
    int32_t linearization;   /* PARAPN_LIN_*: the Jacobian of every Gauss-Newton
                              * linearisation (the coarse-grid start always uses
                              * EK1).  A fixed point still satisfies the ODE at the
                              * grid points; the iteration converges more slowly
                              * (or not at all) when the dropped entries matter.
                              * For PARAPN_MOL_HEAT_REACTION with EK0 or DiagonalEK1
                              * the linearised model is block diagonal over the d
                              * grid points and the solve runs as d independent
                              * problems of state size q+1 (cost linear in d); its
                              * factors (sqrtcov_out) are block diagonal, and
                              * sigma-hat is available there as for the fixed-size
                              * fields (under EK1 the method-of-lines field reports
                              * V but not sigma-hat).                             */
} parapn_problem;

typedef struct {
    int32_t iterations;     /* linearise+smooth passes run (including the last one)   */
    int32_t converged;      /* 1 when the stopping test passed                        */
    double final_delta;     /* delta of the last pass                                 */
    double tol_used;        /* the threshold actually applied                         */
    double *delta_history;  /* host, max_iter entries, may be NULL                    */
    int32_t start;          /* PARAPN_START_*: the starting trajectory used           */
    double sigma_hat;       /* quasi-maximum-likelihood diffusion (Sec. 2.4) of the final
                             * linearisation: sqrt(sum_n r_n^T S_n^-1 r_n / (N d)) over
                             * the filter's innovations r_n (S_n their covariance at
                             * sigma = 1), accumulated in FP64 (not bitwise reproducible:
                             * atomic sums).  FP64 path: from the last filter pass (for
                             * damped solves from the undamped pass that sqrtcov_out
                             * triggers, else NaN).  FP32 path: from one FP64 filter pass
                             * at the final iterate that calibrate with sqrtcov_out
                             * triggers, else NaN (the FP32 innovations cancel at a
                             * converged iterate).  NaN for the method-of-lines field
                             * under EK1 (its dense engine forms no innovations).     */
    double objective;       /* V (eq. objective-value) of the returned trajectory, FP64 (in
                             * the FP32 path V of a trajectory carrying FP32 increments) */
    double *objective_history; /* host, max_iter entries (V after each iteration), may be NULL */
} parapn_info;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the context may hold (0 = no bound).  The context caches the
 * workspace between solves; it is not thread-safe (one context per thread). */
int parapn_create(parapn_ctx **ctx, int device, size_t hbm_budget_bytes);
void parapn_destroy(parapn_ctx *ctx);

/* Device workspace a solve of this problem needs, in bytes. */
int parapn_workspace_size(const parapn_problem *prob, size_t *bytes);

/* ParaIEKS, Alg. 2.
 * mean_out:    device [N+1][D], original coordinates; row 0 is mu0.
 * sqrtcov_out: device [N+1][D][D] lower-triangular factors of Sigma_n in
 *              original coordinates (row 0 is zero), or NULL.
 * The user-facing solution is E0 mu_n and E0 Sigma_n E0^T (the entries k with
 * k % (q+1) == 0).
 * Convergence test: delta_k = max_n max_i |E0 (mu_n^(k) - mu_n^(k-1))|_i in
 * original coordinates, accumulated in double; PARAPN_FP64 stops when
 * delta_k < tol, PARAPN_FP32_SQRT when delta_k < max(tol, 2^-20 max_n |E0 mu_n|).
 * Returns PARAPN_OK, PARAPN_MAXITER, or an error.  Synchronises the stream once
 * per iteration (8-byte read of delta_k). */
int parapn_solve(parapn_ctx *ctx, const parapn_problem *prob, void *mean_out, void *sqrtcov_out,
                 parapn_info *info, void *stream);

/* The starting trajectory a solve of this problem would use (init_traj,
 * init_mode, coarse_points), without iterating: traj_out is device
 * [N+1][D] FP64 in original coordinates (row 0 = mu0); *start (may be NULL)
 * receives the PARAPN_START_* code.  Fixed-size fields only.  Waits for the
 * stream before returning. */
int parapn_start_trajectory(parapn_ctx *ctx, const parapn_problem *prob, double *traj_out, int32_t *start,
                            void *stream);

/* Alg. 2 for `batch` instances of one problem that differ only in their
 * initial values: instance b starts from y0s + b*d (host, batch*d values;
 * prob->y0 is ignored).  Outputs are stacked: mean_out [batch][N+1][D],
 * sqrtcov_out [batch][N+1][D][D] or NULL, info [batch] (or NULL).  Each
 * instance stops on its own test and its result is the one parapn_solve gives
 * for it.  The method-of-lines field runs all instances in the same launches
 * (one workgroup per element operation of any instance); other fields are
 * solved one instance after another.  Returns PARAPN_ENONFINITE if any
 * instance turned non-finite, else PARAPN_MAXITER if any hit max_iter, else
 * PARAPN_OK; per-instance outcomes are in info. */
int parapn_solve_batch(parapn_ctx *ctx, const parapn_problem *prob, int32_t batch, const double *y0s,
                       void *mean_out, void *sqrtcov_out, parapn_info *info, void *stream);

/* ParaRTS, Alg. 1, on a linear model (eq. affine-estimation) with constant
 * transition:  Y0 ~ N(mu0, S0 S0^T),  Y_n = Phi Y_{n-1} + w_n, w_n ~ N(0, sqrtQ sqrtQ^T),
 * and noiseless affine observations H_n Y_n = dvec_n, n = 1..N.
 * Inputs (device): mu0 [D], sqrt_sigma0 [D][D], Phi [D][D], sqrtQ [D][D],
 * H [N][dobs][D], dvec [N][dobs].  1 <= dobs < D <= PARAPN_MAX_D.
 * Outputs (device): smoothed mean [N+1][D] and factors [N+1][D][D] (or NULL),
 * filtered mean [N+1][D] and factors [N+1][D][D] (either may be NULL); row 0
 * of the filtered outputs is (mu0, sqrt_sigma0), row 0 of the smoothed ones
 * is conditioned on all data. */
int parapn_pararts(parapn_ctx *ctx, int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                   const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                   void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out, void *stream);

/* ParaRTS (Alg. 1) on a time-varying linear model (eq. affine-estimation with
 * Phi_n, Q_n, e.g. a non-uniform time grid):  Y_n = Phi_n Y_{n-1} + w_n,
 * w_n ~ N(0, sqrtQ_n sqrtQ_n^T).  Phi and sqrtQ are device [N][D][D], step n
 * using entry n-1; every other argument, the outputs and the status as for
 * parapn_pararts.  The per-step matrices are copied once into the context's
 * workspace (in the kernels' padded row layout) and read by the forward
 * step kernels at every step. */
int parapn_pararts_tv(parapn_ctx *ctx, int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                      const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                      void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out,
                      void *stream);

/* ParaRTS as parapn_pararts, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, and no hipMalloc, hipFree or other allocating call.
 * Its scratch is one static device array per GPU of 64 MiB (held by the
 * library until the process ends), shared by every call on that GPU and
 * left holding the last call's contents (nothing in it needs to start at
 * zero).  Calls that overlap on one GPU race on that array.  Runs on the
 * current HIP device; the arguments and outputs are those of
 * parapn_pararts.  PARAPN_ENOMEM when the problem needs more scratch than
 * the array holds (N above 46 667 at D = 8 in FP32, 22 495 in FP64, 13 700
 * at D = 15 in FP32). */
int parapn_pararts_noalloc(int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                           const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H,
                           const void *dvec, void *mean_out, void *sqrtcov_out, void *filt_mean_out,
                           void *filt_sqrtcov_out, void *stream);

/* Batched square-root filtering operator (eq. sqrt-associative-filtering):
 * out_k = a_k (x)_f c_k for k < count, a earlier than c.  Each element is the
 * tuple (A [D][D], b [D], sqrtC [D][D], eta [D], sqrtJ [D][D]) stored
 * contiguously as 3D^2 + 2D values in that order; arrays are [count][3D^2+2D]
 * on the device.  sqrtC and sqrtJ need not be triangular; the outputs are
 * lower-triangular with non-negative diagonal. */
int parapn_filter_combine(parapn_ctx *ctx, int32_t D, int64_t count, int32_t precision, const void *a,
                          const void *c, void *out, void *stream);

/* Per-kernel timing for measurement tools (not needed to solve).  While
 * enabled, every solver kernel launch is bracketed by two HIP events recorded
 * on the launch stream; parapn_profile_read waits for them and returns, per
 * kernel name, the summed elapsed milliseconds and the launch count.
 * Enabling (or disabling) clears the counters.  Process-wide; not thread-safe.
 * names receives up to max NUL-terminated names of name_len bytes each;
 * *n_out is the number of distinct kernels seen (may exceed max). */
int parapn_profile_enable(int on);
/* Restrict the timing to launches of one kernel (names as parapn_profile_read
 * reports them, e.g. "fwd_reduce1"); NULL or "" times every kernel. */
int parapn_profile_only(const char *kernel);
int parapn_profile_read(int32_t max, char *names, int32_t name_len, double *total_ms, int64_t *launches,
                        int32_t *n_out);

/* ---- continuous-batching server (many IVPs in flight on one device) ----
 *
 * A served stream runs Alg. 2 for every admitted request in lock step: each
 * parapn_server_step performs one Gauss-Newton iteration (linearisation, the
 * forward filtering scan, the reverse smoothing scan, the trajectory update;
 * Alg. 1 inside Alg. 2) for all active requests, packing requests that share
 * (precision, d, q, damping) into one pair of scans.  The packs of a step are
 * queued back to back on the server's stream and the step waits once, so
 * their device work overlaps.  A pack whose composition did not change since
 * the previous step replays a HIP graph of its iteration (captured once the
 * composition has lasted a step; not on the legacy default stream, and not
 * while parapn_profile_enable is on).  Requests never mix: the first
 * filtering element of each request resets the forward prefix and its last
 * smoothing element cuts the reverse suffix, so one request's NaN or
 * divergence cannot reach another (each converges on its own Delta, Alg. 2's
 * stopping rule).  A finished request's smoothed means are written to its
 * mean_out (device, [N+1][d(q+1)], its precision's element type), and its
 * square-root covariances (the factors of the last linearisation, [N+1][D][D]
 * lower-triangular) to sqrtcov_out when one was given; a completion record
 * is queued.  Requests start from mu0 or, with init_mode = PARAPN_INIT_COARSE,
 * from their coarse-grid start, computed at admission for all requests
 * admitted in a step in one launch per (d, q) (init_traj must be NULL).
 *
 * Admission is in submission order, limited by max_slots active requests and
 * by hbm_budget_bytes (0 = unlimited) summed over the admitted requests'
 * footprints (resident FP64 trajectory, their share of the scan scratch, and
 * their coarse start); a request waits in the queue until both allow it.
 * Resident trajectories come from a pool of device chunks that the server
 * keeps until it is destroyed, and every pack keeps its own scratch between
 * steps, so once a stream's working set has been reached a step allocates
 * nothing.  mean_out and sqrtcov_out must stay valid until the request's
 * completion is polled.  One server per context; a server is not
 * thread-safe. */
typedef struct parapn_server parapn_server;

typedef struct {
    uint64_t req_id;     /* as given to parapn_server_submit */
    int32_t status;      /* PARAPN_OK, PARAPN_MAXITER or PARAPN_ENONFINITE */
    int32_t iterations;  /* Gauss-Newton iterations performed */
    double final_delta;  /* Delta of the last iteration */
    double t_submit, t_start, t_done; /* parapn_server_clock() at submission, admission, completion */
    int32_t start;       /* PARAPN_START_*: the starting trajectory used */
    double sigma_hat;    /* as parapn_info.sigma_hat (NaN for damped requests) */
    double objective;    /* as parapn_info.objective */
} parapn_completion;

/* stream: HIP stream for all of the server's work (NULL = default stream).
 * Errors: PARAPN_EINVAL for NULL ctx/out or max_slots < 1. */
int parapn_server_create(parapn_server **srv, parapn_ctx *ctx, int32_t max_slots, size_t hbm_budget_bytes,
                         void *stream);
/* Waits for the server's stream, frees every request (queued or active)
 * without writing their outputs, and releases the server's device memory. */
void parapn_server_destroy(parapn_server *srv);
/* Seconds on a monotonic clock (the one completion times use). */
double parapn_server_clock(void);
/* Queue one request (validated as for parapn_solve; init_traj must be NULL).
 * sqrtcov_out: device [N+1][D][D] for the request's square-root covariances,
 * or NULL.  PARAPN_ENOMEM if its footprint alone exceeds the server budget. */
int parapn_server_submit(parapn_server *srv, const parapn_problem *prob, uint64_t req_id, void *mean_out,
                         void *sqrtcov_out);
/* Admit what fits, run one iteration for all active requests, retire the
 * finished ones.  Returns after the device work of the step is complete.
 * *n_active / *n_queued (either may be NULL): requests still active / waiting. */
int parapn_server_step(parapn_server *srv, int32_t *n_active, int32_t *n_queued);
/* Move up to max completion records into out (oldest first); *n_out = count. */
int parapn_server_poll(parapn_server *srv, parapn_completion *out, int32_t max, int32_t *n_out);
/* Footprint (bytes) that admission charges for a request without covariances:
 * its resident FP64 trajectory, its share of the scan scratch and its coarse
 * start.  Errors as for submit. */
int parapn_server_footprint(const parapn_problem *prob, size_t *bytes);
/* Admitted bytes now and at most so far; requests admitted and completed.
 * Any output pointer may be NULL. */
int parapn_server_stats(parapn_server *srv, size_t *used_bytes, size_t *peak_bytes, int64_t *admitted,
                        int64_t *completed);

const char *parapn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
