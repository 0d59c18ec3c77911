/*
 * za.h -- C ABI of libza, the MI355X (gfx950) WENO-ZA6 solver library.
 *
 * The calls follow the paper's statement of the problem (Gu, Wang, Don, Jung,
 * arXiv 2603.26272): a hyperbolic conservation law Q_t + div F(Q) = 0 on a
 * uniform mesh (Section 2, eq:hyperbolic_1D_scalar and the 2D Euler system of
 * Section 4.3), discretised by the conservative finite-difference form
 * dQ_i/dt = -(F_{i+1/2} - F_{i-1/2})/dx (eq:hyperbolic_1D_scalar_h) with
 * WENO-ZA6 interface fluxes (Sections 2-3) and integrated by third-order
 * SSP (TVD) Runge-Kutta (Section 4, opening paragraph).
 *
 * Conventions shared by every call:
 *  - No exception crosses the ABI; every call returns a za_status.
 *  - State buffers are DEVICE pointers (HIP/PyTorch allocations on the
 *    context's device).  Layout is structure-of-arrays, row-major with x
 *    fastest: q[c][y][x], c < m, of point values at the cell centres
 *    x_i = xlo + (i + 1/2) dx.  m = 1 (scalar), 3 (1D Euler: rho, rho u, E)
 *    or 4 (2D Euler: rho, rho u, rho v, E).  The caller owns every buffer it
 *    passes; the library never frees it and keeps no reference after the
 *    enqueued work completes.
 *  - All work is enqueued on the context's HIP stream.  za_rhs, za_rhs_fluxes
 *    and za_step (with dt_used == NULL) are asynchronous; za_solve and
 *    za_step with dt_used != NULL synchronise the stream before returning.
 *  - Argument errors are detected before anything is enqueued and change no
 *    state (ZA_ERR_ARG).  Device errors surface as ZA_ERR_DEVICE at the next
 *    synchronising call.  A non-finite or non-physical state (rho <= 0,
 *    p <= 0) seen by a wave-speed reduction yields ZA_ERR_NONFINITE at the
 *    next synchronising call, with za_solve_info.nonfinite_step set.
 *  - A context is used by one host thread at a time.
 */
#ifndef ZA_H
#define ZA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZA_OK = 0,
  ZA_ERR_ARG = 1,          /* invalid argument; nothing was enqueued        */
  ZA_ERR_NOMEM = 2,        /* device allocation failed / over HBM budget    */
  ZA_ERR_DEVICE = 3,       /* a HIP call failed                              */
  ZA_ERR_NONFINITE = 4,    /* NaN/Inf or rho <= 0 / p <= 0 met               */
  ZA_ERR_UNSUPPORTED = 5,  /* valid but not implemented combination          */
  ZA_ERR_BUSY = 6          /* server queue full                              */
} za_status;

/* Flux function.  ZA_ADVECTION: f = a u (Section 2); ZA_EULER: the Euler
 * equations of gas dynamics (Sections 4.2, 4.3); ZA_BURGERS: f = u^2/2 and
 * ZA_BUCKLEY: f = u^2/(u^2 + (1-u)^2/4) (Section 4.1, tab:scalar_fluxes). */
typedef enum { ZA_ADVECTION = 0, ZA_EULER = 1, ZA_BURGERS = 2, ZA_BUCKLEY = 3 } za_system;
typedef enum { ZA_BC_PERIODIC = 0, ZA_BC_TRANSMISSIVE = 1 } za_bc;
/* ZA_FP32_RECON: flux splitting, characteristic projection, smoothness
 * indicators and weights in FP32; the state, the flux difference and the
 * RK3 stage accumulation stay FP64. */
typedef enum { ZA_FP64 = 0, ZA_FP32_RECON = 1 } za_precision;
/* ZA_DT_CFL: 1D dt = cfl dx / max(|u|+c); 2D dt = cfl / (max(|u|+c)/dx +
 * max(|v|+c)/dy) (scalar laws: |f'(u)| in place of |u|+c).
 * ZA_DT_CFL_H2: dt = cfl h^2 with h = min(dx, dy), fixed for the run. */
typedef enum { ZA_DT_CFL = 0, ZA_DT_CFL_H2 = 1 } za_dt_rule;
/* Lax-Friedrichs speed of eq:LF for systems: per characteristic field,
 * alpha_s = max |lambda_s| over the grid, or one max(|u_n|+c) for all. */
typedef enum { ZA_LF_PER_FIELD = 0, ZA_LF_SCALAR = 1 } za_lf;

typedef struct {
  int32_t dim;             /* 1 or 2                                         */
  int32_t system;          /* za_system                                      */
  int32_t nx, ny;          /* cells; ny = 1 when dim == 1                    */
  double  xlo, xhi, ylo, yhi;
  int32_t bc_x, bc_y;      /* za_bc; r ghost cells per side                  */
  double  gamma;           /* ratio of specific heats (1.4 in the paper)     */
  double  adv_speed[2];    /* advection velocity (ZA_ADVECTION)              */
  double  cfl;             /* CFL number (0.45 in the paper)                 */
  int32_t dt_rule;         /* za_dt_rule                                     */
  int32_t precision;       /* za_precision                                   */
  double  p;               /* power parameter of eq:weight_nonlinear (1)     */
  double  eps;             /* sensitivity epsilon (1e-40 FP64, 1e-20 FP32);  */
                           /* at least 1e-300 (FP64) or 1e-37 (FP32)         */
  int32_t affine_invariant;/* 0: mu = 1 (Section 3); 1: mu[f] of eq:aimu      */
  double  mu0;             /* mu_0 of eq:aimu (1e-40 FP64, 1e-8 FP32);       */
                           /* at least 1e-150 (FP64) or 1e-18 (FP32)         */
  int32_t lf;              /* za_lf                                          */
  int32_t linear_weights;  /* 1: omega = d (the linear central flux), tests  */
  int32_t order;           /* r of the order-2r central-upwind scheme: 3 (or  */
                           /* 0) WENO-ZA6, Section 3; 2, 4, 5 the fourth-,    */
                           /* eighth- and tenth-order schemes of Appendix A,  */
                           /* FP64 only (ZA_ERR_UNSUPPORTED otherwise; the    */
                           /* server takes r = 3 only)                        */
  int32_t pp_limiter;      /* 1: positivity-preserving flux limiter (Euler,   */
                           /* FP64) in every stage of za_step / za_solve and  */
                           /* the server: each face flux is blended with the  */
                           /* first-order LF flux so that density and         */
                           /* pressure stay >= 1e-13 (Hu, Adams and Shu 2013, */
                           /* cited in Section 4.3; needs cfl <= 0.5); the    */
                           /* right-hand-side calls are not limited           */
  int32_t alt_tau;         /* 1: the alternative global indicator tau' =      */
                           /* (13/12) <c_tau,f>^2 + <c'_tau,f>^2 of eq:GSI_alt */
                           /* (r = 3; for the dispersion analysis, Section    */
                           /* 3.2); 0: tau of eq:GSI                           */
  double  weight_L;        /* L and q of eq:weights_unnormalized,             */
  double  weight_q;        /* alpha_k = d_k (L + Gamma_k)^q (tab:SpecialCases: */
                           /* Z and Ai-Z: L = q = 1; JS and Ai-JS: L = 0,     */
                           /* p = 2).  L >= 0, q >= 1; both 0 select the      */
                           /* paper's L = q = 1.  With L = 0 the common       */
                           /* factor tau^(pq) cancels in omega and is left    */
                           /* out, which also defines omega where tau = 0.    */
                           /* The server takes L = q = 1 only                 */
} za_problem;

typedef struct za_ctx za_ctx;

typedef struct {
  int64_t steps;           /* RK3 steps taken                                 */
  double  t;               /* final simulated time                            */
  double  dt_min, dt_max;  /* extreme step sizes used                         */
  int64_t nonfinite_step;  /* first step whose input was non-finite, else -1  */
} za_solve_info;

/* Create a context for one problem shape on the current HIP device: the
 * conservation law, mesh, initial-boundary setting and scheme parameters of
 * the paper's problem statement (Section 2, eq:hyperbolic_1D_scalar; the
 * Euler systems eq:Euler1D and Section 4.3; eps and p of
 * eq:weight_nonlinear, Section 4).
 * hip_stream: a hipStream_t (NULL = the default stream).  Allocates the
 * workspace (two RK3 stage states, the x-sweep partial RHS in 2D, the
 * reduction partials and a device control block).  *out receives the
 * context; on error *out is NULL.  Launch shapes are fixed here; the
 * environment variable ZA_XL_CHUNKS, read at this call, sets the chunks of
 * 64 interfaces per row segment of the looped 2D x-sweep (0: one-shot
 * sweep; results are identical either way). */
za_status za_ctx_create(const za_problem* problem, void* hip_stream, za_ctx** out);
/* Not from the paper (resource management): synchronise the context's
 * stream, free its workspace and the context.  ZA_ERR_ARG for NULL. */
za_status za_ctx_destroy(za_ctx* ctx);
/* Not from the paper (stream plumbing): rebind the stream used by later
 * calls.  ZA_ERR_ARG for NULL. */
za_status za_ctx_set_stream(za_ctx* ctx, void* hip_stream);
/* Number of doubles in one state: m * nx * ny, the point values Q_i of
 * eq:hyperbolic_1D_scalar_h (0 if the problem is invalid). */
size_t    za_state_count(const za_problem* problem);
/* Not from the paper (admission control): device bytes the context
 * allocates for this problem (0 if the problem is invalid). */
size_t    za_workspace_bytes(const za_problem* problem);

/* rhs = L(q) = -(F_{i+1/2} - F_{i-1/2})/dx [- (G_{j+1/2} - G_{j-1/2})/dy]
 * (eq:hyperbolic_1D_scalar_h, dimension by dimension in 2D), with the
 * Lax-Friedrichs speeds taken from q itself.  q and rhs: device, m*nx*ny
 * doubles, must not overlap. */
za_status za_rhs(za_ctx* ctx, const double* q, double* rhs);

/* The numerical fluxes themselves (parity checks): h_{i+1/2} = f^+ + f^-
 * of the global Lax-Friedrichs splitting eq:LF, each half the convex
 * combination eq:numerical_flux_WENO of the candidate fluxes
 * eq:numerical_subflux with the weights eq:weights_general; for the Euler
 * equations per characteristic field (Section 4.2).  fx[c][y][k] is F at
 * x_{k-1/2}, k = 0..nx (device, m*ny*(nx+1) doubles); fy[c][k][x] is G at
 * y_{k-1/2}, k = 0..ny (device, m*(ny+1)*nx doubles; 2D only, may be NULL).
 * Asynchronous; ZA_ERR_ARG for NULL q or fx. */
za_status za_rhs_fluxes(za_ctx* ctx, const double* q, double* fx, double* fy);

/* One step of the explicit third-order TVD Runge-Kutta method of Shu and
 * Osher (Section 4, opening paragraph) in place, in its Shu-Osher form
 * Q1 = Q + dt L(Q), Q2 = 3/4 Q + 1/4 (Q1 + dt L(Q1)),
 * Q <- 1/3 Q + 2/3 (Q2 + dt L(Q2)), with L of eq:hyperbolic_1D_scalar_h.
 * q: device state, updated in place.  dt > 0: that step; dt <= 0: the CFL
 * step of the problem's dt rule from q.  dt_used (host, may be NULL): if
 * given, the call synchronises and stores the dt taken (and reports
 * ZA_ERR_NONFINITE for a non-physical state). */
za_status za_step(za_ctx* ctx, double* q, double dt, double* dt_used);

/* Integrate q in place to the final time of an experiment (Section 4: every
 * test runs the TVD Runge-Kutta steps of za_step from t = 0 to its final
 * time T, e.g. T = 0.8 for configuration 3 of Section 4.3) with the CFL
 * rule recomputed each step.  t_final > 0: to t_final, the last step
 * clipped to land on it (ZA_DT_CFL_H2: n = ceil(T/dt (1 - 1e-12)) equal steps, the
 * last T - (n-1) dt), stopping early after max_steps if max_steps > 0.
 * t_final <= 0: exactly max_steps CFL steps without clipping.  dt and t stay
 * on the device; the host checks progress once per captured chunk of steps.
 * info (host, may be NULL) receives the step statistics.  Synchronises. */
za_status za_solve(za_ctx* ctx, double* q, double t_final, int64_t max_steps, za_solve_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): za_rhs
 * without a context.  problem: as for za_ctx_create; q, rhs: device,
 * m*nx*ny doubles each, must not overlap; hip_stream: the hipStream_t to
 * enqueue on (NULL = the default stream).  Computes exactly what za_rhs
 * computes, with the same kernels.  Allocates nothing: the wave-speed
 * partials and the control block live in one static device array of 48.25
 * KiB per GPU (held until the process ends), which covers every grid the
 * library accepts (at most 2^31 cells; the reduction pass strides over the
 * cells with at most 1024 blocks).  Every call on a GPU shares that GPU's
 * array and overwrites it: calls that overlap on one GPU (from other streams
 * or threads) race, and the caller must serialise them.  Asynchronous; a
 * non-finite state is not reported (za_rhs reports it through a context).
 * ZA_ERR_ARG for an invalid problem, NULL or overlapping buffers;
 * ZA_ERR_DEVICE if the device array cannot be found or a launch fails. */
za_status za_rhs_noalloc(const za_problem* problem, const double* q, double* rhs, void* hip_stream);

/* FP64 totals of each conserved variable, sums[c] = sum over cells of q[c]
 * (the conservative form eq:hyperbolic_1D_scalar_h telescopes, so with
 * periodic boundaries these stay constant up to rounding).  Fixed-order
 * tree, repeatable bit for bit.  q: device; sums: host, m doubles.
 * Synchronises. */
za_status za_conserved_sums(za_ctx* ctx, const double* q, double* sums);

/* Not from the paper (diagnostics): a static string naming a status, and
 * the last error message of a context (owned by the context). */
const char* za_status_str(za_status s);
const char* za_ctx_last_error(const za_ctx* ctx);
/* Not from the paper (measurement): per-launch device time (ms) of the most
 * recent za_rhs/za_step/za_solve kernels, by kernel class, when timing is
 * enabled (za_ctx_set_timing; timing records events around every launch and
 * runs steps without the captured step graphs):
 * out[0] = x-sweep, out[1] = y-sweep(+stage), out[2] = wave-speed reduction;
 * counts[k] = number of launches averaged.  Synchronises. */
za_status za_ctx_set_timing(za_ctx* ctx, int32_t enable);
za_status za_ctx_kernel_times(za_ctx* ctx, double* avg_ms, int64_t* counts);

/* ---------------------------------------------------------------------- */
/* Serving (not from the paper, which solves one problem at a time): each  */
/* request is a za_solve of its own problem (the paper's method, as above); */
/* the server adds continuous batching of independent solve requests.      */
/* Requests are admitted while their device footprint fits the HBM budget */
/* and a slot is free; every scheduler step advances all admitted requests */
/* by one RK3 step with batched launches (one launch per kernel class for  */
/* all slots, dispatched through a device slot table), retires finished    */
/* requests and admits waiting ones.  The server owns a scheduler thread   */
/* and a transfer thread (uploads and result downloads).                   */
/* ---------------------------------------------------------------------- */
typedef struct za_server za_server;
typedef int64_t za_req_id;

typedef struct {
  int64_t arrival_ns, admit_ns, finish_ns;   /* host monotonic clock        */
  int64_t steps, interfaces;                 /* RK3 steps, IR computed      */
  int32_t status;                            /* za_status of the request    */
} za_req_stats;

/* Not from the paper.  hbm_budget_bytes: cap on the summed footprint of
 * admitted requests (the server allocates one pool of that size, and a
 * pinned host staging pool of the same size, at most 1 GiB).
 * max_slots: concurrent requests.  device: HIP device ordinal.  *out
 * receives the server (NULL on error). */
za_status za_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t device, za_server** out);
/* Not from the paper.  Copies q0_host (host, m*nx*ny doubles) and queues
 * the request for n_steps CFL steps (za_step's method).  ZA_ERR_NOMEM if
 * its footprint exceeds the whole budget; ZA_ERR_ARG for an invalid
 * problem or a configuration the server does not run. */
za_status za_server_submit(za_server* s, const za_problem* problem, const double* q0_host,
                           int64_t n_steps, za_req_id* id);
/* Not from the paper.  done = 1 once finished; then q_out_host (host, may
 * be NULL) receives the final state and stats (may be NULL) the request's
 * record.  The request is released after a successful poll with done = 1
 * and q_out_host != NULL. */
za_status za_server_poll(za_server* s, za_req_id id, int32_t* done, double* q_out_host,
                         za_req_stats* stats);
/* Not from the paper.  Block until every submitted request has finished
 * (or failed). */
za_status za_server_drain(za_server* s);
/* Not from the paper.  Stop the scheduler, free the pool and the server. */
za_status za_server_destroy(za_server* s);

#ifdef __cplusplus
}
#endif
#endif /* ZA_H */
