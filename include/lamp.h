/*
 * lamp.h -- C ABI of the MI355X (gfx950) implementation of Log-Averaged
 * Mirror Prox (LAMP, arXiv 2511.11359) for discrete optimal transport with a
 * squared-Euclidean cost generated on the fly from point clouds.
 *
 * Problem (Section 1, problem primal_ot / primal_eot):
 *     min_{X in Pi(r,c)} <C, X> - eta H(X),   C_ij = s * ||x_i - y_j||^2,
 * solved through the saddle form (problem spp) by Algorithm 2 (LAMP).  Only the
 * O(n + m) dual state (nu^t, theta^t, t, lam_t = 1/eta_t) is stored; the plan
 * X^t = diag(r) p^{eta_t}(nu^t) (equation def:dual_to_primal) is implicit.
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer owned by the caller; the library
 *    never frees caller memory and never aborts.  Scratch memory is the caller's
 *    workspace `ws` of `ws_bytes` bytes (size from lamp_workspace_bytes), 256-byte
 *    aligned.
 *  - `stream` is a hipStream_t (NULL: the default stream).  Work is enqueued on
 *    it; the calls that return host values (step with res_out, solve,
 *    certificate, cost_scale) synchronise that stream before returning.
 *  - Concurrent calls are safe when they use distinct workspaces and states.
 *  - Errors are returned as negative lamp_status codes; lamp_last_error() gives
 *    a thread-local message for the last non-OK status of the calling thread.
 */
#ifndef LAMP_H
#define LAMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAMP_OK = 0,
    LAMP_NOT_CONVERGED = 1,  /* max_iter reached before tol; the state is valid   */
    LAMP_EINVAL = -1,        /* null pointer, n, m or d < 1, eta < 0, tau1*eta > 1,
                                tol < 0, unknown precision, bad state (t < 0)      */
    LAMP_EDOMAIN = -2,       /* r or c has an entry <= 0 or a sum off 1 by > 1e-9  */
    LAMP_ENOMEM = -3,        /* ws_bytes < lamp_workspace_bytes(...)               */
    LAMP_EDEVICE = -4,       /* a HIP runtime call failed                          */
    LAMP_ENUMERIC = -5       /* a non-finite value appeared in the dual update     */
} lamp_status;

typedef enum {
    LAMP_FP32 = 0,           /* cost and exponent arguments assembled in FP64 on the
                                vector ALU, exponentials and their sums in FP32,
                                duals FP64: the reference-accuracy form           */
    LAMP_FP32_MFMA = 1,      /* x.y^T tiles on FP32 matrix cores, exponent assembled
                                in FP32, duals FP64                               */
    LAMP_BF16_MFMA = 2,      /* x.y^T tiles from BF16 points on matrix cores with
                                FP32 accumulation; exponentials and sums FP32      */
    LAMP_FP16_MFMA = 3,      /* as LAMP_BF16_MFMA with FP16 points                 */
    LAMP_FP16X3_MFMA = 4     /* x.y^T from split FP16 points on matrix cores: each
                                centred coordinate, times a power-of-two range
                                scale, as hi + lo (two FP16 roundings), and
                                x_hi.y_hi + x_hi.y_lo + x_lo.y_hi in one FP16
                                contraction over 3 d entries with FP32
                                accumulation (about 22 significant bits against
                                FP16's 11); exponentials and sums FP32; d <= 64   */
} lamp_precision;           /* the other matrix-core forms need d <= 128           */

/* Ground cost C_ij = s dist(x_i, y_j) generated from the point clouds: the squared
 * Euclidean cost of Sections 1 and 4.1, and the l1 and l_inf costs of the
 * kernelized experiments (Section 5); or C_ij = s cost_ij from a cost matrix the
 * caller stores (the non-kernelized costs of Appendix E, fused reductions).  The
 * matrix-core forms and the batching form run the squared Euclidean cost only; the
 * adjoints need point clouds. */
typedef enum {
    LAMP_SQEUCLID = 0,   /* ||x - y||_2^2 */
    LAMP_L1 = 1,         /* sum_k |x_k - y_k| */
    LAMP_LINF = 2,       /* max_k |x_k - y_k| */
    LAMP_EXPLICIT = 3    /* cost_ij of lamp_problem.cost */
} lamp_metric;

/* Element type of an explicit cost matrix. */
typedef enum {
    LAMP_COST_F32 = 0,       /* float                                              */
    LAMP_COST_BF16 = 1,      /* bfloat16 (8-bit significand, FP32 exponent range)  */
    LAMP_COST_F16 = 2        /* IEEE half (11-bit significand, entries <= 65504)   */
} lamp_cost_type;

/* Problem data (Section 1; Algorithm 2, REQUIRE line).
 *   x: n x d, y: m x d, row-major FP32 point clouds (device).  Not read, and may be
 *      NULL, with metric LAMP_EXPLICIT; d is then ignored.
 *   metric: lamp_metric of the ground cost.
 *   r: n, c: m, FP64 marginals (device), strictly positive, each summing to 1
 *      (the paper adds 1e-6 and renormalises to get full support, Appendix E).
 *   cost_scale: s in C_ij = s dist(x_i, y_j).  <= 0: s = 1 / max_ij dist(x_i, y_j) is
 *      computed on the device (then ||C||_inf = 1).
 *   cost_norm: ||C||_inf = max_ij C_ij.  <= 0: computed on the device.  Only
 *      trusted as given when both cost_scale and cost_norm are > 0.
 *   cost: with metric LAMP_EXPLICIT, the n x m cost matrix, row-major, of element type
 *      cost_type (device, caller-owned, read only; entry (i, j) at element i m + j;
 *      m <= 2^30, else LAMP_EINVAL).
 *      Entries must be finite and >= 0 with a positive maximum; that maximum is checked
 *      (LAMP_EDOMAIN when it is not positive) only when the library computes the scale,
 *      the rest is not checked.  Each entry is widened exactly to FP32 and then to FP64:
 *      the 2-byte types halve the HBM traffic of the sweeps and solve the problem whose
 *      cost is the rounded matrix.  Ignored, and may be NULL, for the other ground costs.
 *   cost_type: lamp_cost_type of cost (LAMP_EXPLICIT only; else ignored).
 *   reserved: set to 0 (not read; keeps the struct 8-byte aligned). */
typedef struct {
    int64_t n, m;
    int32_t d, metric;
    const float *x, *y;
    const double *r, *c;
    double cost_scale;
    double cost_norm;
    const void *cost;
    int32_t cost_type, reserved;
} lamp_problem;

/* Algorithm parameters (Algorithm 2; defaults from Appendix E, "for all LAMP
 * testing": alpha = 0.01, beta = 1.1, tau1 = tau2 = 1/(2||C||_inf)).
 *   eta >= 0: entropic regularisation; tau1 * eta <= 1 is required
 *      (Lemma primal_md_eq_dual_avg, Proposition equivalence).
 *   tol: stop at the first t >= 1 with ||col(X^t) - c||_1 <= tol (row(X^t) = r by
 *      construction, eq:row_feasible; t = 0, the product coupling, is not tested);
 *      0 runs exactly max_iter iterations.
 *   alpha, beta, tau1, tau2: <= 0 selects the default.
 *   check_every: iterations per host check of the stopping flag in lamp_solve
 *      (<= 0: 64).  The tolerance itself is tested on the device every iteration.
 *   track_dt: 1 accumulates, every iteration, the summand of the partial sums D_t of
 *      Proposition infeas_bound(b) (def:sum_condition) into lamp_state.dt_partial; it
 *      adds one pass over the n x m pairs per iteration (the cost <C, Xbar^{t+1}>).
 *      Only with precision LAMP_FP32 and outside the batched solve (else LAMP_EINVAL).
 *      0: no tracking (the state's dt_partial becomes NaN once an iteration runs).
 *   reserved: set to 0 (not read). */
typedef struct {
    double eta, tol;
    int64_t max_iter;
    double alpha, beta, tau1, tau2;
    int32_t precision, check_every;
    int32_t track_dt, reserved;
} lamp_params;

/* O(n + m) state of Algorithm 2 after t iterations (caller-owned).
 *   nu, theta: m FP64 each (device): nu^t, theta^t.  t = 0 with zeros is the
 *      start of Algorithm 2 (theta^0 = nu^0 = 0, eta_0 = infinity).
 *   t: iterations done; inv_eta: lam_t = 1/eta_t (0 at t = 0).
 *   dt_partial: the part of D_t accumulated by the iterations so far (host value, 0 at
 *      t = 0): for s < t, D_H(thetabar^{s+1}||thetahat^{s+1}) - D_H(thetabar^{s+1}||theta^s)
 *      + (lam_{s+1} - lam_s) <C, Xbar^{s+1}> + K <col(Xbar^{s+1}), lam_{s+1} nu^{s+1} - lam_s nu^s>,
 *      i.e. D_t without the telescoped <r, log Z^t - log Z^0> that lamp_certificate adds
 *      (Lemma kl_diff, Lemma Dha_diff).  NaN once an iteration ran without track_dt.
 * The state fully determines the rest of the run: checkpointing is copying it. */
typedef struct {
    double *nu, *theta;
    int64_t t;
    double inv_eta;
    double dt_partial;
} lamp_state;

/* Optional per-iteration outputs of lamp_step (device, nullable each):
 *   log_za[n], log_zb[n]: natural log Z_i of p^{eta_t}(nu^t) and p^{eta_{t+1}}(nubar^{t+1})
 *      (Section 4.1, first display);
 *   col_a[m], col_b[m]: col_r of the same two maps (Section 4.1, second display);
 *   theta_bar[m], theta_hat[m]: the two dual mirror steps (step:lamp_mid_theta,
 *      step:lamp_main_theta). */
typedef struct {
    double *log_za, *log_zb, *col_a, *col_b, *theta_bar, *theta_hat;
} lamp_trace;

/* Certificate of X^t = diag(r) p^{eta_t}(nu^t) (Proposition infeas_bound; Appendix B).
 * Pair terms as in the sweeps (FP64 exponent argument, FP32 exponential, FP32 sums over
 * blocks of columns, FP64 beyond); the minima of the dual values D(.) in FP64. */
typedef struct {
    double col_res;          /* ||col(X^t) - c||_1                                   */
    double row_res;          /* ||row(X^t) - r||_1, measured                          */
    double cost;             /* <C, X^t>                                              */
    double dual_theta;       /* D(theta^t) (def:dual_spp), a lower bound on OPT       */
    double dual_nu;          /* D(nu^t)                                               */
    double primal_penalized; /* <C,X^t> + 2||C||_inf (row_res + col_res) >= OPT       */
    double gap;              /* primal_penalized - max(dual_theta, dual_nu)           */
    double prop_bound;       /* 4||C||_inf col_res + 2||C||_inf log(m) / t (t >= 1)   */
    double cost_scale;       /* s used                                                */
    double cost_norm;        /* ||C||_inf used                                        */
    int64_t t;
    double rounded_cost;     /* <C, Round(X^t)>, Round of Algorithm 3 applied to X^t
                                on the device, without forming X                      */
    double dt;               /* D_t (def:sum_condition): state.dt_partial + <r, log Z^t>
                                - log m; NaN unless every iteration tracked it        */
    double midpoint_bound;   /* 2||C||_inf (log m + (1 + alpha) log 2 + D_t) / t, the
                                right-hand side of ineq:spp_midpoint_conv (eta = 0)  */
    double dual_eta_theta;   /* D^eta(theta^t) (def:dual_spp_e) at the params' eta > 0:
                                sum_i r_i softmin^eta_j (C_ij + 2||C||_inf theta_j)
                                - 2||C||_inf <c, theta>; NaN when eta = 0           */
    double dual_eta_nu;      /* D^eta(nu^t), likewise                                 */
} lamp_cert;

typedef struct {
    int64_t iters;           /* iterations performed by this call                     */
    int64_t t;               /* state.t on return                                     */
    double seconds;          /* wall time of the call                                 */
    double final_res;        /* ||col(X^t) - c||_1 of the returned iterate            */
    double cost_scale;       /* s used                                                */
    double cost_norm;        /* ||C||_inf used                                        */
    int32_t converged;       /* 1 if final_res <= tol                                 */
    int32_t row_fallbacks;   /* rows whose normaliser was recomputed exactly          */
} lamp_report;

/* Bytes of workspace needed for this problem and these parameters. */
size_t lamp_workspace_bytes(const lamp_problem *prob, const lamp_params *params);

/* s = 1 / max_ij dist(x_i, y_j) for the problem's ground cost (FP64 from the FP32
 * points; max_ij cost_ij for LAMP_EXPLICIT), the normalisation that makes
 * ||C||_inf = 1.  *max_sqdist_out (host, nullable) gets the maximum. */
lamp_status lamp_cost_scale(const lamp_problem *prob, void *ws, size_t ws_bytes, void *stream,
                            double *s_out, double *max_sqdist_out);

/* One iteration t -> t+1 of Algorithm 2 (steps step:eta_update ... tclip), in
 * place on `state`.  res_out (host, nullable) receives ||col(X^t) - c||_1 of the
 * iterate X^t the step started from.  trace (nullable) receives intermediates. */
lamp_status lamp_step(const lamp_problem *prob, const lamp_params *params, lamp_state *state,
                      void *ws, size_t ws_bytes, void *stream, const lamp_trace *trace,
                      double *res_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lamp_step with the workspace taken
 * from a fixed device array of LAMP_NOALLOC_WS_BYTES bytes that the library holds, one
 * per device, until the process ends.  Same arguments, kernels and results as lamp_step
 * without ws / ws_bytes.  The call allocates nothing (no hipMalloc, no allocating library
 * routine); it looks the array's address up once per device on its first call there.
 * Problems whose lamp_workspace_bytes exceeds LAMP_NOALLOC_WS_BYTES are rejected with
 * LAMP_ENOMEM (64 MiB: enough for n = m = 2^16 at d = 3 in LAMP_FP32, 49 MiB).  Every call
 * on one device shares that array, so calls that overlap in time on one device race
 * (serialise them, e.g. on one stream); nothing in it has to start at zero. */
#define LAMP_NOALLOC_WS_BYTES ((size_t)64 << 20)
lamp_status lamp_step_noalloc(const lamp_problem *prob, const lamp_params *params, lamp_state *state,
                              void *stream, const lamp_trace *trace, double *res_out);

/* Runs Algorithm 2 from `state` (t = 0: a fresh start; t > 0: resumes) until
 * ||col(X^t) - c||_1 <= tol or max_iter iterations of this call.  On LAMP_OK the
 * state holds the iterate that met the tolerance (that iteration's update is not
 * applied); on LAMP_NOT_CONVERGED it holds the last iterate.  The iteration loop
 * runs as a captured HIP graph replayed in chunks of check_every iterations. */
lamp_status lamp_solve(const lamp_problem *prob, const lamp_params *params, lamp_state *state,
                       void *ws, size_t ws_bytes, void *stream, lamp_report *out);

/* Certificate of the state's iterate (Proposition infeas_bound(a), def:dual_spp,
 * problem l1_ot_primal); out is a host pointer. */
lamp_status lamp_certificate(const lamp_problem *prob, const lamp_params *params,
                             const lamp_state *state, void *ws, size_t ws_bytes, void *stream,
                             lamp_cert *out);

/* Transport cost <C, X^t> = sum_i r_i sum_j p_ij C_ij of the state's iterate (the cost
 * term of the certificate, Proposition infeas_bound(a), without its other passes) in one
 * pass over the pairs: per row, unnormalised weights with a running integer offset and the
 * sums Z_i, S_i = sum_j q_ij C_ij (FP32 within blocks of 8 columns, FP64 across them), then
 * s r_i S_i / Z_i summed in a fixed order.  *cost (device, one double) is written
 * stream-ordered; the call returns without waiting for it.  Requires state->t >= 1 and
 * point clouds (LAMP_EXPLICIT: LAMP_EINVAL; lamp_certificate reports that cost). */
lamp_status lamp_transport_cost(const lamp_problem *prob, const lamp_params *params,
                                const lamp_state *state, void *ws, size_t ws_bytes, void *stream,
                                double *cost);

/* Envelope gradient of the transport cost with respect to the source points at
 * the state's iterate (not in the paper; the derivative sum_j X_ij dC_ij/dx_i of
 * <C, X> with X = X^t held fixed, at fixed s):
 *     squared Euclidean: grad_x[i, :] = grad_out * 2 s r_i sum_j p_ij (x_i - y_j),
 *     l1:                grad_x[i, k] = grad_out * s r_i sum_j p_ij sign(x_ik - y_jk),
 *     l_inf:             the same restricted to the coordinate of max_k |x_ik - y_jk|
 *                        (the first on ties), sign(0) = 0 (subgradients at kinks),
 * written to grad_x (device, n x d, FP32, row-major).  Requires state->t >= 1 and
 * point clouds (LAMP_EXPLICIT: LAMP_EINVAL). */
lamp_status lamp_backward(const lamp_problem *prob, const lamp_params *params,
                          const lamp_state *state, double grad_out, float *grad_x, void *ws,
                          size_t ws_bytes, void *stream);

/* Envelope gradient with respect to the target points (the column-side counterpart
 * of lamp_backward): grad_y[j, :] = grad_out * sum_i X_ij dC_ij/dy_j at the state's
 * iterate X^t, i.e. 2 s sum_i X_ij (y_j - x_i) for the squared Euclidean cost and the
 * subgradients -s sign(x_ik - y_jk) (l1; l_inf on the coordinate of the largest
 * |x_k - y_k|) for the others; written to grad_y (device, m x d, FP32, row-major).
 * Requires state->t >= 1 and point clouds (LAMP_EXPLICIT: LAMP_EINVAL). */
lamp_status lamp_backward_y(const lamp_problem *prob, const lamp_params *params,
                            const lamp_state *state, double grad_out, float *grad_y, void *ws,
                            size_t ws_bytes, void *stream);

/* Measurement support (not part of the method): average device time in ms of one
 * row sweep and one column sweep of iteration state->t (the two O(nm) kernels of
 * Section 4.1), each launched `reps` times back to back between HIP events on
 * `stream`.  The state is not modified. */
lamp_status lamp_sweep_times(const lamp_problem *prob, const lamp_params *params,
                             const lamp_state *state, void *ws, size_t ws_bytes, void *stream,
                             int32_t reps, double *row_ms, double *col_ms);

/* Measurement support (not part of the method): the issue rate of the exponential
 * instruction the sweeps are bound by.  Launches `blocks` blocks of 256 threads, each lane
 * running 8 independent chains of `iters` base-2 exponentials, `reps` times back to back
 * between HIP events on `stream` (after one untimed launch); *exp_per_s (host) receives
 * exponentials per second.  Reads and writes no memory. */
lamp_status lamp_exp_rate(void *stream, int32_t blocks, int32_t iters, int32_t reps, double *exp_per_s);

/* Batching form: `count` independent problems of any n, m, d advance together.  Each
 * phase of an iteration (row sweep, row finish, column sweep, dual update) is one
 * launch for the whole batch: a persistent grid loops over a work list of
 * (problem, tile) items.  The iteration loop is a captured HIP graph.  A problem whose
 * residual meets tol stops there (its items exit at once) while the others continue.
 * The launch shape (sweep items per phase, grid size) is chosen by timing candidate
 * shapes on the batch (autotuner, cached per batch shape for the process).
 *   probs[count], states[count], outs[count] (host arrays of the structs above);
 *   all problems run LAMP_FP32 with the same params (track_dt = 0); their costs must share one
 *   ||C||_inf (e.g. all normalised: cost_scale <= 0) and their states one t and lam_t.
 * The workspace (lamp_batch_workspace_bytes) holds every problem's scratch. */
size_t lamp_batch_workspace_bytes(const lamp_problem *probs, int32_t count, const lamp_params *params);
lamp_status lamp_solve_batched(const lamp_problem *probs, int32_t count, const lamp_params *params,
                               lamp_state *states, void *ws, size_t ws_bytes, void *stream,
                               lamp_report *outs);

/* Message for the last non-OK status returned to the calling thread. */
const char *lamp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAMP_H */
