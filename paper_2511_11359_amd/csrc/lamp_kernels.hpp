// HIP kernels (gfx950) of the LAMP iteration: Algorithm 2 with the log-domain
// marginals of Section 4.1, for the cost C_ij = s ||x_i - y_j||^2 generated on
// the fly.
//
// Notation (all logarithms of probabilities are kept in base 2; LOG2E = 1/ln 2):
//   points are centred, x~_i = x_i - mu, y~_j = y_j - mu (C is translation
//   invariant), stored as FP64, with squared norms xn2_i, yn2_j;
//   for a dual vector v and inverse temperature lam (= 1/eta),
//     e_ij = -lam LOG2E (C_ij + K v_j)                                  K = 2||C||_inf
//          = q_i + g_j + cfac * (x~_i . y~_j)
//     q_i  = -lam LOG2E s xn2_i,  g_j = -lam LOG2E (s yn2_j + K v_j),  cfac = 2 s lam LOG2E.
//   The row log-normaliser (Section 4.1, first display) in base 2 is
//     l_i = q_i + sigma_i,   sigma_i = log2 sum_j 2^(g_j + cfac x~_i.y~_j).
//   Iteration t evaluates two couplings: A = p^{eta_t}(nu^t) and B = p^{eta_{t+1}}(nubar^{t+1}).
//
// Row sweep: a per-row offset h_i (in dot-product units) is shared by A and B;
//     S_i = sum_j 2^(cfac (h_i + x~_i.y~_j) + g_j) = 2^(cfac h_i + sigma_i).
// h_i is the previous iteration's -sigma^B_i / cfac^B, which keeps every
// exponent within a few units of 0 (the per-iteration change of the exponents
// is bounded by tau1 ||C||_inf-scaled terms); rows whose sums leave a safe range
// are recomputed exactly.  No running max is needed.
//
// Column sweep (Section 4.1, second display): with k_i = -sigma^B_i / cfac^B,
//     p^B_ij = 2^(cfac^B (k_i + x~.y~) + g^B_j)
//     p^A_ij = 2^(rho sigma^B_i - sigma^A_i) * 2^(cfac^A (k_i + x~.y~) + g^A_j),  rho = cfac^A/cfac^B,
// so col_j = sum_i w_i 2^(...) with per-row weights w^B_i = r_i, w^A_i = r_i 2^(rho sigma^B - sigma^A).
//
// Every (i, j) exponent is assembled in FP64 (full-rate FMA on CDNA4), converted
// to FP32 and exponentiated with v_exp_f32; sums run in FP32 within short chunks
// and are carried in FP64.  The streamed side of each sweep (columns for the row
// sweep, rows for the column sweep) is wave-uniform and is read through scalar
// loads; the owned side lives in VGPRs, one row (or column) per lane.  Partial
// sums over splits of the streamed range go to a workspace and are merged in a
// fixed order, so results are deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lampk {

constexpr double LOG2E = 1.4426950408889634074;
constexpr double LN2 = 0.69314718055994530942;
constexpr int BLOCK = 256;
constexpr int UNROLL = 8;

// Device-side control block (lives in the workspace).
struct Ctrl {
    int64_t t;          // index of the iteration the next kernels execute
    int64_t t_end;      // exclusive end of this call's iterations
    int64_t t_base;     // schedule index base: sched[t - t_base]
    int64_t t_done;     // iteration whose residual met tol (-1 otherwise)
    int32_t done;       // 1 once res_t <= tol
    int32_t err;        // bit 0: non-finite value in the dual update
    int32_t fallbacks;  // rows recomputed exactly
    uint32_t pad0;
    double tol;         // 0: never stop early
    double res_last;    // ||col(X^t) - c||_1 of the last completed iteration
    double dt_acc;      // accumulated D_t summands without the normaliser telescope
    double dt_cost;     // <C, Xbar^{t+1}> of the running iteration (D_t tracking)
};

// Per-iteration scalars, filled on the host in FP64 by the recursion of step:eta_update.
struct Sched {
    double lamA;   // lam_t
    double lamB;   // lam_{t+1}
    double w;      // tau1 / lam_{t+1}  (= tau1 eta_{t+1})
    double lamC;   // lam_{t+2}
    double w2;     // tau1 / lam_{t+2}
    double pad[3];
};

// Per-solve constants.
struct Consts {
    int64_t n, m;
    double s;       // cost scale
    double K;       // 2 ||C||_inf
    double kappa;   // 2 tau2 ||C||_inf
    double alpha_m; // alpha / m
    double clipb;   // tanh(beta / 2)
    int metric;     // ground cost, METRIC_*
    int factor_cols;     // one-chain matrix-core column sweep: per-column factor (see there)
    double dscale;       // matrix-core dot products are dscale^-1 times x~.y~ (a power of two; 1 but
                         // for the split FP16 form, whose operands carry a range scale)
    int cost_type;       // COST_* element type of `cost`
    const void* cost;    // METRIC_EXPLICIT: the caller's n x m cost matrix, row-major
};

enum : int { COST_F32 = 0, COST_BF16 = 1, COST_F16 = 2 };

// One cost entry widened exactly to FP32 (a 2-byte entry by its bit pattern).
__device__ __forceinline__ float widen_cost(float v) { return v; }
__device__ __forceinline__ float widen_cost(__bf16 v) {
    return __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(uint16_t, v) << 16);
}
__device__ __forceinline__ float widen_cost(_Float16 v) { return (float)v; }

// Non-temporal load of one entry of type T, widened to FP32.
template <typename T>
__device__ __forceinline__ float load_cost(const T* p) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_nontemporal_load(p);
    } else {
        const uint16_t bits = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
        return widen_cost(__builtin_bit_cast(T, bits));
    }
}

// The entry at column j of a row: a wave-uniform row base plus a 32-bit byte offset (the
// explicit cost has m <= 2^30 columns), which the loads take as a scalar base and a vector
// offset instead of a 64-bit vector address per load.
template <typename T>
__device__ __forceinline__ float load_cost_col(const T* row, int64_t j) {
    const uint32_t off = (uint32_t)j * (uint32_t)sizeof(T);
    return load_cost(reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + off));
}

// ---------------------------------------------------------------------------
// Ground costs.  Every kernel works with a pair term P(x, y) defined so that
//     C_ij = s (|x~_i|^2 + |y~_j|^2 - 2 P(x~_i, y~_j)):
// the inner product with the squared norms for the squared Euclidean cost
// (Sections 1 and 4.1), and -dist(x, y)/2 with zero norm arrays for the l1 and
// l_inf costs of the kernelized experiments (Section 5).  The exponent assembly,
// the offsets, the certificate and the cost maximum are then the same for all of them.
// A cost matrix given by the caller (METRIC_EXPLICIT) enters the same way, with
// P_ij = -cost_ij / 2 and zero norms: its points carry index codes instead of
// coordinates (d = 1), row i the code i and column j the code -(j + 1), so that the
// generic pair term finds (i, j) whichever of the two points it is given first.
// ---------------------------------------------------------------------------
enum : int { METRIC_SQEUCLID = 0, METRIC_L1 = 1, METRIC_LINF = 2, METRIC_EXPLICIT = 3 };

// init + P(x, y) with x in registers and y streamed.
template <int M, int D>
__device__ __forceinline__ double pair_term(const double (&x)[D], const double* __restrict__ y, double init) {
    if constexpr (M == METRIC_SQEUCLID) {
        double d = init;
#pragma unroll
        for (int k = 0; k < D; ++k) d = fma(x[k], y[k], d);
        return d;
    } else {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = fabs(x[k] - y[k]);
            a = (M == METRIC_L1) ? a + t : fmax(a, t);
        }
        return fma(-0.5, a, init);
    }
}

// init - cost_ij / 2 for the index codes a, b of a row and a column (either order).
__device__ __forceinline__ double pair_term_cost(const Consts& kc, double a, double b, double init) {
    const bool row_first = a >= 0.0;
    const int64_t i = (int64_t)(row_first ? a : b);
    const int64_t j = -(int64_t)(row_first ? b : a) - 1;
    const int64_t e = i * kc.m + j;
    float v;
    if (kc.cost_type == COST_BF16) v = widen_cost(static_cast<const __bf16*>(kc.cost)[e]);
    else if (kc.cost_type == COST_F16) v = widen_cost(static_cast<const _Float16*>(kc.cost)[e]);
    else v = static_cast<const float*>(kc.cost)[e];
    return fma(-0.5, (double)v, init);
}

// init + P(x, y), both operands in memory, metric and dimension at run time.
__device__ __forceinline__ double pair_term_dyn(const Consts& kc, int D, const double* __restrict__ x,
                                                const double* __restrict__ y, double init) {
    const int M = kc.metric;
    if (M == METRIC_EXPLICIT) return pair_term_cost(kc, x[0], y[0], init);
    if (M == METRIC_SQEUCLID) {
        double d = init;
        for (int k = 0; k < D; ++k) d = fma(x[k], y[k], d);
        return d;
    }
    double a = 0.0;
    for (int k = 0; k < D; ++k) {
        const double t = fabs(x[k] - y[k]);
        a = (M == METRIC_L1) ? a + t : fmax(a, t);
    }
    return fma(-0.5, a, init);
}

// Row data streamed by the column sweep.
struct RowVar {
    double k;   // -sigma^B_i / cfac^B
    float wA;   // r_i 2^(rho sigma^B_i - sigma^A_i)
    float wB;   // r_i
};

__device__ __forceinline__ bool halted(const Ctrl* ctrl) {
    return ctrl->done != 0 || ctrl->t >= ctrl->t_end;
}

// Sweeps over (blocks of the owned points) x (P splits of the streamed range of length len,
// `split` points each) run on a one-dimensional grid: block b takes split b mod P of owned
// block b / P.  Consecutive block indices go to the eight XCDs in turn, so with P a multiple
// of 8 every XCD streams the same P / 8 splits, whose data then stay in its L2.
struct SweepBlock {
    int64_t bx, p;
};
__device__ __forceinline__ SweepBlock sweep_block(int64_t len, int64_t split) {
    const int64_t P = (len + split - 1) / split;
    return SweepBlock{(int64_t)blockIdx.x / P, (int64_t)blockIdx.x % P};
}

__device__ __forceinline__ float fexp2(double e) {
    return __builtin_amdgcn_exp2f(static_cast<float>(e));
}

// ---------------------------------------------------------------------------
// Preparation: centred FP64 copies, squared norms.
// ---------------------------------------------------------------------------
__global__ void prep_points(const float* __restrict__ pts, int64_t cnt, int d,
                            const float* __restrict__ mu_src_a, const float* __restrict__ mu_src_b,
                            double* __restrict__ out, double* __restrict__ nrm2,
                            float* __restrict__ outf, int metric) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        // centre mu = (x_0 + y_0) / 2: any fixed point works, this one keeps
        // the coordinates of both clouds within one diameter of the origin
        double mu = 0.5 * ((double)mu_src_a[k] + (double)mu_src_b[k]);
        double v = (double)pts[i * d + k] - mu;
        out[i * d + k] = v;
        if (outf) outf[i * d + k] = (float)v;
        acc = fma(v, v, acc);
    }
    nrm2[i] = metric == METRIC_SQEUCLID ? acc : 0.0;   // the l1 / l_inf pair term carries the cost
}

// Index codes of the points of an explicit cost matrix: i for row i, -(i + 1) for
// column i (cols = 1); zero norms.
__global__ void prep_cost_codes(int64_t cnt, int cols, double* __restrict__ out, double* __restrict__ nrm2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    out[i] = cols ? -(double)(i + 1) : (double)i;
    nrm2[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Column table of iteration t from the state (nu^t, theta^t):
//   g^A_j = -lam_t LOG2E (s yn2_j + K nu_j),  g^B_j = -lam_{t+1} LOG2E (s yn2_j + K nubar_j),
//   nubar = nu + w (theta - nu)  (step:lamp_mid_nu).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void col_table_init_body(const Ctrl* ctrl, const Sched* sched, Consts kc,
                               const double* __restrict__ yn2, const double* __restrict__ nu,
                               const double* __restrict__ theta, double2* __restrict__ gtab2,
                               float2* __restrict__ gtabf, int64_t m_pad, int64_t bx_, int64_t by_, int64_t nb_) {
    int64_t j = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    double nb = nu[j] + sc.w * (theta[j] - nu[j]);
    double base = kc.s * yn2[j];
    double2 g;
    g.x = -sc.lamA * LOG2E * (base + kc.K * nu[j]);
    g.y = -sc.lamB * LOG2E * (base + kc.K * nb);
    gtab2[(t & 1) * kc.m + j] = g;
    if (gtabf) gtabf[(t & 1) * m_pad + j] = make_float2((float)g.x, (float)g.y);
}

__global__ void col_table_init(const Ctrl* ctrl, const Sched* sched, Consts kc,
                               const double* __restrict__ yn2, const double* __restrict__ nu,
                               const double* __restrict__ theta, double2* __restrict__ gtab2,
                               float2* __restrict__ gtabf, int64_t m_pad) {
    col_table_init_body(ctrl, sched, kc, yn2, nu, theta, gtab2, gtabf, m_pad, (int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)gridDim.x);
}

// a_j = -g^B_j / cfac^B for the exact offset initialisation.
__device__ __forceinline__ void offset_coeffs_body(const Ctrl* ctrl, const Sched* sched, Consts kc,
                              const double2* __restrict__ gtab2, double* __restrict__ a, int64_t bx_, int64_t by_, int64_t nb_) {
    int64_t j = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    a[j] = -gtab2[(t & 1) * kc.m + j].y / cB;
}

__global__ void offset_coeffs(const Ctrl* ctrl, const Sched* sched, Consts kc,
                              const double2* __restrict__ gtab2, double* __restrict__ a) {
    offset_coeffs_body(ctrl, sched, kc, gtab2, a, (int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)gridDim.x);
}

// ---------------------------------------------------------------------------
// Row extreme sweep: out_i = min_j (a_j + sgn * x~_i . y~_j), FP64, exact.
// Used for the exact offsets, D(theta) and the cost maximum.
// part: [P][n] partial minima over column splits.
// ---------------------------------------------------------------------------
template <int M, int D>
__device__ __forceinline__ void row_extreme_body(Consts kc, const double* __restrict__ xc,
                                                     const double* __restrict__ yc,
                                                     const double* __restrict__ a, double sgn,
                                                     double* __restrict__ part, int64_t split, int64_t bx_, int64_t by_, int64_t nb_) {
    const int64_t i = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = (M == METRIC_SQEUCLID ? sgn : 1.0) * xc[ii * D + k];
    // a_j + sgn P(x_i, y_j): the inner product takes the sign on x, the distances after
    auto term = [&](const double* yj, double aj) {
        return M == METRIC_SQEUCLID ? pair_term<M, D>(x, yj, aj) : fma(sgn, pair_term<M, D>(x, yj, 0.0), aj);
    };
    // blocks of UNROLL columns with independent chains, as in the sweeps: the column data
    // are wave-uniform and their scalar loads overlap the arithmetic of the block
    double best = __builtin_inf();
    const int nfull = (int)((j1 - j0) / UNROLL);
    const double* __restrict__ yp = yc + j0 * D;
    const double* __restrict__ ap = a + j0;
    for (int c = 0; c < nfull; ++c, yp += UNROLL * D, ap += UNROLL) {
        double v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = term(yp + u * D, ap[u]);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) best = fmin(best, v[u]);
    }
    const int rem = (int)((j1 - j0) - (int64_t)nfull * UNROLL);
    for (int u = 0; u < rem; ++u) best = fmin(best, term(yp + u * D, ap[u]));
    if (i < kc.n) part[p * kc.n + i] = best;
}

template <int M, int D>
__global__ __launch_bounds__(BLOCK) void row_extreme(Consts kc, const double* __restrict__ xc,
                                                     const double* __restrict__ yc,
                                                     const double* __restrict__ a, double sgn,
                                                     double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    row_extreme_body<M, D>(kc, xc, yc, a, sgn, part, split, sb.bx, sb.p, 0);
}

// Generic-d version: coordinates read per pair.
__device__ __forceinline__ void row_extreme_dyn_body(Consts kc, int D, const double* __restrict__ xc,
                                                         const double* __restrict__ yc,
                                                         const double* __restrict__ a, double sgn,
                                                         double* __restrict__ part, int64_t split, int64_t bx_, int64_t by_, int64_t nb_) {
    const int64_t i = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    double best = __builtin_inf();
    for (int64_t j = j0; j < j1; ++j) {
        best = fmin(best, fma(sgn, pair_term_dyn(kc, D, xc + ii * D, yc + j * D, 0.0), a[j]));
    }
    if (i < kc.n) part[p * kc.n + i] = best;
}

__global__ __launch_bounds__(BLOCK) void row_extreme_dyn(Consts kc, int D, const double* __restrict__ xc,
                                                         const double* __restrict__ yc,
                                                         const double* __restrict__ a, double sgn,
                                                         double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    row_extreme_dyn_body(kc, D, xc, yc, a, sgn, part, split, sb.bx, sb.p, 0);
}

// Merge the partial minima (exact, order independent); optionally transform.
//   mode 0: out_i = min            (offset init, writes H)
//   mode 1: out_i = xn2_i - 2 min  (squared distance maximum of row i)
__device__ __forceinline__ void row_extreme_merge_body(Consts kc, const double* __restrict__ part, int P,
                                  const double* __restrict__ xn2, int mode,
                                  double* __restrict__ out, int64_t bx_, int64_t by_, int64_t nb_) {
    int64_t i = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double best = part[i];
#pragma unroll 8
    for (int p = 1; p < P; ++p) best = fmin(best, part[(int64_t)p * kc.n + i]);
    out[i] = (mode == 0) ? best : xn2[i] - 2.0 * best;
}

__global__ void row_extreme_merge(Consts kc, const double* __restrict__ part, int P,
                                  const double* __restrict__ xn2, int mode,
                                  double* __restrict__ out) {
    row_extreme_merge_body(kc, part, P, xn2, mode, out, (int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)gridDim.x);
}

// ---------------------------------------------------------------------------
// Row sweep: the two row sums S^A_i, S^B_i with the shared offset h_i.
// part: [P][n] double2.
// ---------------------------------------------------------------------------
// e = a * b + c with c wave-uniform (an SGPR pair).  The VOP3 form takes the
// scalar operand directly; the compiler otherwise copies c into VGPRs for the
// two-address v_fmac_f64 form, costing two extra VALU moves per use.
__device__ __forceinline__ double fma_su(double a, double b, double c_uniform) {
    double e;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(e) : "v"(a), "v"(b), "s"(c_uniform));
    return e;
}

// One column j of the row sweep for this lane's row: returns 2^eA, 2^eB.
template <int M, int D>
__device__ __forceinline__ void row_terms(const double (&x)[D], double h, const double* __restrict__ yj,
                                          double2 g, double cA, double cB, float& pA, float& pB) {
    const double dot = pair_term<M, D>(x, yj, h);
    pA = fexp2(fma_su(dot, cA, g.x));
    pB = fexp2(fma_su(dot, cB, g.y));
}

// The same with the cost term of the B coupling for D_t tracking: tB = 2^eB C_ij / s, with
// C_ij / s = |x~_i|^2 + |y~_j|^2 - 2 P_ij taken from the exponent's dot product
// dot = h + P_ij as (|x~_i|^2 + 2 h + |y~_j|^2) - 2 dot (xa = |x~_i|^2 + 2 h; the norms are
// zero for l1 / l_inf, where P_ij = -dist / 2): two FP64 operations, a conversion and an FMA.
template <int M, int D>
__device__ __forceinline__ void row_terms_dt(const double (&x)[D], double h, double xa, const double* __restrict__ yj,
                                             double yn2j, double2 g, double cA, double cB, float& pA, float& pB,
                                             float& tB) {
    const double dot = pair_term<M, D>(x, yj, h);
    pA = fexp2(fma_su(dot, cA, g.x));
    pB = fexp2(fma_su(dot, cB, g.y));
    const double cs = fma(-2.0, dot, M == METRIC_SQEUCLID ? xa + yn2j : xa);
    tB = pB * (float)cs;
}

// Row sweep body; with DT the sweep also sums the B coupling's cost terms for D_t tracking
// (tpart[p][i], under the same row offset as the B sums, so the splits add up directly).
template <int M, int D, bool DT = false>
__device__ __forceinline__ void row_sweep_body(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                   const double* __restrict__ xc,
                                                   const double* __restrict__ yc,
                                                   const double2* __restrict__ gtab2,
                                                   const double* __restrict__ H,
                                                   double2* __restrict__ part, int64_t split, int64_t bx_, int64_t by_, int64_t nb_,
                                                   const double* __restrict__ xn2 = nullptr,
                                                   const double* __restrict__ yn2 = nullptr,
                                                   double* __restrict__ tpart = nullptr) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;

    const int64_t i = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = xc[ii * D + k];
    const double h = H[ii];

    double sumA = 0.0, sumB = 0.0, sumT = 0.0;
    double xa = 0.0;
    if constexpr (DT) xa = (M == METRIC_SQEUCLID ? xn2[ii] : 0.0) + 2.0 * h;
    const int nfull = (int)((j1 - j0) / UNROLL);
    const double* __restrict__ yp = yc + j0 * D;
    const double2* __restrict__ gp = g + j0;
    const double* __restrict__ np = DT ? yn2 + j0 : nullptr;
    for (int c = 0; c < nfull; ++c, yp += UNROLL * D, gp += UNROLL) {
        float pA[UNROLL], pB[UNROLL], tB[UNROLL];
        if constexpr (DT) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                row_terms_dt<M, D>(x, h, xa, yp + u * D, M == METRIC_SQEUCLID ? np[u] : 0.0, gp[u], cA, cB, pA[u],
                                   pB[u], tB[u]);
            np += UNROLL;
        } else {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) row_terms<M, D>(x, h, yp + u * D, gp[u], cA, cB, pA[u], pB[u]);
        }
        float accA = pA[0], accB = pB[0];
#pragma unroll
        for (int u = 1; u < UNROLL; ++u) {
            accA += pA[u];
            accB += pB[u];
        }
        sumA += (double)accA;
        sumB += (double)accB;
        if constexpr (DT) {
            float accT = tB[0];
#pragma unroll
            for (int u = 1; u < UNROLL; ++u) accT += tB[u];
            sumT += (double)accT;
        }
    }
    {
        const int rem = (int)((j1 - j0) - (int64_t)nfull * UNROLL);
        float accA = 0.f, accB = 0.f, accT = 0.f;
        for (int u = 0; u < rem; ++u) {
            float a, b;
            if constexpr (DT) {
                float tb;
                row_terms_dt<M, D>(x, h, xa, yp + u * D, M == METRIC_SQEUCLID ? np[u] : 0.0, gp[u], cA, cB, a, b,
                                   tb);
                accT += tb;
            } else {
                row_terms<M, D>(x, h, yp + u * D, gp[u], cA, cB, a, b);
            }
            accA += a;
            accB += b;
        }
        sumA += (double)accA;
        sumB += (double)accB;
        sumT += (double)accT;
    }
    if (i < kc.n) {
        part[p * kc.n + i] = make_double2(sumA, sumB);
        if constexpr (DT) tpart[p * kc.n + i] = sumT;
    }
}

template <int M, int D>
__global__ __launch_bounds__(BLOCK) void row_sweep(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                   const double* __restrict__ xc,
                                                   const double* __restrict__ yc,
                                                   const double2* __restrict__ gtab2,
                                                   const double* __restrict__ H,
                                                   double2* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    row_sweep_body<M, D>(ctrl, sched, kc, xc, yc, gtab2, H, part, split, sb.bx, sb.p, 0);
}

// The row sweep of a D_t-tracked iteration: the row sweep above plus the B coupling's cost
// sums, tpart: [P][n].
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void row_sweep_dt(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                      const double* __restrict__ xc,
                                                      const double* __restrict__ yc,
                                                      const double2* __restrict__ gtab2,
                                                      const double* __restrict__ H,
                                                      double2* __restrict__ part, int64_t split,
                                                      const double* __restrict__ xn2,
                                                      const double* __restrict__ yn2,
                                                      double* __restrict__ tpart) {
    const SweepBlock sb = sweep_block(kc.m, split);
    row_sweep_body<M, D, true>(ctrl, sched, kc, xc, yc, gtab2, H, part, split, sb.bx, sb.p, 0, xn2, yn2, tpart);
}

__device__ __forceinline__ void row_sweep_dyn_body(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                                       const double* __restrict__ xc,
                                                       const double* __restrict__ yc,
                                                       const double2* __restrict__ gtab2,
                                                       const double* __restrict__ H,
                                                       double2* __restrict__ part, int64_t split, int64_t bx_, int64_t by_, int64_t nb_) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int64_t i = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    const double h = H[ii];
    double sumA = 0.0, sumB = 0.0;
    for (int64_t jb = j0; jb < j1; jb += UNROLL) {
        float accA = 0.f, accB = 0.f;
        const int64_t je = min(j1, jb + UNROLL);
        for (int64_t j = jb; j < je; ++j) {
            const double dot = pair_term_dyn(kc, D, xc + ii * D, yc + j * D, h);
            accA += fexp2(fma(cA, dot, g[j].x));
            accB += fexp2(fma(cB, dot, g[j].y));
        }
        sumA += (double)accA;
        sumB += (double)accB;
    }
    if (i < kc.n) part[p * kc.n + i] = make_double2(sumA, sumB);
}

__global__ __launch_bounds__(BLOCK) void row_sweep_dyn(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                                       const double* __restrict__ xc,
                                                       const double* __restrict__ yc,
                                                       const double2* __restrict__ gtab2,
                                                       const double* __restrict__ H,
                                                       double2* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    row_sweep_dyn_body(ctrl, sched, kc, D, xc, yc, gtab2, H, part, split, sb.bx, sb.p, 0);
}

// Exact recomputation of sigma_i = log2 sum_j 2^(g_j + cfac x~_i.y~_j) (two passes, FP64 max).
__device__ double exact_sigma(const Consts& kc, const double* __restrict__ xi, const double* __restrict__ yc, int D,
                              const double2* __restrict__ g, int which, double cfac) {
    const int64_t m = kc.m;
    double mx = -__builtin_inf();
    for (int64_t j = 0; j < m; ++j) {
        const double dot = pair_term_dyn(kc, D, xi, yc + j * D, 0.0);
        double e = fma(cfac, dot, which ? g[j].y : g[j].x);
        mx = fmax(mx, e);
    }
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        const double dot = pair_term_dyn(kc, D, xi, yc + j * D, 0.0);
        double e = fma(cfac, dot, which ? g[j].y : g[j].x);
        s += exp2(e - mx);
    }
    return mx + log2(s);
}

// Merge the row partials; derive sigma^A, sigma^B, the next offsets and the
// column-sweep row data; optional natural-log normalisers.
// FP32 row data of the matrix-core column sweep (nullable): {k, w^A, w^B, 0} per row,
// k rounded to FP32 with the rounding error folded exactly into the weights.
// f32_offsets: the row sweep applied (float)H, so that value is the one to subtract.
struct RowVarF32 {
    float4* q;
    int f32_offsets;
};

__device__ __forceinline__ void row_finish_body(Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                           const double* __restrict__ xc, const double* __restrict__ yc,
                           const double2* __restrict__ gtab2, const double* __restrict__ r,
                           const double* __restrict__ xn2, const double2* __restrict__ part, int P,
                           double* __restrict__ H, RowVar* __restrict__ rowvar, double2* __restrict__ rowck,
                           double* __restrict__ log_za, double* __restrict__ log_zb, RowVarF32 rf, int64_t bx_, int64_t by_, int64_t nb_) {
    if (halted(ctrl)) return;
    int64_t i = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    double SA = 0.0, SB = 0.0;
#pragma unroll 8   // independent loads in flight; the sum order is unchanged
    for (int p = 0; p < P; ++p) {
        double2 v = part[(int64_t)p * kc.n + i];
        SA += v.x;
        SB += v.y;
    }
    const double h = rf.f32_offsets ? (double)(float)H[i] : H[i];
    double sigA, sigB;
    const double lo = 0x1p-60, hi = 0x1p+60;
    if (SA >= lo && SA <= hi && SB >= lo && SB <= hi) {
        sigA = log2(SA) - cA * h;
        sigB = log2(SB) - cB * h;
    } else {
        const double2* g = gtab2 + (t & 1) * kc.m;
        sigA = exact_sigma(kc, xc + i * D, yc, D, g, 0, cA);
        sigB = exact_sigma(kc, xc + i * D, yc, D, g, 1, cB);
        atomicAdd(&ctrl->fallbacks, 1);
    }
    const double hnew = -sigB / cB;
    const double rho = cA / cB;
    double ew = rho * sigB - sigA;
    ew = fmin(fmax(ew, -1000.0), 1000.0);
    H[i] = hnew;
    // The column sweeps that take FP32 row weights see the A factor 2^ew in w^A; a row with
    // |ew| > 100 (large tau1: ew grows with K tau1 (theta - nu)) moves their shared offset by
    // dl = ew / (c^A + c^B), which leaves |ew| / (1 + rho) in each weight's exponent
    // (w^A 2^(c^A (x.y + k)) and w^B 2^(c^B (x.y + k)) are unchanged).
    double kw = hnew, ea = ew, eb = 0.0;
    if (fabs(ew) > 100.0) {
        const double dl = ew / (cA + cB);
        kw = hnew + dl;
        ea = ew - cA * dl;
        eb = -cB * dl;
    }
    RowVar rv;
    rv.k = kw;
    rv.wA = (float)(r[i] * exp2(ea));
    rv.wB = (float)(r[i] * exp2(eb));
    rowvar[i] = rv;
    // the vector-ALU column sweep takes the row weights into its exponents: the A coupling's
    // row factor 2^ew (unclamped: no FP32 weight to overflow) and n r_i (1 for uniform r; the
    // sweep multiplies its sums by 1/n)
    if (rowck) {
        const double lw = log2((double)kc.n * r[i]);
        rowck[i] = make_double2(cA * hnew + (rho * sigB - sigA) + lw, cB * hnew + lw);
    }
    if (rf.q) {
        const float kf = (float)kw;
        const double dk = kw - (double)kf;
        const float wa = (float)(r[i] * exp2(fmin(fmax(ea + cA * dk, -1000.0), 1000.0)));
        const float wb = (float)(r[i] * exp2(eb + cB * dk));
        rf.q[i] = make_float4(kf, wa, wb, 0.f);
    }
    if (log_za) log_za[i] = LN2 * (-sc.lamA * LOG2E * kc.s * xn2[i] + sigA);
    if (log_zb) log_zb[i] = LN2 * (-sc.lamB * LOG2E * kc.s * xn2[i] + sigB);
}

__global__ void row_finish(Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                           const double* __restrict__ xc, const double* __restrict__ yc,
                           const double2* __restrict__ gtab2, const double* __restrict__ r,
                           const double* __restrict__ xn2, const double2* __restrict__ part, int P,
                           double* __restrict__ H, RowVar* __restrict__ rowvar, double2* __restrict__ rowck,
                           double* __restrict__ log_za, double* __restrict__ log_zb, RowVarF32 rf) {
    row_finish_body(ctrl, sched, kc, D, xc, yc, gtab2, r, xn2, part, P, H, rowvar, rowck, log_za, log_zb, rf, (int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)gridDim.x);
}

// ---------------------------------------------------------------------------
// Column sweep: col^A_j, col^B_j.  cpart: [P][m] double2.
// ---------------------------------------------------------------------------
// One row i of the column sweep for this lane's column.  With k_i the row's offset,
// ew_i = rho sigma^B_i - sigma^A_i the A coupling's row factor and G_j = g^B_j / cfac^B this
// column's term, the base-2 exponents of the normalised couplings are
//     e^B = cfac^B (P_ij + G_j) + cfac^B k_i,
//     e^A = cfac^A (P_ij + G_j) + (cfac^A k_i + ew_i) + D_j,   D_j = g^A_j - cfac^A G_j:
// the dot product starts from G_j (per lane), the row terms come precomputed (rowck,
// scalar, with the row weight as log2(n r_i) in both), and D_j, constant down the column,
// is applied once to the column's A sum (`factor`) or added to each exponent; the sums are
// plain FP32 adds, multiplied by 1/n at the end.
template <int M, int D, bool FACTOR>
__device__ __forceinline__ void col_terms(const double (&y)[D], const double* __restrict__ xi, double2 ck,
                                          double G, double Dj, double cA, double cB, float& accA, float& accB) {
    const double dot = pair_term<M, D>(y, xi, G);   // the distances are symmetric
    double eA = fma_su(dot, cA, ck.x);
    if constexpr (!FACTOR) eA += Dj;
    accA += fexp2(eA);
    accB += fexp2(fma_su(dot, cB, ck.y));
}

template <int M, int D, bool FACTOR>
__device__ __forceinline__ void col_sweep_run(double cA, double cB, const double (&y)[D], double G, double Dj,
                                              const double* __restrict__ xc, const double2* __restrict__ rowck,
                                              int64_t i0, int64_t i1, double& sumA, double& sumB) {
    const int nfull = (int)((i1 - i0) / UNROLL);
    const double* __restrict__ xp = xc + i0 * D;
    const double2* __restrict__ kp = rowck + i0;
    for (int c = 0; c < nfull; ++c, xp += UNROLL * D, kp += UNROLL) {
        float accA = 0.f, accB = 0.f;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) col_terms<M, D, FACTOR>(y, xp + u * D, kp[u], G, Dj, cA, cB, accA, accB);
        sumA += (double)accA;
        sumB += (double)accB;
    }
    const int rem = (int)((i1 - i0) - (int64_t)nfull * UNROLL);
    float accA = 0.f, accB = 0.f;
    for (int u = 0; u < rem; ++u) col_terms<M, D, FACTOR>(y, xp + u * D, kp[u], G, Dj, cA, cB, accA, accB);
    sumA += (double)accA;
    sumB += (double)accB;
}

template <int M, int D>
__device__ __forceinline__ void col_sweep_body(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                   const double* __restrict__ xc,
                                                   const double* __restrict__ yc,
                                                   const double2* __restrict__ gtab2,
                                                   const RowVar* __restrict__ rowvar,
                                                   const double2* __restrict__ rowck,
                                                   double2* __restrict__ cpart, int64_t split, int64_t bx_, int64_t by_, int64_t nb_) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const int64_t j = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    const int64_t jj = j < kc.m ? j : kc.m - 1;
    double y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = yc[jj * D + k];
    const double2 g = gtab2[(t & 1) * kc.m + jj];
    const double G = g.y / cB;
    const double Dj = g.x - cA * G;

    double sumA = 0.0, sumB = 0.0;
    const double inv_n = 1.0 / (double)kc.n;   // the row weights r_i enter as n r_i (rowck)
    if (kc.factor_cols) {
        col_sweep_run<M, D, true>(cA, cB, y, G, Dj, xc, rowck, i0, i1, sumA, sumB);
        sumA *= exp2(Dj) * inv_n;
    } else {
        col_sweep_run<M, D, false>(cA, cB, y, G, Dj, xc, rowck, i0, i1, sumA, sumB);
        sumA *= inv_n;
    }
    sumB *= inv_n;
    if (j < kc.m) cpart[p * kc.m + j] = make_double2(sumA, sumB);
}

template <int M, int D>
__global__ __launch_bounds__(BLOCK) void col_sweep(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                   const double* __restrict__ xc,
                                                   const double* __restrict__ yc,
                                                   const double2* __restrict__ gtab2,
                                                   const RowVar* __restrict__ rowvar,
                                                   const double2* __restrict__ rowck,
                                                   double2* __restrict__ cpart, int64_t split) {
    const SweepBlock sb = sweep_block(kc.n, split);
    col_sweep_body<M, D>(ctrl, sched, kc, xc, yc, gtab2, rowvar, rowck, cpart, split, sb.bx, sb.p, 0);
}

__device__ __forceinline__ void col_sweep_dyn_body(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                                       const double* __restrict__ xc,
                                                       const double* __restrict__ yc,
                                                       const double2* __restrict__ gtab2,
                                                       const RowVar* __restrict__ rowvar,
                                                       const double2* __restrict__ rowck,
                                                       double2* __restrict__ cpart, int64_t split, int64_t bx_, int64_t by_, int64_t nb_) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const int64_t j = (int64_t)bx_ * BLOCK + threadIdx.x;
    const int64_t p = by_;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    const int64_t jj = j < kc.m ? j : kc.m - 1;
    const double2 g = gtab2[(t & 1) * kc.m + jj];
    const double G = g.y / cB;   // the exponent assembly of col_terms
    const double Dj = g.x - cA * G;
    double sumA = 0.0, sumB = 0.0;
    for (int64_t ib = i0; ib < i1; ib += UNROLL) {
        float accA = 0.f, accB = 0.f;
        const int64_t ie = min(i1, ib + UNROLL);
        for (int64_t i = ib; i < ie; ++i) {
            const double2 ck = rowck[i];
            const double dot = pair_term_dyn(kc, D, yc + jj * D, xc + i * D, G);
            double eA = fma(dot, cA, ck.x);
            if (!kc.factor_cols) eA += Dj;
            accA += fexp2(eA);
            accB += fexp2(fma(dot, cB, ck.y));
        }
        sumA += (double)accA;
        sumB += (double)accB;
    }
    const double inv_n = 1.0 / (double)kc.n;
    sumA *= (kc.factor_cols ? exp2(Dj) : 1.0) * inv_n;
    sumB *= inv_n;
    if (j < kc.m) cpart[p * kc.m + j] = make_double2(sumA, sumB);
}

__global__ __launch_bounds__(BLOCK) void col_sweep_dyn(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                                       const double* __restrict__ xc,
                                                       const double* __restrict__ yc,
                                                       const double2* __restrict__ gtab2,
                                                       const RowVar* __restrict__ rowvar,
                                                       const double2* __restrict__ rowck,
                                                       double2* __restrict__ cpart, int64_t split) {
    const SweepBlock sb = sweep_block(kc.n, split);
    col_sweep_dyn_body(ctrl, sched, kc, D, xc, yc, gtab2, rowvar, rowck, cpart, split, sb.bx, sb.p, 0);
}

// ---------------------------------------------------------------------------
// D_t tracking (Proposition infeas_bound(b)): <C, Xbar^{t+1}> of the second coupling
// of iteration t, Xbar^{t+1} = diag(r) p^{eta_{t+1}}(nubar^{t+1}).  Per row, with the
// row sweep's offset h_i and column table g^B:
//     S_i = sum_j 2^(cB (h_i + P_ij) + g^B_j),   T_i = sum_j 2^(...) C_ij,
//     out_i = r_i T_i / S_i  (the normaliser cancels),  C_ij = s (|x~_i|^2 + |y~_j|^2 - 2 P_ij).
// Same arithmetic as the row sweep (FP64 exponent, FP32 exponential and per-block
// sums, FP64 across blocks); one thread per row over all columns.
// ---------------------------------------------------------------------------
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void dt_cost_rows(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                      const double* __restrict__ xc,
                                                      const double* __restrict__ yc,
                                                      const double* __restrict__ xn2,
                                                      const double* __restrict__ yn2,
                                                      const double2* __restrict__ gtab2,
                                                      const double* __restrict__ H,
                                                      const double* __restrict__ r,
                                                      double* __restrict__ out) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = xc[ii * D + k];
    const double h = H[ii];
    const double xa = kc.s * xn2[ii];
    double S = 0.0, T = 0.0;
    for (int64_t jb = 0; jb < kc.m; jb += UNROLL) {
        float aS = 0.f, aT = 0.f;
        const int64_t je = min(kc.m, jb + UNROLL);
        for (int64_t j = jb; j < je; ++j) {
            const double dot = pair_term<M, D>(x, yc + j * D, 0.0);
            const float p = fexp2(fma(cB, h + dot, g[j].y));
            const double cij = fma(-2.0 * kc.s, dot, xa + kc.s * yn2[j]);
            aS += p;
            aT = fmaf(p, (float)cij, aT);
        }
        S += (double)aS;
        T += (double)aT;
    }
    if (i < kc.n) out[i] = r[i] * T / S;
}

__global__ __launch_bounds__(BLOCK) void dt_cost_rows_dyn(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                                          const double* __restrict__ xc,
                                                          const double* __restrict__ yc,
                                                          const double* __restrict__ xn2,
                                                          const double* __restrict__ yn2,
                                                          const double2* __restrict__ gtab2,
                                                          const double* __restrict__ H,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ out) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    const double h = H[ii];
    const double xa = kc.s * xn2[ii];
    double S = 0.0, T = 0.0;
    for (int64_t jb = 0; jb < kc.m; jb += UNROLL) {
        float aS = 0.f, aT = 0.f;
        const int64_t je = min(kc.m, jb + UNROLL);
        for (int64_t j = jb; j < je; ++j) {
            const double dot = pair_term_dyn(kc, D, xc + ii * D, yc + j * D, 0.0);
            const float p = fexp2(fma(cB, h + dot, g[j].y));
            const double cij = fma(-2.0 * kc.s, dot, xa + kc.s * yn2[j]);
            aS += p;
            aT = fmaf(p, (float)cij, aT);
        }
        S += (double)aS;
        T += (double)aT;
    }
    if (i < kc.n) out[i] = r[i] * T / S;
}

// Row i's share of <C, Xbar^{t+1}> from the D_t-tracked row sweep's splits: s r_i T_i / S^B_i
// (both sums under the row's offset h_i, so the splits add directly).  A row whose S^B leaves
// [2^-60, 2^60] -- the rows whose normalisers row_finish recomputes -- is evaluated again in
// FP64 under its exact largest exponent.
// pair(j) = P(x_i, y_j); sq: squared Euclidean (the norms enter the cost).
template <typename Pair>
__device__ __forceinline__ void dt_rows_finish_body(const Ctrl* ctrl, const Sched* sched, Consts kc, bool sq,
                                                    const double* __restrict__ xn2, const double* __restrict__ yn2,
                                                    const double2* __restrict__ gtab2, const double* __restrict__ r,
                                                    const double2* __restrict__ part,
                                                    const double* __restrict__ tpart, int P, int64_t i,
                                                    double* __restrict__ out, Pair&& pair) {
    double SB = 0.0, T = 0.0;
#pragma unroll 8   // independent loads in flight; the sum order is unchanged
    for (int p = 0; p < P; ++p) {
        SB += part[(int64_t)p * kc.n + i].y;
        T += tpart[(int64_t)p * kc.n + i];
    }
    if (SB >= 0x1p-60 && SB <= 0x1p+60) {
        out[i] = kc.s * r[i] * (T / SB);
        return;
    }
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    double emax = -__builtin_inf();
    for (int64_t j = 0; j < kc.m; ++j) emax = fmax(emax, fma(cB, pair(j), g[j].y));
    const double xa = sq ? xn2[i] : 0.0;
    double S = 0.0, Tx = 0.0;
    for (int64_t j = 0; j < kc.m; ++j) {
        const double dot = pair(j);
        const double q = exp2(fma(cB, dot, g[j].y) - emax);
        S += q;
        Tx += q * fma(-2.0, dot, sq ? xa + yn2[j] : xa);
    }
    out[i] = kc.s * r[i] * (Tx / S);
}

template <int M, int D>
__global__ void dt_rows_finish(const Ctrl* ctrl, const Sched* sched, Consts kc, const double* __restrict__ xc,
                               const double* __restrict__ yc, const double* __restrict__ xn2,
                               const double* __restrict__ yn2, const double2* __restrict__ gtab2,
                               const double* __restrict__ r, const double2* __restrict__ part,
                               const double* __restrict__ tpart, int P, double* __restrict__ out) {
    if (halted(ctrl)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = xc[i * D + k];
    dt_rows_finish_body(ctrl, sched, kc, M == METRIC_SQEUCLID, xn2, yn2, gtab2, r, part, tpart, P, i, out,
                        [&](int64_t j) { return pair_term<M, D>(x, yc + j * D, 0.0); });
}

// The same with the metric and the dimension at run time (the FP64 matrix-core sweeps).
__global__ void dt_rows_finish_dyn(const Ctrl* ctrl, const Sched* sched, Consts kc, int D,
                                   const double* __restrict__ xc, const double* __restrict__ yc,
                                   const double* __restrict__ xn2, const double* __restrict__ yn2,
                                   const double2* __restrict__ gtab2, const double* __restrict__ r,
                                   const double2* __restrict__ part, const double* __restrict__ tpart, int P,
                                   double* __restrict__ out) {
    if (halted(ctrl)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const double* __restrict__ xi = xc + i * D;
    dt_rows_finish_body(ctrl, sched, kc, kc.metric == METRIC_SQEUCLID, xn2, yn2, gtab2, r, part, tpart, P, i, out,
                        [&](int64_t j) { return pair_term_dyn(kc, D, xi, yc + j * D, 0.0); });
}

// ctrl->dt_cost = sum_i out_i, one block, fixed order (deterministic).
__global__ __launch_bounds__(1024) void dt_cost_total(Ctrl* ctrl, const double* __restrict__ vals, int64_t n) {
    if (halted(ctrl)) return;
    __shared__ double sh[1024];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) a += vals[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctrl->dt_cost = sh[0];
}

// ---------------------------------------------------------------------------
// Dual update (S5-S6 of Algorithm 2), residual, next column table, stop flag.
// State is double-buffered by iteration parity: iteration t reads buffer t&1 and
// writes buffer (t+1)&1, so the iterate that met the tolerance is never
// overwritten.
// ---------------------------------------------------------------------------
// Dual part of the D_t summand for one column, from the natural parameters of the mirror
// steps (thetabar = tanh abar, thetahat = tanh ahat, theta^t = tanh a):
//   D(thetabar||thetahat) - D(thetabar||theta^t)  per coordinate of def:DHa_explicit, with
//   (1 + tanh x)/2 = sigma(2x), is  2 sigma(2 abar) (a - ahat) + softplus(2 ahat) - softplus(2 a):
// exact where tanh rounds to +-1 (a step with c^alpha_j ~ alpha/m and |col_j - c_j| >> c^alpha_j).
__device__ __forceinline__ double softplus(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }

__device__ __forceinline__ double dual_dt_term(double abar, double ahat, double a) {
    const double sig = 0.5 * (1.0 + tanh(abar));   // sigma(2 abar)
    return 2.0 * sig * (a - ahat) + softplus(2.0 * ahat) - softplus(2.0 * a);
}

struct DualBufs {
    double* nu[2];
    double* theta[2];
};

struct TraceCols {
    double *col_a, *col_b, *theta_bar, *theta_hat;
};

__device__ __forceinline__ void dual_update_body(Ctrl* ctrl, const Sched* sched, Consts kc,
                                                     const double2* __restrict__ cpart, int P,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ yn2, DualBufs buf,
                                                     double2* __restrict__ gtab2,
                                                     float2* __restrict__ gtabf, int64_t m_pad,
                                                     double* __restrict__ respart, TraceCols tr,
                                                     double* __restrict__ dtpart, int64_t bx_) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const int64_t j = (int64_t)bx_ * BLOCK + threadIdx.x;
    double res = 0.0, dtj = 0.0;
    int bad = 0;
    if (j < kc.m) {
        double colA = 0.0, colB = 0.0;
#pragma unroll 8   // independent loads in flight; the sum order is unchanged
        for (int p = 0; p < P; ++p) {
            double2 v = cpart[(int64_t)p * kc.m + j];
            colA += v.x;
            colB += v.y;
        }
        const double* nu_r = buf.nu[t & 1];
        const double* th_r = buf.theta[t & 1];
        double* nu_w = buf.nu[(t + 1) & 1];
        double* th_w = buf.theta[(t + 1) & 1];
        const double cj = c[j];
        const double calpha = cj + kc.alpha_m;       // c^alpha = c + (alpha/m) 1
        const double nu = nu_r[j], th = th_r[j];
        const double a = atanh(th);
        // closed form of the dual mirror map (def:closed_form_opt)
        const double abar = a + kc.kappa * (colA - cj) / calpha;
        const double ahat = a + kc.kappa * (colB - cj) / calpha;
        const double tbar = tanh(abar);
        const double that = tanh(ahat);
        const double nun = nu + sc.w * (tbar - nu);            // step:lamp_main_nu
        const double thn = fmin(fmax(that, -kc.clipb), kc.clipb);  // tclip
        nu_w[j] = nun;
        th_w[j] = thn;
        // column table of iteration t+1
        const double nbn = nun + sc.w2 * (thn - nun);          // step:lamp_mid_nu at t+1
        const double base = kc.s * yn2[j];
        double2 gn;
        gn.x = -sc.lamB * LOG2E * (base + kc.K * nun);
        gn.y = -sc.lamC * LOG2E * (base + kc.K * nbn);
        gtab2[((t + 1) & 1) * kc.m + j] = gn;
        if (gtabf) gtabf[((t + 1) & 1) * m_pad + j] = make_float2((float)gn.x, (float)gn.y);
        res = fabs(colA - cj);
        bad = !(isfinite(nun) && isfinite(thn) && isfinite(colA) && isfinite(colB)) || fabs(th) >= 1.0;
        if (dtpart) {
            // D_t summand of this column (Lemma kl_diff, def:DHa_explicit):
            // c^a (D(tbar||that) - D(tbar||th)) + K colB (lam_{t+1} nu^{t+1} - lam_t nu^t)
            dtj = calpha * dual_dt_term(abar, ahat, a) + kc.K * colB * (sc.lamB * nun - sc.lamA * nu);
        }
        if (tr.col_a) tr.col_a[j] = colA;
        if (tr.col_b) tr.col_b[j] = colB;
        if (tr.theta_bar) tr.theta_bar[j] = tbar;
        if (tr.theta_hat) tr.theta_hat[j] = that;
    }
    // block reduction of the residual (and D_t summand; fixed order: deterministic)
    __shared__ double sh[BLOCK];
    __shared__ double shd[BLOCK];
    __shared__ int shbad;
    if (threadIdx.x == 0) shbad = 0;
    __syncthreads();
    if (bad) atomicOr(&shbad, 1);
    sh[threadIdx.x] = res;
    shd[threadIdx.x] = dtj;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            shd[threadIdx.x] += shd[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        respart[bx_] = sh[0];
        if (dtpart) dtpart[bx_] = shd[0];
        if (shbad) atomicOr(&ctrl->err, 1);
    }
}

// Completes iteration t after the dual update (a kernel of its own: the block partials are
// visible at the kernel boundary, so the dual update needs no device-scope fence and no
// last-block counter -- on a chip whose XCDs keep separate L2 caches every such fence writes
// back the L2).  One block: the residual ||col(X^t) - c||_1 as a fixed-order tree over the
// block partials, the stop decision (iterates t >= 1 only; t = 0 is the product coupling of
// eta_0 = infinity), and otherwise the D_t summand of the step and t + 1.
__device__ __forceinline__ void dual_finish_body(Ctrl* ctrl, const Sched* sched, const double* __restrict__ respart,
                                                 const double* __restrict__ dtpart, int64_t nb) {
    if (halted(ctrl)) return;   // the same control block for every thread: uniform
    const int64_t t = ctrl->t;
    __shared__ double sh[BLOCK];
    __shared__ double shd[BLOCK];
    double a = 0.0, b = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += BLOCK) {
        a += respart[k];
        if (dtpart) b += dtpart[k];
    }
    sh[threadIdx.x] = a;
    shd[threadIdx.x] = b;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            shd[threadIdx.x] += shd[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double tot = sh[0];
    ctrl->res_last = tot;
    if (ctrl->err) {
        ctrl->done = 1;
        ctrl->t_done = t;
    } else if (ctrl->tol > 0.0 && t >= 1 && tot <= ctrl->tol) {
        ctrl->done = 1;
        ctrl->t_done = t;
    } else {
        if (dtpart) {
            // the step is taken: its D_t summand joins the sum
            const Sched sc = sched[t - ctrl->t_base];
            ctrl->dt_acc += (sc.lamB - sc.lamA) * ctrl->dt_cost + shd[0];
        }
        ctrl->t = t + 1;
    }
}

__global__ __launch_bounds__(BLOCK) void dual_finish(Ctrl* ctrl, const Sched* sched, const double* __restrict__ respart,
                                                     const double* __restrict__ dtpart, int64_t nb) {
    dual_finish_body(ctrl, sched, respart, dtpart, nb);
}

__global__ __launch_bounds__(BLOCK) void dual_update(Ctrl* ctrl, const Sched* sched, Consts kc,
                                                     const double2* __restrict__ cpart, int P,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ yn2, DualBufs buf,
                                                     double2* __restrict__ gtab2,
                                                     float2* __restrict__ gtabf, int64_t m_pad,
                                                     double* __restrict__ respart, TraceCols tr,
                                                     double* __restrict__ dtpart) {
    dual_update_body(ctrl, sched, kc, cpart, P, c, yn2, buf, gtab2, gtabf, m_pad, respart, tr, dtpart, (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Deterministic single-block reductions.
// ---------------------------------------------------------------------------
// out[k] = sum_i v_k(i) for the certificate: mode selects the terms.
__global__ void reduce_max(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
    __shared__ double sh[1024];
    double best = -__builtin_inf();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) best = fmax(best, v[i]);
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// sums[q] = sum_i vals[q * stride + i] for q < Q (each a fixed-order tree).
__global__ void reduce_sums(const double* __restrict__ vals, int64_t n, int64_t stride, int Q,
                            double* __restrict__ out) {
    __shared__ double sh[1024];
    for (int q = 0; q < Q; ++q) {
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += vals[q * stride + i];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// Checks of a marginal a[0..len) in one block: out[0] = sum (fixed order), out[1] = the
// first index whose entry is not a positive finite number (-1: none), out[2] = that entry.
__global__ void marginal_stats(const double* __restrict__ a, int64_t len, double* __restrict__ out) {
    __shared__ double sh[1024];
    __shared__ long long bad[1024];
    double acc = 0.0;
    long long first = -1;
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
        const double v = a[i];
        acc += v;
        if (first < 0 && !(v > 0.0 && v <= 1.7976931348623157e308)) first = (long long)i;
    }
    sh[threadIdx.x] = acc;
    bad[threadIdx.x] = first;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            const long long b = bad[threadIdx.x + o];
            if (b >= 0 && (bad[threadIdx.x] < 0 || b < bad[threadIdx.x])) bad[threadIdx.x] = b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0];
        out[1] = (double)bad[0];
        out[2] = bad[0] >= 0 ? a[bad[0]] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// The pair term of the thread's own point against streamed points: coordinates in
// registers for a compile-time dimension (M, D), read from memory for the run-time
// metric and dimension (M = -1, D = 0).  The pair term is symmetric in its points.
// ---------------------------------------------------------------------------
template <int M, int D>
struct OwnPoint {
    double x[D];
    __device__ __forceinline__ OwnPoint(const double* __restrict__ src, int, const Consts&) {
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = src[k];
    }
    __device__ __forceinline__ double pair(const double* __restrict__ y) const { return pair_term<M, D>(x, y, 0.0); }
};

template <>
struct OwnPoint<-1, 0> {
    const double* x;
    int d;
    Consts kc;
    __device__ __forceinline__ OwnPoint(const double* __restrict__ src, int d_, const Consts& kc_)
        : x(src), d(d_), kc(kc_) {}
    __device__ __forceinline__ double pair(const double* __restrict__ y) const {
        return pair_term_dyn(kc, d, x, y, 0.0);
    }
};

// ---------------------------------------------------------------------------
// Certificate row sweep at the state's iterate (offsets from an A-only
// row_finish so that log2 p_ij = cfac (h_i + x~.y~) + g_j exactly):
//   vals[0][i] = r_i |sum_j p_ij - 1|                 (row infeasibility)
//   vals[1][i] = r_i sum_j C_ij p_ij                  (<C, X^t>)
//   vals[2][i] = r_i min_j (C_ij + K theta_j)         (D(theta), def:dual_spp)
//   vals[3][i] = r_i min_j (C_ij + K nu_j)            (D(nu))
//   psum_out[i] = sum_j p_ij                          (row sum of p, for Round)
// Terms as in the sweeps: FP64 exponent, FP32 exponential and sums over blocks of
// UNROLL columns, FP64 across blocks; the two minima in FP64.  Dm = run-time d.  Over XCD-aware
// column splits (sweep_block): part[p][i] = (sum_j p_ij, sum_j C_ij p_ij, the two minima) of
// split p, combined in order by cert_rows_merge.
// ---------------------------------------------------------------------------
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void cert_rows(Consts kc, int Dm, double cA,
                                                   const double* __restrict__ xc,
                                                   const double* __restrict__ yc,
                                                   const double* __restrict__ xn2,
                                                   const double* __restrict__ yn2,
                                                   const double* __restrict__ gA,
                                                   const double* __restrict__ H,
                                                   const double* __restrict__ nu,
                                                   const double* __restrict__ theta,
                                                   double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    if (i >= kc.n) return;
    const int64_t j0 = sb.p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const OwnPoint<M, D> own(xc + i * Dm, Dm, kc);
    const double h = H[i];
    double psum = 0.0, csum = 0.0, mth = __builtin_inf(), mnu = __builtin_inf();
    for (int64_t jb = j0; jb < j1; jb += UNROLL) {
        const int64_t je = min(j1, jb + UNROLL);
        float ap = 0.f, ac = 0.f;
        for (int64_t j = jb; j < je; ++j) {
            const double dot = own.pair(yc + j * Dm);
            const float p = fexp2(fma(cA, h + dot, gA[j]));
            const double cij = kc.s * (xn2[i] + yn2[j] - 2.0 * dot);
            ap += p;
            ac = fmaf((float)cij, p, ac);
            mth = fmin(mth, cij + kc.K * theta[j]);
            mnu = fmin(mnu, cij + kc.K * nu[j]);
        }
        psum += (double)ap;
        csum += (double)ac;
    }
    double* o = part + (sb.p * kc.n + i) * 4;
    o[0] = psum;
    o[1] = csum;
    o[2] = mth;
    o[3] = mnu;
}

// The splits of the certificate row pass in order: the two sums added, the minima taken;
// mu (2 x n) keeps the minima for the entropic pass.
__global__ void cert_rows_merge(Consts kc, int P, const double* __restrict__ r, const double* __restrict__ part,
                                double* __restrict__ vals, double* __restrict__ psum_out, double* __restrict__ mu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double psum = 0.0, csum = 0.0, mth = __builtin_inf(), mnu = __builtin_inf();
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        const double* o = part + ((int64_t)p * kc.n + i) * 4;
        psum += o[0];
        csum += o[1];
        mth = fmin(mth, o[2]);
        mnu = fmin(mnu, o[3]);
    }
    const double ri = r[i];
    vals[i] = ri * fabs(psum - 1.0);
    vals[kc.n + i] = ri * csum;
    vals[2 * kc.n + i] = ri * mth;
    vals[3 * kc.n + i] = ri * mnu;
    psum_out[i] = psum;
    mu[i] = mth;
    mu[kc.n + i] = mnu;
}

// ---------------------------------------------------------------------------
// Entropic dual values at eta = 1/lam > 0 (def:dual_spp_e): per row i and dual v in {theta, nu},
//   softmin_i(v) = mu_i - eta ln sum_j exp(-(C_ij + K v_j - mu_i) / eta),  mu_i = min_j (C_ij + K v_j),
// with the minimum exact in FP64 (from the certificate row pass), the terms (each <= 1, one of
// them 1) FP32 exponentials of FP64 arguments summed in FP32 over blocks of UNROLL columns and in
// FP64 across them and across the splits (in order).
//   part[p][i] = (split p's sum for theta, for nu);  vals[0][i] = r_i softmin_i(theta), vals[1][i] likewise.
// ---------------------------------------------------------------------------
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void cert_soft_rows(Consts kc, int Dm, double lam,
                                                        const double* __restrict__ xc,
                                                        const double* __restrict__ yc,
                                                        const double* __restrict__ xn2,
                                                        const double* __restrict__ yn2,
                                                        const double* __restrict__ nu,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ mu,
                                                        double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    if (i >= kc.n) return;
    const int64_t j0 = sb.p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const OwnPoint<M, D> own(xc + i * Dm, Dm, kc);
    const double mth = mu[i], mnu = mu[kc.n + i];
    const double f = -lam * LOG2E;
    double sth = 0.0, snu = 0.0;
    for (int64_t jb = j0; jb < j1; jb += UNROLL) {
        const int64_t je = min(j1, jb + UNROLL);
        float at = 0.f, an = 0.f;
        for (int64_t j = jb; j < je; ++j) {
            const double cij = kc.s * (xn2[i] + yn2[j] - 2.0 * own.pair(yc + j * Dm));
            at += fexp2(f * (cij + kc.K * theta[j] - mth));
            an += fexp2(f * (cij + kc.K * nu[j] - mnu));
        }
        sth += (double)at;
        snu += (double)an;
    }
    double* o = part + (sb.p * kc.n + i) * 2;
    o[0] = sth;
    o[1] = snu;
}

__global__ void cert_soft_merge(Consts kc, int P, double lam, const double* __restrict__ r,
                                const double* __restrict__ mu, const double* __restrict__ part,
                                double* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double sth = 0.0, snu = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        sth += part[((int64_t)p * kc.n + i) * 2];
        snu += part[((int64_t)p * kc.n + i) * 2 + 1];
    }
    const double ri = r[i];
    vals[i] = ri * (mu[i] - log(sth) / lam);
    vals[kc.n + i] = ri * (mu[kc.n + i] - log(snu) / lam);
}

// ---------------------------------------------------------------------------
// Round (Algorithm 3) of the same X = diag(r) p on the device, without forming it:
//   step 1  xr_i = min(r_i / row_i(X), 1) = min(1 / sum_j p_ij, 1)
//   step 2  X' = diag(xr) X;  y_j = min(c_j / col_j(X'), 1);  X'' = X' diag(y)
//   step 3  dr = r - row(X''),  dc = c - col(X'') = c - y * col(X')
//   step 4  Round(X) = X'' + dr dc^T / ||dr||_1
// so that <C, Round(X)> = <C, X''> + dr^T C dc / ||dr||_1, where for the squared
// Euclidean cost on centred points
//   (C dc)_i = s (||x~_i||^2 sum_j dc_j + sum_j dc_j ||y~_j||^2 - 2 x~_i . sum_j dc_j y~_j)
// is O(d) per row once the column sums are known.  The pair passes use the terms of
// the certificate row sweep (FP32 exponentials, FP64 sums), the O(n + m) steps FP64.
// ---------------------------------------------------------------------------
__global__ void round_row_factors(Consts kc, const double* __restrict__ psum, double* __restrict__ xr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kc.n) xr[i] = fmin(1.0 / psum[i], 1.0);
}

// part[p][j] = sum over the rows i of split p of xr_i r_i p_ij (one thread per
// column, rows in order); round_cols_merge adds the splits in order: colp_j.
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void round_cols(Consts kc, int Dm, double cA, const double* __restrict__ xc,
                                                    const double* __restrict__ yc, const double* __restrict__ gA,
                                                    const double* __restrict__ H, const double* __restrict__ r,
                                                    const double* __restrict__ xr, double* __restrict__ part,
                                                    int64_t split) {
    const SweepBlock sb = sweep_block(kc.n, split);
    const int64_t j = sb.bx * BLOCK + threadIdx.x;
    if (j >= kc.m) return;
    const int64_t p = sb.p;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    const OwnPoint<M, D> own(yc + j * Dm, Dm, kc);
    const double g = gA[j];
    double acc = 0.0;
    for (int64_t ib = i0; ib < i1; ib += UNROLL) {
        const int64_t ie = min(i1, ib + UNROLL);
        float a = 0.f;
        for (int64_t i = ib; i < ie; ++i) {
            const double dot = own.pair(xc + i * Dm);
            a = fmaf((float)(xr[i] * r[i]), fexp2(fma(cA, H[i] + dot, g)), a);
        }
        acc += (double)a;
    }
    part[p * kc.m + j] = acc;
}

__global__ void round_cols_merge(Consts kc, const double* __restrict__ part, int P, double* __restrict__ colp) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    double a = part[j];
    for (int p = 1; p < P; ++p) a += part[(int64_t)p * kc.m + j];
    colp[j] = a;
}

// y_j = min(c_j / colp_j, 1) and dc_j = c_j - y_j colp_j.
__global__ void round_col_factors(Consts kc, const double* __restrict__ c, const double* __restrict__ colp,
                                  double* __restrict__ y, double* __restrict__ dc) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    const double yj = colp[j] > 0.0 ? fmin(c[j] / colp[j], 1.0) : 1.0;
    y[j] = yj;
    dc[j] = c[j] - yj * colp[j];
}

// Rows of X'': dr_i = r_i - xr_i r_i sum_j p_ij y_j and cpp_i = xr_i r_i sum_j C_ij p_ij y_j.
// dr is formed as r_i (1 - xr_i psum_i) + xr_i r_i sum_j p_ij (1 - y_j) (the same value)
// with psum_i recomputed in this pass: no difference of two nearly equal sums.  Over XCD-aware
// column splits: part[p][i] = split p's three sums, combined in order by round_rows_merge.
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void round_rows(Consts kc, int Dm, double cA, const double* __restrict__ xc,
                                                    const double* __restrict__ yc, const double* __restrict__ xn2,
                                                    const double* __restrict__ yn2, const double* __restrict__ gA,
                                                    const double* __restrict__ H, const double* __restrict__ y,
                                                    double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    if (i >= kc.n) return;
    const int64_t j0 = sb.p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const OwnPoint<M, D> own(xc + i * Dm, Dm, kc);
    const double h = H[i];
    double ps = 0.0, pq = 0.0, cs = 0.0;
    for (int64_t jb = j0; jb < j1; jb += UNROLL) {
        const int64_t je = min(j1, jb + UNROLL);
        float a = 0.f, b = 0.f, e = 0.f;
        for (int64_t j = jb; j < je; ++j) {
            const double dot = own.pair(yc + j * Dm);
            const float p = fexp2(fma(cA, h + dot, gA[j]));
            const double yj = y[j];
            const float py = p * (float)yj;
            a += p;
            b = fmaf(p, (float)(1.0 - yj), b);
            e = fmaf((float)(kc.s * (xn2[i] + yn2[j] - 2.0 * dot)), py, e);
        }
        ps += (double)a;
        pq += (double)b;
        cs += (double)e;
    }
    double* o = part + (sb.p * kc.n + i) * 3;
    o[0] = ps;
    o[1] = pq;
    o[2] = cs;
}

__global__ void round_rows_merge(Consts kc, int P, const double* __restrict__ r, const double* __restrict__ xr,
                                 const double* __restrict__ part, double* __restrict__ dr, double* __restrict__ cpp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double ps = 0.0, pq = 0.0, cs = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        const double* o = part + ((int64_t)p * kc.n + i) * 3;
        ps += o[0];
        pq += o[1];
        cs += o[2];
    }
    const double w = xr[i] * r[i];
    dr[i] = r[i] * (1.0 - xr[i] * ps) + w * pq;
    cpp[i] = w * cs;
}

// Column sums of dc: S[k] = sum_j dc_j y~_jk (k < D), S[D] = sum_j dc_j,
// S[D+1] = sum_j dc_j ||y~_j||^2; block b computes S[b] in a fixed order.
__global__ void round_col_sums(Consts kc, int D, const double* __restrict__ yc, const double* __restrict__ yn2,
                               const double* __restrict__ dc, double* __restrict__ S) {
    __shared__ double sh[BLOCK];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < kc.m; j += BLOCK) {
        const double v = b < D ? yc[j * D + b] : (b == D ? 1.0 : yn2[j]);
        acc = fma(dc[j], v, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) S[b] = sh[0];
}

// t_i = dr_i (C dc)_i and |dr_i| by a pass over all pairs (the l1 / l_inf costs, whose
// C dc has no closed form): C_ij = -2 s P(x~_i, y~_j).
__global__ __launch_bounds__(BLOCK) void round_rank_one_pairs(Consts kc, int D, const double* __restrict__ xc,
                                                              const double* __restrict__ yc,
                                                              const double* __restrict__ dr,
                                                              const double* __restrict__ dc, double* __restrict__ t,
                                                              double* __restrict__ absdr) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= kc.n) return;
    double acc = 0.0;
    for (int64_t j = 0; j < kc.m; ++j)
        acc = fma(-2.0 * kc.s * pair_term_dyn(kc, D, xc + i * D, yc + j * D, 0.0), dc[j], acc);
    t[i] = dr[i] * acc;
    absdr[i] = fabs(dr[i]);
}

// t_i = dr_i (C dc)_i and |dr_i|.
__global__ void round_rank_one(Consts kc, int D, const double* __restrict__ xc, const double* __restrict__ xn2,
                               const double* __restrict__ dr, const double* __restrict__ S,
                               double* __restrict__ t, double* __restrict__ absdr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double xs = 0.0;
    for (int k = 0; k < D; ++k) xs = fma(xc[i * D + k], S[k], xs);
    t[i] = dr[i] * kc.s * (xn2[i] * S[D] + S[D + 1] - 2.0 * xs);
    absdr[i] = fabs(dr[i]);
}

// g^A_j for an arbitrary (lam, v): gA_j = -lam LOG2E (s yn2_j + K v_j).
__global__ void col_table_single(Consts kc, double lam, const double* __restrict__ yn2,
                                 const double* __restrict__ v, double* __restrict__ gA) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    gA[j] = -lam * LOG2E * (kc.s * yn2[j] + kc.K * v[j]);
}

// c_j * theta_j products for <c, theta>, <c, nu>.
__global__ void col_products(Consts kc, const double* __restrict__ c, const double* __restrict__ a,
                             const double* __restrict__ b, double* __restrict__ out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    out[j] = c[j] * a[j];
    out[kc.m + j] = c[j] * b[j];
}

// ---------------------------------------------------------------------------
// Adjoint sweep (envelope gradient), one pass over the pairs: per row i and column split p,
// with unnormalised weights q_ij = 2^(cfac P_ij + g_j - M_ip) (g_j = g^A_j of X^t), the
// partial sums Z_ip = sum_j q_ij and S1_ip (d values) and the split's offset M_ip, an
// integer that each lane raises to ceil(max e) whenever a block of columns exceeds it
// (the first block sets it), so every term is at most 1 and a raise rescales the sums
// exactly by a power of two.  grad_i = 2 s r_i (c_x Z_i x~_i - S1_i) / Z_i, the
// normaliser cancelling in the ratio:
//   squared Euclidean (dC/dx = 2 s (x - y)):  c_x = 1, S1 = sum_j q_ij y~_j;
//   l1 (dC/dx_k = s sign(x_k - y_k)):       c_x = 0, S1_k = -1/2 sum_j q_ij sign(x_k - y_jk);
//   l_inf (the coordinate k* of the largest |x_k - y_k|, the first one on ties):
//                                           c_x = 0, S1_k = -1/2 sum_j q_ij sign(x_k - y_jk) [k = k*].
// (sign(0) = 0: the subgradient at a kink.)  part: [P][n][D+2] = (M, Z, S1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sgnf(double v) { return v > 0.0 ? 1.f : (v < 0.0 ? -1.f : 0.f); }

// The one-pass row sweeps at X^t -- the adjoint above and the transport cost
// <C, X^t> = sum_i r_i sum_j p_ij C_ij -- share the exponent assembly and the offset
// handling; what each adds per column is a policy:
//   Col     the column record, read with a few wide scalar loads;
//   W       the number of sums (FP32 within a block of columns, FP64 across blocks);
//   block   called with the dot products' initial value hb of each block of columns;
//   add     accumulates one column with weight q, given ph = hb + P_ij.

// One column's data for the adjoint: y~_j in FP64 (dot product), g^A_j, y~_j in FP32 (S1).
template <int D>
struct alignas(16) AdjCol {
    double y[D];
    double g;
    float yf[D];
};

// The adjoint's sums: Z and S1 (d values, in the form of the metric).
template <int M, int D>
struct GradSums {
    using Col = AdjCol<D>;
    static constexpr int W = D + 1;
    __device__ __forceinline__ void block(double) {}
    __device__ __forceinline__ void add(const double (&x)[D], const Col& c, double, float q, float (&a)[W]) const {
        a[0] += q;
        if constexpr (M == METRIC_SQEUCLID) {
#pragma unroll
            for (int k = 0; k < D; ++k) a[1 + k] = fmaf(q, c.yf[k], a[1 + k]);
        } else if constexpr (M == METRIC_L1) {
#pragma unroll
            for (int k = 0; k < D; ++k) a[1 + k] = fmaf(-0.5f * q, sgnf(x[k] - c.y[k]), a[1 + k]);
        } else {
            int ks = 0;
            double best = -1.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double t = fabs(x[k] - c.y[k]);
                if (t > best) {
                    best = t;
                    ks = k;
                }
            }
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (k == ks) a[1 + k] = fmaf(-0.5f * q, sgnf(x[k] - c.y[k]), a[1 + k]);
        }
    }
};

// One column's data for the transport cost: y~_j (FP64), g^A_j, |y~_j|^2.
template <int D>
struct alignas(16) CostCol {
    double y[D];
    double g;
    double yn2;
};

// The transport cost's sums: Z and S_C = sum_j q_ij C_ij / s.  C_ij / s = |x~_i|^2 + |y~_j|^2
// - 2 P_ij is taken from the exponent's dot product ph = hb + P_ij as
// (|x~_i|^2 + 2 hb + |y~_j|^2) - 2 ph, two FP64 operations per pair (the norms are zero
// for l1 / l_inf, where P_ij = -dist / 2); each term is nonnegative, so the FP32 block sums
// lose no digits to cancellation.
template <int M, int D>
struct CostSums {
    using Col = CostCol<D>;
    static constexpr int W = 2;
    double xn2 = 0.0, a = 0.0;
    __device__ __forceinline__ void block(double hb) { a = xn2 + 2.0 * hb; }
    __device__ __forceinline__ void add(const double (&)[D], const Col& c, double ph, float q, float (&s)[W]) const {
        s[0] += q;
        const double cs = fma(-2.0, ph, M == METRIC_SQEUCLID ? a + c.yn2 : a);
        s[1] = fmaf(q, (float)cs, s[1]);
    }
};

// The row sums alone (Z): X^t's row normalisers in one pass, for the adjoint with respect to
// y, whose column pass weights each row by r_i / Z_i.
template <int D>
struct NormSums {
    using Col = CostCol<D>;
    static constexpr int W = 1;
    __device__ __forceinline__ void block(double) {}
    __device__ __forceinline__ void add(const double (&)[D], const Col&, double, float q, float (&s)[W]) const {
        s[0] += q;
    }
};

template <int D>
__global__ void adjoint_pack(int64_t m, const double* __restrict__ yc, const float* __restrict__ ycf,
                             const double* __restrict__ gA, AdjCol<D>* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    AdjCol<D> c;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c.y[k] = yc[j * D + k];
        c.yf[k] = ycf[j * D + k];
    }
    c.g = gA[j];
    out[j] = c;
}

template <int D>
__global__ void cost_pack(int64_t m, const double* __restrict__ yc, const double* __restrict__ yn2,
                          const double* __restrict__ gA, CostCol<D>* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    CostCol<D> c;
#pragma unroll
    for (int k = 0; k < D; ++k) c.y[k] = yc[j * D + k];
    c.g = gA[j];
    c.yn2 = yn2[j];
    out[j] = c;
}

// Per row i and column split p: the split's offset M_ip, an integer that each lane raises to
// ceil(max e) whenever a block of columns exceeds it (the first block sets it), so every
// term is at most 1 and a raise rescales the sums exactly by a power of two; then the W sums
// of the policy.  part: [P][n][W + 1] = (M, sums); an empty split writes M = -inf.
template <int M, int D, class Pol>
__device__ __forceinline__ void weighted_row_sums(const Consts& kc, double cA, const double* __restrict__ xc,
                                                  const typename Pol::Col* __restrict__ cols, Pol pol,
                                                  double* __restrict__ part, int64_t split) {
    constexpr int W = Pol::W;
    using Col = typename Pol::Col;
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    const int64_t p = sb.p;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const int64_t ii = i < kc.n ? i : kc.n - 1;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = xc[ii * D + k];
    double off = 0.0;      // M: integer offset of this lane's exponents
    double h = 0.0;        // -M / cfac, the dot products' initial value
    bool first = true;
    double s[W];
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] = 0.0;
    // raise the offset by ceil(bm) (bm: the largest exponent under the current offset),
    // rescaling the sums exactly; returns the raise
    auto raise = [&](double bm) {
        const double sh = ceil(bm);
#pragma unroll
        for (int w = 0; w < W; ++w) s[w] = ldexp(s[w], -(int)sh);
        off += sh;
        h = -off / cA;
        return sh;
    };
    // blocks of UNROLL columns with a compile-time trip count (the column data are
    // wave-uniform scalar loads, issued together); the offset is checked once per block
    const int64_t nfull = (j1 - j0) / UNROLL;
    const Col* __restrict__ cp = cols + j0;
    for (int64_t c = 0; c < nfull; ++c, cp += UNROLL) {
        const double hb = h;
        double ph[UNROLL], e[UNROLL];
        float ef[UNROLL];
        float bm = -__builtin_inff();
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            ph[u] = pair_term<M, D>(x, cp[u].y, hb);
            e[u] = fma_su(ph[u], cA, cp[u].g);
            ef[u] = (float)e[u];
            bm = fmaxf(bm, ef[u]);
        }
        if (first || bm > 0.f) {   // rare after the first block
            double bmd = e[0];
#pragma unroll
            for (int u = 1; u < UNROLL; ++u) bmd = fmax(bmd, e[u]);
            const double sh = raise(bmd);
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) ef[u] = (float)(e[u] - sh);
            first = false;
        }
        pol.block(hb);
        float a[W];
#pragma unroll
        for (int w = 0; w < W; ++w) a[w] = 0.f;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) pol.add(x, cp[u], ph[u], __builtin_amdgcn_exp2f(ef[u]), a);
#pragma unroll
        for (int w = 0; w < W; ++w) s[w] += (double)a[w];
    }
    // the remaining columns one at a time
    for (int64_t j = j0 + nfull * UNROLL; j < j1; ++j) {
        const double hb = h;
        const double ph = pair_term<M, D>(x, cols[j].y, hb);
        double e = fma_su(ph, cA, cols[j].g);
        if (first || e > 0.0) {
            e -= raise(e);
            first = false;
        }
        pol.block(hb);
        float a[W];
#pragma unroll
        for (int w = 0; w < W; ++w) a[w] = 0.f;
        pol.add(x, cols[j], ph, fexp2(e), a);
#pragma unroll
        for (int w = 0; w < W; ++w) s[w] += (double)a[w];
    }
    if (i < kc.n) {
        double* o = part + (p * kc.n + i) * (W + 1);
        o[0] = first ? -__builtin_inf() : off;   // an empty split contributes nothing
#pragma unroll
        for (int w = 0; w < W; ++w) o[1 + w] = s[w];
    }
}

// part: [P][n][D + 2] = (M, Z, S1).
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void adjoint_sweep(Consts kc, double cA, const double* __restrict__ xc,
                                                       const AdjCol<D>* __restrict__ cols,
                                                       double* __restrict__ part, int64_t split) {
    weighted_row_sums<M, D>(kc, cA, xc, cols, GradSums<M, D>{}, part, split);
}

// part: [P][n][3] = (M, Z, S_C).
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void cost_sweep(Consts kc, double cA, const double* __restrict__ xc,
                                                    const double* __restrict__ xn2,
                                                    const CostCol<D>* __restrict__ cols,
                                                    double* __restrict__ part, int64_t split) {
    const int64_t i = sweep_block(kc.m, split).bx * BLOCK + threadIdx.x;
    CostSums<M, D> pol;
    if constexpr (M == METRIC_SQEUCLID) pol.xn2 = xn2[i < kc.n ? i : kc.n - 1];
    weighted_row_sums<M, D>(kc, cA, xc, cols, pol, part, split);
}

// part: [P][n][2] = (M, Z).
template <int M, int D>
__global__ __launch_bounds__(BLOCK) void norm_sweep(Consts kc, double cA, const double* __restrict__ xc,
                                                    const CostCol<D>* __restrict__ cols,
                                                    double* __restrict__ part, int64_t split) {
    weighted_row_sums<M, D>(kc, cA, xc, cols, NormSums<D>{}, part, split);
}

// X^t's row data for the column-side adjoint from the splits' (M, Z) at their common offset:
// sigma_i = M + log2 Z (base 2), k_i = -sigma_i / cfac, so that
// X_ij = r_i 2^(cfac (k_i + P_ij) + g_j); wA = wB = r_i.
__global__ void norm_finish(Consts kc, int P, double cA, const double* __restrict__ r,
                            const double* __restrict__ part, RowVar* __restrict__ rowvar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double off = -__builtin_inf();
#pragma unroll 8
    for (int p = 0; p < P; ++p) off = fmax(off, part[((int64_t)p * kc.n + i) * 2]);
    double z = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        const double* o = part + ((int64_t)p * kc.n + i) * 2;
        if (o[0] > -__builtin_inf()) z += ldexp(o[1], (int)(o[0] - off));
    }
    RowVar rv;
    rv.k = -(off + log2(z)) / cA;
    rv.wA = rv.wB = (float)r[i];
    rowvar[i] = rv;
}

// The transport cost for any dimension and metric at run time, FP64 sums.  part as above.
__global__ __launch_bounds__(BLOCK) void cost_sweep_dyn(Consts kc, int D, double cA,
                                                        const double* __restrict__ xc,
                                                        const double* __restrict__ yc,
                                                        const double* __restrict__ xn2,
                                                        const double* __restrict__ yn2,
                                                        const double* __restrict__ gA,
                                                        double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    const int64_t p = sb.p;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    if (i >= kc.n) return;
    const double* xi = xc + i * D;
    double off = -__builtin_inf(), s0 = 0.0, sc = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double pij = pair_term_dyn(kc, D, xi, yc + j * D, 0.0);
        const double e = fma(cA, pij, gA[j]);
        if (e > off) {   // raise the offset to ceil(e), rescaling the sums exactly
            const double nm = ceil(e);
            const int sh = j == j0 ? 0 : (int)(off - nm);
            s0 = ldexp(s0, sh);
            sc = ldexp(sc, sh);
            off = nm;
        }
        const double q = (double)fexp2(e - off);
        s0 += q;
        sc += q * fma(-2.0, pij, xn2[i] + yn2[j]);
    }
    double* o = part + (p * kc.n + i) * 3;
    o[0] = off;
    o[1] = s0;
    o[2] = sc;
}

// Row i's share of the transport cost, s r_i S_C / Z, from the splits' (M, Z, S_C) brought to
// their common offset (exact powers of two).
__global__ void cost_finish(Consts kc, int P, const double* __restrict__ r, const double* __restrict__ part,
                            double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    double off = -__builtin_inf();
#pragma unroll 8
    for (int p = 0; p < P; ++p) off = fmax(off, part[((int64_t)p * kc.n + i) * 3]);
    double z = 0.0, c = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        const double* o = part + ((int64_t)p * kc.n + i) * 3;
        if (o[0] > -__builtin_inf()) {
            z += ldexp(o[1], (int)(o[0] - off));
            c += ldexp(o[2], (int)(o[0] - off));
        }
    }
    out[i] = kc.s * r[i] * (c / z);
}

__global__ __launch_bounds__(BLOCK) void adjoint_sweep_dyn(Consts kc, int D, double cA,
                                                           const double* __restrict__ xc,
                                                           const double* __restrict__ yc,
                                                           const float* __restrict__ ycf,
                                                           const double* __restrict__ gA,
                                                           double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.m, split);
    const int64_t i = sb.bx * BLOCK + threadIdx.x;
    const int64_t p = sb.p;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    if (i >= kc.n) return;
    const double* xi = xc + i * D;
    double* o = part + (p * kc.n + i) * (D + 2);
    for (int k = 0; k < D; ++k) o[2 + k] = 0.0;
    double off = -__builtin_inf(), s0 = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double* yj = yc + j * D;
        double e = fma(cA, pair_term_dyn(kc, D, xi, yj, 0.0), gA[j]);
        if (e > off) {   // raise the offset to ceil(e), rescaling the sums exactly
            const double nm = ceil(e);
            const int sh = j == j0 ? 0 : (int)(off - nm);
            s0 = ldexp(s0, sh);
            for (int k = 0; k < D; ++k) o[2 + k] = ldexp(o[2 + k], sh);
            off = nm;
        }
        const double q = (double)fexp2(e - off);
        s0 += q;
        if (kc.metric == METRIC_SQEUCLID) {
            for (int k = 0; k < D; ++k) o[2 + k] += q * (double)ycf[j * D + k];
        } else if (kc.metric == METRIC_L1) {
            for (int k = 0; k < D; ++k) o[2 + k] += -0.5 * q * (double)sgnf(xi[k] - yj[k]);
        } else {
            int ks = 0;
            double best = -1.0;
            for (int k = 0; k < D; ++k) {
                const double t = fabs(xi[k] - yj[k]);
                if (t > best) {
                    best = t;
                    ks = k;
                }
            }
            o[2 + ks] += -0.5 * q * (double)sgnf(xi[ks] - yj[ks]);
        }
    }
    o[0] = off;
    o[1] = s0;
}

// ---------------------------------------------------------------------------
// Adjoint with respect to the target points: per column j, with
// X_ij = w_i 2^(cfac (k_i + P_ij) + g_j) (the column sweep's terms of X^t, w_i = r_i),
// partial sums S0_j, S1_j (d values) such that grad_y_j = 2 s (S0_j y~_j - S1_j):
//   squared Euclidean (dC/dy = 2 s (y - x)):  S0 = sum_i X_ij,  S1 = sum_i X_ij x~_i;
//   l1 (dC/dy_k = -s sign(x_k - y_k)):      S0 = 0,  S1_k = 1/2 sum_i X_ij sign(x_ik - y_k);
//   l_inf: the same on the coordinate of the largest |x_k - y_k| (first on ties).
// part: [P][m][D+1] partial sums over row splits.
// ---------------------------------------------------------------------------
// One row's data for the column-side adjoint: x~_i in FP64 (dot product), the row's exponent
// term cfac k_i, x~_i in FP32 (S1) and the weight w_i, read with a few wide scalar loads.
template <int D>
struct alignas(16) AdjRow {
    double x[D];
    double ck;
    float xf[D];
    float w;
};

template <int D>
__global__ void adjoint_y_pack(int64_t n, double cA, const double* __restrict__ xc, const float* __restrict__ xcf,
                               const RowVar* __restrict__ rowvar, AdjRow<D>* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    AdjRow<D> a;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        a.x[k] = xc[i * D + k];
        a.xf[k] = xcf[i * D + k];
    }
    const RowVar rv = rowvar[i];
    a.ck = cA * rv.k;
    a.w = rv.wA;
    out[i] = a;
}

template <int M, int D>
__global__ __launch_bounds__(BLOCK) void adjoint_y_sweep(Consts kc, double cA, const AdjRow<D>* __restrict__ rows,
                                                         const double* __restrict__ yc,
                                                         const double* __restrict__ gA,
                                                         double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.n, split);
    const int64_t j = sb.bx * BLOCK + threadIdx.x;
    const int64_t p = sb.p;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    const int64_t jj = j < kc.m ? j : kc.m - 1;
    double y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = yc[jj * D + k];
    // e_ij = cfac (G_j + P_ij) + cfac k_i with G_j = g_j / cfac: the dot product starts from
    // the lane's term and the row's term enters as the scalar addend of the exponent FMA
    const double G = gA[jj] / cA;
    double s0 = 0.0, s1[D];
#pragma unroll
    for (int k = 0; k < D; ++k) s1[k] = 0.0;
    auto term = [&](int64_t i, float& a0, float (&a1)[D]) {
        const AdjRow<D>& rw = rows[i];
        const double* xi = rw.x;
        const double dot = pair_term<M, D>(y, xi, G);   // P is symmetric
        const float xij = rw.w * fexp2(fma_su(dot, cA, rw.ck));
        if constexpr (M == METRIC_SQEUCLID) {
            a0 += xij;
#pragma unroll
            for (int k = 0; k < D; ++k) a1[k] = fmaf(xij, rw.xf[k], a1[k]);
        } else if constexpr (M == METRIC_L1) {
#pragma unroll
            for (int k = 0; k < D; ++k) a1[k] = fmaf(0.5f * xij, sgnf(xi[k] - y[k]), a1[k]);
        } else {
            int ks = 0;
            double best = -1.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double t = fabs(xi[k] - y[k]);
                if (t > best) {
                    best = t;
                    ks = k;
                }
            }
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (k == ks) a1[k] = fmaf(0.5f * xij, sgnf(xi[k] - y[k]), a1[k]);
        }
    };
    const int64_t nfull = (i1 - i0) / UNROLL;
    for (int64_t c = 0; c <= nfull; ++c) {
        const int64_t ib = i0 + c * UNROLL;
        float a0 = 0.f, a1[D];
#pragma unroll
        for (int k = 0; k < D; ++k) a1[k] = 0.f;
        if (c < nfull) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) term(ib + u, a0, a1);
        } else {
            for (int64_t i = ib; i < i1; ++i) term(i, a0, a1);
        }
        s0 += (double)a0;
#pragma unroll
        for (int k = 0; k < D; ++k) s1[k] += (double)a1[k];
    }
    if (j < kc.m) {
        double* o = part + (p * kc.m + j) * (D + 1);
        o[0] = s0;
#pragma unroll
        for (int k = 0; k < D; ++k) o[1 + k] = s1[k];
    }
}

__global__ __launch_bounds__(BLOCK) void adjoint_y_sweep_dyn(Consts kc, int D, double cA,
                                                             const double* __restrict__ xc,
                                                             const float* __restrict__ xcf,
                                                             const double* __restrict__ yc,
                                                             const double* __restrict__ gA,
                                                             const RowVar* __restrict__ rowvar,
                                                             double* __restrict__ part, int64_t split) {
    const SweepBlock sb = sweep_block(kc.n, split);
    const int64_t j = sb.bx * BLOCK + threadIdx.x;
    const int64_t p = sb.p;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    const int64_t jj = j < kc.m ? j : kc.m - 1;
    const double* yj = yc + jj * D;
    const double g = gA[jj];
    double* o = part + (p * kc.m + jj) * (D + 1);
    double s0 = 0.0;
    if (j < kc.m)
        for (int k = 0; k < D; ++k) o[1 + k] = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const RowVar rv = rowvar[i];
        const double* xi = xc + i * D;
        const double xij = (double)rv.wA * (double)fexp2(fma(cA, pair_term_dyn(kc, D, yj, xi, rv.k), g));
        if (kc.metric == METRIC_SQEUCLID) {
            s0 += xij;
            if (j < kc.m)
                for (int k = 0; k < D; ++k) o[1 + k] += xij * (double)xcf[i * D + k];
        } else if (kc.metric == METRIC_L1) {
            if (j < kc.m)
                for (int k = 0; k < D; ++k) o[1 + k] += 0.5 * xij * (double)sgnf(xi[k] - yj[k]);
        } else {
            int ks = 0;
            double best = -1.0;
            for (int k = 0; k < D; ++k) {
                const double t = fabs(xi[k] - yj[k]);
                if (t > best) {
                    best = t;
                    ks = k;
                }
            }
            if (j < kc.m) o[1 + ks] += 0.5 * xij * (double)sgnf(xi[ks] - yj[ks]);
        }
    }
    if (j < kc.m) o[0] = s0;
}

__global__ void adjoint_y_finish(Consts kc, int D, int P, double scale, const double* __restrict__ yc,
                                 const double* __restrict__ part, float* __restrict__ grad) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    double s0 = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) s0 += part[((int64_t)p * kc.m + j) * (D + 1)];
    for (int k = 0; k < D; ++k) {
        double s1 = 0.0;
#pragma unroll 8
        for (int p = 0; p < P; ++p) s1 += part[((int64_t)p * kc.m + j) * (D + 1) + 1 + k];
        grad[j * D + k] = (float)(scale * (s0 * yc[j * D + k] - s1));
    }
}

__global__ void adjoint_finish(Consts kc, int D, int P, double scale, const double* __restrict__ xc,
                               const double* __restrict__ r, const double* __restrict__ part,
                               float* __restrict__ grad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int W = D + 2;
    double off = -__builtin_inf();
#pragma unroll 8
    for (int p = 0; p < P; ++p) off = fmax(off, part[((int64_t)p * kc.n + i) * W]);
    // split p's sums are scaled by 2^-M_p: bring them to the common offset (exact)
    double s0 = 0.0;
#pragma unroll 8
    for (int p = 0; p < P; ++p) {
        const double* o = part + ((int64_t)p * kc.n + i) * W;
        if (o[0] > -__builtin_inf()) s0 += ldexp(o[1], (int)(o[0] - off));
    }
    const double cx = kc.metric == METRIC_SQEUCLID ? 1.0 : 0.0;
    for (int k = 0; k < D; ++k) {
        double s1 = 0.0;
#pragma unroll 8
        for (int p = 0; p < P; ++p) {
            const double* o = part + ((int64_t)p * kc.n + i) * W;
            if (o[0] > -__builtin_inf()) s1 += ldexp(o[2 + k], (int)(o[0] - off));
        }
        grad[i * D + k] = (float)(scale * r[i] * (cx * xc[i * D + k] - s1 / s0));
    }
}

}  // namespace lampk
