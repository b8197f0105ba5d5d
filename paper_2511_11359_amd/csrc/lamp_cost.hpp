// Row and column sweeps of Algorithm 2 over a cost matrix the caller stores
// (METRIC_EXPLICIT: C_ij = s cost_ij, cost row-major n x m FP32 in device memory).
//
// The exponents are those of the generic sweeps with the pair term P_ij = -cost_ij / 2
// and zero norms, evaluated in the same order and precision (FP64 argument, FP32
// exponential and partial sums over 8 terms, FP64 across them), so the row data
// (offsets h_i, RowVar) and the column table g^A, g^B are shared with every other
// pass.  What differs is the data layout: the pair data are 4 bytes of cost per pair
// read from HBM once per sweep, so both sweeps are bandwidth kernels, and both read C
// along its rows with a wave's 64 lanes on 64 consecutive columns: every load is one
// contiguous 256-byte segment, loaded non-temporally (C is streamed once per sweep and
// would only evict the column table and row data from the caches; measured 4-8% faster
// at n = m = 2^16).  The column sweep gives each lane its own columns and walks the
// rows, the natural order of a row-major matrix.  The row sweep gives each wave 8 rows
// and spreads their columns over the lanes, reducing over the lanes once at the end,
// so no transposed copy of C is stored (the paper's column-major implementation keeps
// one so that its row reductions read contiguously, Appendix E, fused reductions).
#pragma once
#include "lamp_kernels.hpp"

#include <type_traits>

namespace lampk {

constexpr int COST_ROWS = 8;   // rows per wave of the row sweep
constexpr int COST_U = 4;      // 64-column groups per lane and step of the row sweep
constexpr int COST_Q = 4;      // 64-column groups per lane of the column sweep

// Column extent of one step of the row sweep: the column splits are multiples of it.
constexpr int64_t COST_ROW_STEP = 64 * COST_U;
// Columns of one block of the column sweep.
constexpr int64_t COST_COL_BLOCK = 4 * 64 * COST_Q;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Row sweep: part[p][i] = (sum_j 2^(cA (h_i + P_ij) + g^A_j), same with cB, g^B) over
// the columns of split p = blockIdx.y, [p split, (p + 1) split) with split a multiple
// of COST_ROW_STEP; block b owns rows [32 b, 32 b + 32), wave w of it 8 of them.
template <typename T>
__global__ __launch_bounds__(BLOCK) void row_sweep_cost(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                        const double2* __restrict__ gtab2,
                                                        const double* __restrict__ H,
                                                        double2* __restrict__ part, int64_t split) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * COST_ROWS;
    const int64_t p = blockIdx.y;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const T* __restrict__ row[COST_ROWS];
    double h[COST_ROWS];
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) {
        const int64_t ii = min(i0 + r, kc.n - 1);   // rows past n repeat the last one, unwritten
        row[r] = static_cast<const T*>(kc.cost) + ii * kc.m;
        h[r] = H[ii];
    }
    double sA[COST_ROWS], sB[COST_ROWS];
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) sA[r] = sB[r] = 0.0;
    // one step of COST_ROW_STEP columns; only the last step of a split can pass its end (its
    // columns past the end read the split's last column and contribute 2^-inf = 0)
    auto step = [&](int64_t jb, auto masked_tag) {
        constexpr bool MASKED = decltype(masked_tag)::value;
        int64_t jj[COST_U];
        double2 gj[COST_U];
        float cv[COST_ROWS][COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            const int64_t j = jb + u * 64 + lane;
            jj[u] = MASKED ? min(j, j1 - 1) : j;
            gj[u] = g[jj[u]];
            if (MASKED && j >= j1) gj[u] = make_double2(-__builtin_inf(), -__builtin_inf());
        }
#pragma unroll
        for (int r = 0; r < COST_ROWS; ++r)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) cv[r][u] = load_cost_col(row[r], jj[u]);
        // every load of the step is issued before the first use: left to itself the
        // scheduler interleaves each load with its use and waits for it, one load in flight
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < COST_ROWS; ++r) {
            float aA = 0.f, aB = 0.f;
#pragma unroll
            for (int u = 0; u < COST_U; ++u) {
                const double dot = fma(-0.5, (double)cv[r][u], h[r]);
                aA += fexp2(fma(cA, dot, gj[u].x));
                aB += fexp2(fma(cB, dot, gj[u].y));
            }
            sA[r] += (double)aA;
            sB[r] += (double)aB;
        }
    };
    int64_t jb = j0;
    for (; jb + COST_ROW_STEP <= j1; jb += COST_ROW_STEP) step(jb, std::false_type{});
    if (jb < j1) step(jb, std::true_type{});
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) {
        const double a = wave_sum(sA[r]);
        const double b = wave_sum(sB[r]);
        if (lane == r && i0 + r < kc.n) part[p * kc.n + i0 + r] = make_double2(a, b);
    }
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Row extreme pass, the layout of the row sweep: part[p][i] = min_j (a_j + sgn P_ij) over the
// columns of split p, P_ij = -cost_ij / 2 (exact offsets, the cost maximum, D(theta)).  The
// terms are those of the generic pass and a minimum is exact, so the result is the same.
template <typename T>
__global__ __launch_bounds__(BLOCK) void row_extreme_cost(Consts kc, const double* __restrict__ a, double sgn,
                                                          double* __restrict__ part, int64_t split) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * COST_ROWS;
    const int64_t p = blockIdx.y;
    const int64_t j0 = p * split;
    const int64_t j1 = min(kc.m, j0 + split);
    const T* __restrict__ row[COST_ROWS];
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) row[r] = static_cast<const T*>(kc.cost) + min(i0 + r, kc.n - 1) * kc.m;
    double best[COST_ROWS];
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) best[r] = __builtin_inf();
    for (int64_t jb = j0; jb < j1; jb += COST_ROW_STEP) {
        int64_t jj[COST_U];
        double aj[COST_U];
        float cv[COST_ROWS][COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            const int64_t j = jb + u * 64 + lane;
            jj[u] = min(j, j1 - 1);
            aj[u] = j < j1 ? a[jj[u]] : __builtin_inf();
        }
#pragma unroll
        for (int r = 0; r < COST_ROWS; ++r)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) cv[r][u] = load_cost_col(row[r], jj[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < COST_ROWS; ++r)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) best[r] = fmin(best[r], fma(sgn, -0.5 * (double)cv[r][u], aj[u]));
    }
#pragma unroll
    for (int r = 0; r < COST_ROWS; ++r) {
        const double v = wave_min(best[r]);
        if (lane == r && i0 + r < kc.n) part[p * kc.n + i0 + r] = v;
    }
}

// <C, Xbar^{t+1}> per row for the D_t tracking, the layout of the row sweep over whole rows:
// out_i = r_i T_i / S_i with S_i = sum_j 2^(cB (h_i + P_ij) + g^B_j), T_i the same sum
// weighted by C_ij = s cost_ij; the terms of the generic pass.
template <typename T>
__global__ __launch_bounds__(BLOCK) void dt_cost_rows_cost(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                           const double2* __restrict__ gtab2,
                                                           const double* __restrict__ H,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ out) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * COST_ROWS;
    const T* __restrict__ row[COST_ROWS];
    double h[COST_ROWS];
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        const int64_t ii = min(i0 + r_, kc.n - 1);
        row[r_] = static_cast<const T*>(kc.cost) + ii * kc.m;
        h[r_] = H[ii];
    }
    double S[COST_ROWS], Tw[COST_ROWS];
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) S[r_] = Tw[r_] = 0.0;
    for (int64_t jb = 0; jb < kc.m; jb += COST_ROW_STEP) {
        int64_t jj[COST_U];
        double gB[COST_U];
        float cv[COST_ROWS][COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            const int64_t j = jb + u * 64 + lane;
            jj[u] = min(j, kc.m - 1);
            gB[u] = j < kc.m ? g[jj[u]].y : -__builtin_inf();
        }
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) cv[r_][u] = load_cost_col(row[r_], jj[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_) {
            float aS = 0.f, aT = 0.f;
#pragma unroll
            for (int u = 0; u < COST_U; ++u) {
                const double dot = -0.5 * (double)cv[r_][u];
                const float pij = fexp2(fma(cB, h[r_] + dot, gB[u]));
                aS += pij;
                aT = fmaf(pij, (float)fma(-2.0 * kc.s, dot, 0.0), aT);
            }
            S[r_] += (double)aS;
            Tw[r_] += (double)aT;
        }
    }
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        const double sS = wave_sum(S[r_]);
        const double sT = wave_sum(Tw[r_]);
        if (lane == r_ && i0 + r_ < kc.n) out[i0 + r_] = r[i0 + r_] * sT / sS;
    }
}

// ---------------------------------------------------------------------------
// Certificate and Round passes over whole rows, in the layout of the row sweep (8 rows per
// wave, 64 consecutive columns per load, one lane reduction per row at the end), with the
// terms of the generic passes: C_ij = s cost_ij, p_ij = 2^(cA (h_i + P_ij) + g^A_j).
// ---------------------------------------------------------------------------
template <typename T>
struct CostRows {
    int64_t i0;
    int lane;
    const T* row[COST_ROWS];
    __device__ __forceinline__ CostRows(const Consts& kc) {
        lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        i0 = ((int64_t)blockIdx.x * 4 + wave) * COST_ROWS;
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_) row[r_] = static_cast<const T*>(kc.cost) + min(i0 + r_, kc.n - 1) * kc.m;
    }
    // the step's columns (clamped to m - 1; valid[u] false past m) and their cost entries
    __device__ __forceinline__ void load(const Consts& kc, int64_t jb, int64_t (&jj)[COST_U], bool (&valid)[COST_U],
                                         float (&cv)[COST_ROWS][COST_U]) const {
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            const int64_t j = jb + u * 64 + lane;
            valid[u] = j < kc.m;
            jj[u] = min(j, kc.m - 1);
        }
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) cv[r_][u] = load_cost_col(row[r_], jj[u]);
    }
};

// vals[0..3][i] and psum_out[i] as cert_rows.
template <typename T>
__global__ __launch_bounds__(BLOCK) void cert_rows_cost(Consts kc, double cA, const double* __restrict__ gA,
                                                        const double* __restrict__ H, const double* __restrict__ r,
                                                        const double* __restrict__ nu,
                                                        const double* __restrict__ theta,
                                                        double* __restrict__ vals, double* __restrict__ psum_out) {
    const CostRows<T> cr(kc);
    double h[COST_ROWS], psum[COST_ROWS], csum[COST_ROWS], mth[COST_ROWS], mnu[COST_ROWS];
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        h[r_] = H[min(cr.i0 + r_, kc.n - 1)];
        psum[r_] = csum[r_] = 0.0;
        mth[r_] = mnu[r_] = __builtin_inf();
    }
    for (int64_t jb = 0; jb < kc.m; jb += COST_ROW_STEP) {
        int64_t jj[COST_U];
        bool valid[COST_U];
        float cv[COST_ROWS][COST_U];
        cr.load(kc, jb, jj, valid, cv);
        double ga[COST_U], th[COST_U], nv[COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            ga[u] = valid[u] ? gA[jj[u]] : -__builtin_inf();
            th[u] = valid[u] ? theta[jj[u]] : __builtin_inf();
            nv[u] = valid[u] ? nu[jj[u]] : __builtin_inf();
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_) {
            float ap = 0.f, ac = 0.f;
#pragma unroll
            for (int u = 0; u < COST_U; ++u) {
                const double dot = -0.5 * (double)cv[r_][u];
                const float p = fexp2(fma(cA, h[r_] + dot, ga[u]));
                const double cij = kc.s * (double)cv[r_][u];
                ap += p;
                ac = fmaf((float)cij, p, ac);
                mth[r_] = fmin(mth[r_], cij + kc.K * th[u]);
                mnu[r_] = fmin(mnu[r_], cij + kc.K * nv[u]);
            }
            psum[r_] += (double)ap;
            csum[r_] += (double)ac;
        }
    }
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        const double ps = wave_sum(psum[r_]), cs = wave_sum(csum[r_]);
        const double a = wave_min(mth[r_]), b = wave_min(mnu[r_]);
        const int64_t i = cr.i0 + r_;
        if (cr.lane == r_ && i < kc.n) {
            const double ri = r[i];
            vals[i] = ri * fabs(ps - 1.0);
            vals[kc.n + i] = ri * cs;
            vals[2 * kc.n + i] = ri * a;
            vals[3 * kc.n + i] = ri * b;
            if (psum_out) psum_out[i] = ps;
        }
    }
}

// dr[i], cpp[i] as round_rows.
template <typename T>
__global__ __launch_bounds__(BLOCK) void round_rows_cost(Consts kc, double cA, const double* __restrict__ gA,
                                                         const double* __restrict__ H, const double* __restrict__ r,
                                                         const double* __restrict__ xr, const double* __restrict__ y,
                                                         double* __restrict__ dr, double* __restrict__ cpp) {
    const CostRows<T> cr(kc);
    double h[COST_ROWS], ps[COST_ROWS], pq[COST_ROWS], cs[COST_ROWS];
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        h[r_] = H[min(cr.i0 + r_, kc.n - 1)];
        ps[r_] = pq[r_] = cs[r_] = 0.0;
    }
    for (int64_t jb = 0; jb < kc.m; jb += COST_ROW_STEP) {
        int64_t jj[COST_U];
        bool valid[COST_U];
        float cv[COST_ROWS][COST_U];
        cr.load(kc, jb, jj, valid, cv);
        double ga[COST_U], yj[COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) {
            ga[u] = valid[u] ? gA[jj[u]] : -__builtin_inf();
            yj[u] = y[jj[u]];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_) {
            float a = 0.f, b = 0.f, e = 0.f;
#pragma unroll
            for (int u = 0; u < COST_U; ++u) {
                const double dot = -0.5 * (double)cv[r_][u];
                const float p = fexp2(fma(cA, h[r_] + dot, ga[u]));
                const float py = p * (float)yj[u];
                a += p;
                b = fmaf(p, (float)(1.0 - yj[u]), b);
                e = fmaf((float)(kc.s * (double)cv[r_][u]), py, e);
            }
            ps[r_] += (double)a;
            pq[r_] += (double)b;
            cs[r_] += (double)e;
        }
    }
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        const double sps = wave_sum(ps[r_]), spq = wave_sum(pq[r_]), scs = wave_sum(cs[r_]);
        const int64_t i = cr.i0 + r_;
        if (cr.lane == r_ && i < kc.n) {
            const double w = xr[i] * r[i];
            dr[i] = r[i] * (1.0 - xr[i] * sps) + w * spq;
            cpp[i] = w * scs;
        }
    }
}

// t_i = dr_i (C dc)_i and |dr_i| as round_rank_one_pairs.
template <typename T>
__global__ __launch_bounds__(BLOCK) void round_rank_one_cost(Consts kc, const double* __restrict__ dr,
                                                             const double* __restrict__ dc, double* __restrict__ t,
                                                             double* __restrict__ absdr) {
    const CostRows<T> cr(kc);
    double acc[COST_ROWS];
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) acc[r_] = 0.0;
    for (int64_t jb = 0; jb < kc.m; jb += COST_ROW_STEP) {
        int64_t jj[COST_U];
        bool valid[COST_U];
        float cv[COST_ROWS][COST_U];
        cr.load(kc, jb, jj, valid, cv);
        double dcj[COST_U];
#pragma unroll
        for (int u = 0; u < COST_U; ++u) dcj[u] = valid[u] ? dc[jj[u]] : 0.0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r_ = 0; r_ < COST_ROWS; ++r_)
#pragma unroll
            for (int u = 0; u < COST_U; ++u) acc[r_] = fma(kc.s * (double)cv[r_][u], dcj[u], acc[r_]);
    }
#pragma unroll
    for (int r_ = 0; r_ < COST_ROWS; ++r_) {
        const double a = wave_sum(acc[r_]);
        const int64_t i = cr.i0 + r_;
        if (cr.lane == r_ && i < kc.n) {
            t[i] = dr[i] * a;
            absdr[i] = fabs(dr[i]);
        }
    }
}

// Round step 2 over the row splits of the column sweep: part[p][j] = sum over the rows i of
// split p of xr_i r_i p_ij (the terms of round_cols, merged by round_cols_merge).
template <typename T>
__global__ __launch_bounds__(BLOCK) void round_cols_cost(Consts kc, double cA, const double* __restrict__ gA,
                                                         const double* __restrict__ H, const double* __restrict__ r,
                                                         const double* __restrict__ xr, double* __restrict__ part,
                                                         int64_t split) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t jw = ((int64_t)blockIdx.x * 4 + wave) * 64 * COST_Q;
    const int64_t p = blockIdx.y;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    int64_t jj[COST_Q];
    double g[COST_Q], acc[COST_Q];
#pragma unroll
    for (int q = 0; q < COST_Q; ++q) {
        jj[q] = min(jw + q * 64 + lane, kc.m - 1);
        g[q] = gA[jj[q]];
        acc[q] = 0.0;
    }
    auto rows = [&](int64_t i, float (&a)[COST_Q]) {
        const float w = (float)(xr[i] * r[i]);
        const double h = H[i];
        const T* __restrict__ crow = static_cast<const T*>(kc.cost) + i * kc.m;
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) {
            const double dot = -0.5 * (double)load_cost_col(crow, jj[q]);
            a[q] = fmaf(w, fexp2(fma(cA, h + dot, g[q])), a[q]);
        }
    };
    int64_t ib = i0;
    for (; ib + UNROLL <= i1; ib += UNROLL) {
        float a[COST_Q];
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) a[q] = 0.f;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) rows(ib + u, a);
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) acc[q] += (double)a[q];
    }
    if (ib < i1) {
        float a[COST_Q];
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) a[q] = 0.f;
        for (; ib < i1; ++ib) rows(ib, a);
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) acc[q] += (double)a[q];
    }
#pragma unroll
    for (int q = 0; q < COST_Q; ++q) {
        const int64_t j = jw + q * 64 + lane;
        if (j < kc.m) part[p * kc.m + j] = acc[q];
    }
}

// Column sweep: cpart[p][j] = (sum_i wA_i 2^(cA (k_i + P_ij) + g^A_j), sum_i wB_i 2^(cB ...))
// over the rows of split p = blockIdx.y; wave w of block b owns the 64 COST_Q columns
// from (4 b + w) 64 COST_Q, lane l the columns l + 64 q.
template <typename T>
__global__ __launch_bounds__(BLOCK) void col_sweep_cost(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                        const double2* __restrict__ gtab2,
                                                        const RowVar* __restrict__ rowvar,
                                                        double2* __restrict__ cpart, int64_t split) {
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t jw = ((int64_t)blockIdx.x * 4 + wave) * 64 * COST_Q;
    const int64_t p = blockIdx.y;
    const int64_t i0 = p * split;
    const int64_t i1 = min(kc.n, i0 + split);
    // columns past m read column m - 1 and are not written
    int64_t jj[COST_Q];
    double2 gj[COST_Q];
#pragma unroll
    for (int q = 0; q < COST_Q; ++q) {
        jj[q] = min(jw + q * 64 + lane, kc.m - 1);
        gj[q] = gtab2[(t & 1) * kc.m + jj[q]];
    }
    double sA[COST_Q], sB[COST_Q];
#pragma unroll
    for (int q = 0; q < COST_Q; ++q) sA[q] = sB[q] = 0.0;
    auto rows = [&](int64_t i, float (&aA)[COST_Q], float (&aB)[COST_Q]) {
        const RowVar rv = rowvar[i];
        const T* __restrict__ crow = static_cast<const T*>(kc.cost) + i * kc.m;
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) {
            const double dot = fma(-0.5, (double)load_cost_col(crow, jj[q]), rv.k);
            aA[q] = fmaf(rv.wA, fexp2(fma(cA, dot, gj[q].x)), aA[q]);
            aB[q] = fmaf(rv.wB, fexp2(fma(cB, dot, gj[q].y)), aB[q]);
        }
    };
    const int64_t nfull = (i1 - i0) / UNROLL;
    int64_t ib = i0;
    for (int64_t c = 0; c < nfull; ++c, ib += UNROLL) {
        float aA[COST_Q], aB[COST_Q];
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) aA[q] = aB[q] = 0.f;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) rows(ib + u, aA, aB);
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) {
            sA[q] += (double)aA[q];
            sB[q] += (double)aB[q];
        }
    }
    if (ib < i1) {
        float aA[COST_Q], aB[COST_Q];
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) aA[q] = aB[q] = 0.f;
        for (; ib < i1; ++ib) rows(ib, aA, aB);
#pragma unroll
        for (int q = 0; q < COST_Q; ++q) {
            sA[q] += (double)aA[q];
            sB[q] += (double)aB[q];
        }
    }
#pragma unroll
    for (int q = 0; q < COST_Q; ++q) {
        const int64_t j = jw + q * 64 + lane;
        if (j < kc.m) cpart[p * kc.m + j] = make_double2(sA[q], sB[q]);
    }
}

}  // namespace lampk
