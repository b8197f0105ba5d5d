// C ABI of the LAMP library (declared in include/lamp.h): argument checking,
// workspace layout, the FP64 inverse-temperature schedule, kernel dispatch and
// the graph-captured iteration loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <map>
#include <mutex>
#include <string>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>
#include <cstring>
#include <cstdlib>
#include <vector>

#include "../../include/lamp.h"
#include "lamp_kernels.hpp"
#include "lamp_mfma.hpp"
#include "lamp_batch.hpp"
#include "lamp_cost.hpp"
#include "lamp_measure.hpp"

using namespace lampk;

// Fixed workspace of lamp_step_noalloc (see scratch_address below).
static_assert(LAMP_NOALLOC_WS_BYTES % 256 == 0, "scratch size is a multiple of 256 bytes");
static __device__ __align__(256) unsigned char scratch[LAMP_NOALLOC_WS_BYTES];

namespace {

thread_local char g_err[512] = "";

lamp_status fail(lamp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(LAMP_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

constexpr int TAB = 4096;              // schedule entries per epoch

// Sweep blocks in flight per launch of the vector-ALU sweeps: 256 CUs x 8 blocks of
// 4 waves keeps 8 waves per SIMD to hide the scalar-load and transcendental latency.
// LAMP_TARGET_BLOCKS overrides it (launch-shape experiments).
int64_t target_blocks_default() {
    static const int64_t v = [] {
        const char* e = std::getenv("LAMP_TARGET_BLOCKS");
        const long long x = e ? std::atoll(e) : 0;
        return (int64_t)(x > 0 ? x : 2048);
    }();
    return v;
}
#define TARGET_BLOCKS (target_blocks_default())

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Split of the streamed extent `len` for `owned` lanes: returns elements per split.
// Split of the streamed range of a vector-ALU sweep: about `target` blocks in all, splits of
// at least 128 points.  With xcd, the count is rounded up to a multiple of 8 where the range
// allows it: the sweeps run split p of a block on XCD p mod 8 (sweep_block), so each XCD's
// L2 holds the data of its own splits only.  (The batching form hands its items to any block
// and skips the rounding.)
int64_t choose_split(int64_t owned, int64_t len, int64_t target = TARGET_BLOCKS, bool xcd = true) {
    const int64_t blocks = cdiv(owned, BLOCK);
    int64_t P = cdiv(target, blocks);
    const int64_t cap = cdiv(len, 128);
    if (xcd && cap >= 8) P = cdiv(P, 8) * 8;
    P = std::max<int64_t>(1, std::min<int64_t>(P, cap));
    return cdiv(len, P);
}

// One-dimensional grid of a sweep over the blocks of `owned` points times P splits.
unsigned sweep_grid(int64_t owned, int64_t P) { return (unsigned)(cdiv(owned, BLOCK) * P); }

struct Layout {
    size_t ctrl, sched, xc, yc, xcf, ycf, xn2, yn2, gtab, H, rowvar, rowck, rpart, cpart, nu1, th1, respart,
        dtrow, dtpart, scratch, small, xop, yop, gtabf, rowq, total;
    int64_t split_r, P_r, split_c, P_c;
    // matrix-core forms
    int prec, KP, esize;
    int64_t n_pad, m_pad, tps_r, P_rm, tps_c, P_cm;
    // FP64 matrix-core sweeps of the reference-accuracy form (d > 16)
    bool use64;
    int KP64;
    int64_t n_pad64, m_pad64, tps_r64, P_r64, tps_c64, P_c64;
    size_t xop64, yop64;
    // sweeps over an explicit cost matrix
    bool cost;
    int64_t split_rx, P_rx, split_cx, P_cx;
};

bool is_mfma(int prec) {
    return prec == LAMP_FP32_MFMA || prec == LAMP_BF16_MFMA || prec == LAMP_FP16_MFMA || prec == LAMP_FP16X3_MFMA;
}

// Smallest supported operand width >= d for the matrix-core forms (0: unsupported).
int mfma_kp(int prec, int d) {
    if (prec == LAMP_FP32_MFMA) {
        for (int kp : {4, 16, 64, 128})
            if (d <= kp) return kp;
        return 0;
    }
    if (prec == LAMP_FP16X3_MFMA) {   // three parts of d coordinates per point (split operands)
        for (int kp : {16, 64, 128, 192})
            if (3 * d <= kp) return kp;
        return 0;
    }
    for (int kp : {16, 64, 128})
        if (d <= kp) return kp;
    return 0;
}

// FP64 matrix-core operand width for the reference-accuracy form (0: vector-ALU sweeps).
// For d <= 16 the vector-ALU sweeps are faster (measured at d = 3: 25 / 32 ms against
// 36 / 45 ms for the row / column sweep at n = m = 2^18).
int fp64_kp(int d) {
    if (d <= 16) return 0;
    for (int kp : {32, 64, 128})
        if (d <= kp) return kp;
    return 0;
}

// Splits of the streamed tile range for the matrix-core sweeps: a multiple of 8 so that
// split p runs on XCD p mod 8, enough blocks to fill the chip.
void mfma_split(int64_t owned_pad, int64_t streamed_tiles, int64_t* tps, int64_t* P, int64_t rows_per_block = 128) {
    const int64_t blocks = owned_pad / rows_per_block;
    int64_t want = cdiv(TARGET_BLOCKS * 2, blocks);
    want = std::max<int64_t>(8, cdiv(want, 8) * 8);
    want = std::min<int64_t>(want, streamed_tiles);
    *tps = cdiv(streamed_tiles, want);
    *P = cdiv(streamed_tiles, *tps);
}

static_assert(LAMP_SQEUCLID == METRIC_SQEUCLID && LAMP_L1 == METRIC_L1 && LAMP_LINF == METRIC_LINF &&
                  LAMP_EXPLICIT == METRIC_EXPLICIT,
              "ground-cost codes of the ABI and the kernels agree");
static_assert(LAMP_COST_F32 == COST_F32 && LAMP_COST_BF16 == COST_BF16 && LAMP_COST_F16 == COST_F16,
              "cost element types of the ABI and the kernels agree");

Layout layout(int64_t n, int64_t m, int d, int prec = LAMP_FP32, int64_t target = TARGET_BLOCKS,
              int metric = METRIC_SQEUCLID) {
    Layout L{};
    L.split_r = choose_split(n, m, target);
    L.P_r = cdiv(m, L.split_r);
    L.split_c = choose_split(m, n, target);
    L.P_c = cdiv(n, L.split_c);
    L.prec = prec;
    L.n_pad = cdiv(n, 128) * 128;
    L.m_pad = cdiv(m, 128) * 128;
    if (is_mfma(prec)) {
        L.KP = mfma_kp(prec, d);
        L.esize = prec == LAMP_FP32_MFMA ? 4 : 2;
        mfma_split(L.n_pad, L.m_pad / 32, &L.tps_r, &L.P_rm);
        mfma_split(L.m_pad, L.n_pad / 32, &L.tps_c, &L.P_cm);
    }
    L.KP64 = fp64_kp(d);
    L.n_pad64 = cdiv(n, 64) * 64;
    L.m_pad64 = cdiv(m, 64) * 64;
    // FP64 matrix cores compute inner products only; their tile loads take 32-bit byte offsets
    // (operand copies and 16-byte point tables below 4 GiB; otherwise the vector-ALU sweeps run)
    L.use64 = L.KP64 > 0 && metric == METRIC_SQEUCLID &&
              (uint64_t)std::max(L.n_pad64, L.m_pad64) * (uint64_t)(L.KP64 * 8) < (1ull << 32) &&
              std::max(n, m) < ((int64_t)1 << 28);
    L.cost = metric == METRIC_EXPLICIT;
    if (L.cost) {
        // row sweep: 32 rows per block, column splits in whole steps; column sweep:
        // COST_COL_BLOCK columns per block, row splits of at least 64 rows
        const int64_t rb = cdiv(n, 4 * COST_ROWS);
        int64_t P = std::max<int64_t>(1, std::min<int64_t>(cdiv(target, rb), cdiv(m, COST_ROW_STEP)));
        L.split_rx = cdiv(cdiv(m, P), COST_ROW_STEP) * COST_ROW_STEP;
        L.P_rx = cdiv(m, L.split_rx);
        const int64_t cb = cdiv(m, COST_COL_BLOCK);
        P = std::max<int64_t>(1, std::min<int64_t>(cdiv(target, cb), cdiv(n, 64)));
        L.split_cx = cdiv(n, P);
        L.P_cx = cdiv(n, L.split_cx);
    }
    if (L.use64) {
        mfma_split(L.n_pad64, L.m_pad64 / 16, &L.tps_r64, &L.P_r64, 64);
        mfma_split(L.m_pad64, L.n_pad64 / 16, &L.tps_c64, &L.P_c64, 64);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    // row partials: [P][n] double2 for the sweeps, [P_r][n][d+2] for the adjoint,
    // [P_r][n][4] for the certificate's row passes
    size_t rpart_d = std::max<size_t>((size_t)L.P_r * n * std::max(4, d + 2), (size_t)4 * n);
    // column partials: [P][m] double2 for the sweeps, [P_c][m][d+1] doubles for the y adjoint
    size_t cpart_d2 = std::max<size_t>((size_t)L.P_c * m, ((size_t)L.P_c * m * (d + 1) + 1) / 2);
    if (is_mfma(prec)) {
        rpart_d = std::max<size_t>(rpart_d, (size_t)L.P_rm * n * 2);
        cpart_d2 = std::max<size_t>(cpart_d2, (size_t)L.P_cm * m);
    }
    if (L.use64) {   // D_t tracking: [P][n] double2 sums, then [P][n] cost sums
        rpart_d = std::max<size_t>(rpart_d, (size_t)L.P_r64 * n * 3);
        cpart_d2 = std::max<size_t>(cpart_d2, (size_t)L.P_c64 * m);
    }
    if (L.cost) {
        rpart_d = std::max<size_t>(rpart_d, (size_t)L.P_rx * n * 2);
        cpart_d2 = std::max<size_t>(cpart_d2, (size_t)L.P_cx * m);
    }
    L.ctrl = take(sizeof(Ctrl));
    L.sched = take(sizeof(Sched) * (TAB + 2));
    L.xc = take(sizeof(double) * n * d);
    L.yc = take(sizeof(double) * m * d);
    L.xcf = take(sizeof(float) * n * d);
    L.ycf = take(sizeof(float) * m * d);
    L.xn2 = take(sizeof(double) * n);
    L.yn2 = take(sizeof(double) * m);
    L.gtab = take(sizeof(double2) * 2 * m);
    L.H = take(sizeof(double) * n);
    L.rowvar = take(sizeof(RowVar) * n);
    L.rowck = take(sizeof(double2) * n);
    L.rpart = take(sizeof(double) * rpart_d);
    L.cpart = take(sizeof(double2) * cpart_d2);
    L.nu1 = take(sizeof(double) * m);
    L.th1 = take(sizeof(double) * m);
    L.respart = take(sizeof(double) * cdiv(m, BLOCK));
    // D_t tracking: per-row cost terms and per-block summands
    L.dtrow = take(sizeof(double) * n);
    L.dtpart = take(sizeof(double) * cdiv(m, BLOCK));
    // certificate: 4 arrays of max(n, m), Round: 9 more, the row values (4) and minima (2),
    // and d + 2 column sums
    // (the adjoint: g^A and one record of 12 d + 8 bytes per column, 16-byte aligned; the
    // adjoint with respect to y: g^A and one record of 12 d + 12 bytes per row)
    L.scratch = take(std::max({sizeof(double) * (19 * std::max(n, m) + d + 2),
                               align256(sizeof(double) * m) + (size_t)m * (size_t)((12 * d + 8 + 15) / 16 * 16),
                               align256(sizeof(double) * m) + (size_t)n * (size_t)((12 * d + 12 + 15) / 16 * 16)}));
    L.small = take(sizeof(double) * 64);
    if (is_mfma(prec)) {
        L.xop = take((size_t)L.esize * L.n_pad * L.KP);
        L.yop = take((size_t)L.esize * L.m_pad * L.KP);
        L.gtabf = take(sizeof(float2) * 2 * L.m_pad);
        L.rowq = take(sizeof(float4) * L.n_pad);
    }
    if (L.use64) {
        L.xop64 = take(sizeof(double) * L.n_pad64 * L.KP64);
        L.yop64 = take(sizeof(double) * L.m_pad64 * L.KP64);
    }
    L.total = off;
    return L;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

float2* gtabf_ptr(const Layout& L, void* ws) { return is_mfma(L.prec) ? at<float2>(ws, L.gtabf) : nullptr; }

RowVarF32 rowvar_f32(const Layout& L, void* ws) {
    return RowVarF32{at<float4>(ws, L.rowq), 1};
}

struct Resolved {
    double s, cnorm, K, tau1, tau2, alpha, beta, kappa, clipb;
    double dscale = 1.0;   // 1 / (range scale)^2 of the split FP16 operands, else 1
};

// Slot of the small-scalar area holding the split FP16 form's range scale (prep -> resolve);
// the next slot holds the running maximum its reduction folds into.
constexpr int SPLIT_SCALE_SLOT = 40;

lamp_status check_problem(const lamp_problem* p) {
    if (!p) return fail(LAMP_EINVAL, "problem is NULL");
    if (p->metric != LAMP_SQEUCLID && p->metric != LAMP_L1 && p->metric != LAMP_LINF &&
        p->metric != LAMP_EXPLICIT)
        return fail(LAMP_EINVAL, "unknown ground cost %d", p->metric);
    const bool expl = p->metric == LAMP_EXPLICIT;
    if (p->n < 1 || p->m < 1 || (!expl && p->d < 1))
        return fail(LAMP_EINVAL, "n, m and d must be >= 1 (got %lld, %lld, %d)", (long long)p->n,
                    (long long)p->m, p->d);
    if (!p->r || !p->c || (expl ? !p->cost : (!p->x || !p->y)))
        return fail(LAMP_EINVAL, "a problem array is NULL");
    if (expl && p->cost_type != LAMP_COST_F32 && p->cost_type != LAMP_COST_BF16 && p->cost_type != LAMP_COST_F16)
        return fail(LAMP_EINVAL, "unknown cost element type %d", p->cost_type);
    if (expl && p->m > (int64_t(1) << 30))   // column offsets within a row are 32-bit byte offsets
        return fail(LAMP_EINVAL, "an explicit cost matrix has at most 2^30 columns (got %lld)", (long long)p->m);
    return LAMP_OK;
}

// The explicit-cost form works with one index code per point: d = 1 whatever the
// caller set.  Returns p itself for the other ground costs.
const lamp_problem* canonical(const lamp_problem* p, lamp_problem* buf) {
    if (!p || p->metric != LAMP_EXPLICIT) return p;
    *buf = *p;
    buf->d = 1;
    return buf;
}

lamp_status check_params(const lamp_params* q) {
    if (!q) return fail(LAMP_EINVAL, "params is NULL");
    if (!(q->eta >= 0.0) || !std::isfinite(q->eta)) return fail(LAMP_EINVAL, "eta must be >= 0");
    if (!(q->tol >= 0.0)) return fail(LAMP_EINVAL, "tol must be >= 0");
    if (q->max_iter < 0) return fail(LAMP_EINVAL, "max_iter must be >= 0");
    if (q->precision != LAMP_FP32 && !is_mfma(q->precision))
        return fail(LAMP_EINVAL, "unknown precision %d", q->precision);
    if (q->track_dt != 0 && q->track_dt != 1) return fail(LAMP_EINVAL, "track_dt must be 0 or 1");
    if (q->track_dt && q->precision != LAMP_FP32)
        return fail(LAMP_EINVAL, "D_t tracking runs with precision LAMP_FP32 only");
    return LAMP_OK;
}

lamp_status check_ws(const lamp_problem* p, void* ws, size_t ws_bytes, int prec = LAMP_FP32) {
    if (is_mfma(prec) && mfma_kp(prec, p->d) == 0)
        return fail(LAMP_EINVAL, "the matrix-core forms support d <= 128, the split FP16 form d <= 64 (got %d)",
                    p->d);
    if (is_mfma(prec) && p->metric != LAMP_SQEUCLID)
        return fail(LAMP_EINVAL, "the matrix-core forms need the squared Euclidean cost (inner products)");
    const Layout L = layout(p->n, p->m, p->d, prec, TARGET_BLOCKS, p->metric);
    // the matrix-core sweeps address their operand copies with 32-bit buffer offsets
    if (is_mfma(prec) && (uint64_t)std::max(L.n_pad, L.m_pad) * (uint64_t)(L.KP * L.esize) >= (1ull << 32))
        return fail(LAMP_EINVAL, "the matrix-core forms need operand copies below 4 GiB (n, m <= %lld at d = %d)",
                    (long long)((1ll << 32) / (L.KP * L.esize) - 128), p->d);
    if (!ws) return fail(LAMP_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(LAMP_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(LAMP_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return LAMP_OK;
}

// Marginals must be strictly positive and sum to 1 (r in Delta^n, c in Delta^m with full support).
// Checked on the device, ordered on the call's stream (the marginals may have been written by
// earlier work on it); `dev6` is 6 doubles of device scratch for the two results.
lamp_status check_marginals(const lamp_problem* p, double* dev6, hipStream_t st) {
    hipLaunchKernelGGL(marginal_stats, dim3(1), dim3(1024), 0, st, p->r, p->n, dev6);
    hipLaunchKernelGGL(marginal_stats, dim3(1), dim3(1024), 0, st, p->c, p->m, dev6 + 3);
    HIPCHK(hipGetLastError());
    double h[6];
    HIPCHK(hipMemcpyAsync(h, dev6, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const char* names[2] = {"r", "c"};
    for (int q = 0; q < 2; ++q) {
        const double* v = h + 3 * q;
        if (v[1] >= 0.0)
            return fail(LAMP_EDOMAIN, "%s[%lld] = %g is not a positive finite mass", names[q], (long long)v[1], v[2]);
        if (std::fabs(v[0] - 1.0) > 1e-9) return fail(LAMP_EDOMAIN, "%s sums to %.17g, not 1", names[q], v[0]);
    }
    return LAMP_OK;
}

dim3 grid1(int64_t cnt) { return dim3((unsigned)cdiv(cnt, BLOCK)); }

template <typename T>
void prep_ops(const lamp_problem* p, const Layout& L, void* ws, hipStream_t st) {
    hipLaunchKernelGGL(prep_operands<T>, grid1(L.n_pad * L.KP), dim3(BLOCK), 0, st, at<double>(ws, L.xc), p->n,
                       p->d, L.KP, L.n_pad, at<T>(ws, L.xop));
    hipLaunchKernelGGL(prep_operands<T>, grid1(L.m_pad * L.KP), dim3(BLOCK), 0, st, at<double>(ws, L.yc), p->m,
                       p->d, L.KP, L.m_pad, at<T>(ws, L.yop));
}

lamp_status prep_L(const lamp_problem* p, const Layout& L, void* ws, hipStream_t st) {
    const int prec = L.prec;
    if (L.cost) {
        hipLaunchKernelGGL(prep_cost_codes, grid1(p->n), dim3(BLOCK), 0, st, p->n, 0, at<double>(ws, L.xc),
                           at<double>(ws, L.xn2));
        hipLaunchKernelGGL(prep_cost_codes, grid1(p->m), dim3(BLOCK), 0, st, p->m, 1, at<double>(ws, L.yc),
                           at<double>(ws, L.yn2));
        HIPCHK(hipGetLastError());
        return LAMP_OK;
    }
    hipLaunchKernelGGL(prep_points, grid1(p->n), dim3(BLOCK), 0, st, p->x, p->n, p->d, p->x, p->y,
                       at<double>(ws, L.xc), at<double>(ws, L.xn2), at<float>(ws, L.xcf), p->metric);
    hipLaunchKernelGGL(prep_points, grid1(p->m), dim3(BLOCK), 0, st, p->y, p->m, p->d, p->x, p->y,
                       at<double>(ws, L.yc), at<double>(ws, L.yn2), at<float>(ws, L.ycf), p->metric);
    if (L.use64) {
        hipLaunchKernelGGL(prep_operands64, grid1(L.n_pad64 * L.KP64), dim3(BLOCK), 0, st, at<double>(ws, L.xc),
                           p->n, p->d, L.KP64, L.n_pad64, at<double>(ws, L.xop64));
        hipLaunchKernelGGL(prep_operands64, grid1(L.m_pad64 * L.KP64), dim3(BLOCK), 0, st, at<double>(ws, L.yc),
                           p->m, p->d, L.KP64, L.m_pad64, at<double>(ws, L.yop64));
    }
    if (is_mfma(prec)) {
        if (prec == LAMP_FP32_MFMA) {
            prep_ops<float>(p, L, ws, st);
        } else if (prec == LAMP_BF16_MFMA) {
            prep_ops<__bf16>(p, L, ws, st);
        } else if (prec == LAMP_FP16X3_MFMA) {
            double* scale = at<double>(ws, L.small) + SPLIT_SCALE_SLOT;
            auto* mbits = reinterpret_cast<unsigned long long*>(scale + 1);
            const int64_t cnt = std::max(p->n, p->m) * p->d;
            const int blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(1, cdiv(cnt, BLOCK)));
            hipLaunchKernelGGL(split_scale_clear, dim3(1), dim3(1), 0, st, mbits);
            hipLaunchKernelGGL(split_scale_max, dim3(blocks), dim3(BLOCK), 0, st, (const double*)at<double>(ws, L.xc),
                               p->n * p->d, (const double*)at<double>(ws, L.yc), p->m * p->d, mbits);
            hipLaunchKernelGGL(split_scale_final, dim3(1), dim3(1), 0, st, (const unsigned long long*)mbits, scale);
            hipLaunchKernelGGL(prep_operands_split, grid1(L.n_pad * L.KP), dim3(BLOCK), 0, st,
                               (const double*)at<double>(ws, L.xc), p->n, p->d, L.KP, L.n_pad, (const double*)scale,
                               0, at<_Float16>(ws, L.xop));
            hipLaunchKernelGGL(prep_operands_split, grid1(L.m_pad * L.KP), dim3(BLOCK), 0, st,
                               (const double*)at<double>(ws, L.yc), p->m, p->d, L.KP, L.m_pad, (const double*)scale,
                               1, at<_Float16>(ws, L.yop));
        } else {
            prep_ops<_Float16>(p, L, ws, st);
        }
        if (L.m_pad > p->m)
            hipLaunchKernelGGL(pad_gtabf, grid1(L.m_pad - p->m), dim3(BLOCK), 0, st, p->m, L.m_pad,
                               at<float2>(ws, L.gtabf));
        if (L.n_pad > p->n)
            hipLaunchKernelGGL(pad_rowq, grid1(L.n_pad - p->n), dim3(BLOCK), 0, st, p->n, L.n_pad,
                               at<float4>(ws, L.rowq));
    }
    HIPCHK(hipGetLastError());
    return LAMP_OK;
}

lamp_status prep(const lamp_problem* p, void* ws, hipStream_t st, int prec = LAMP_FP32) {
    return prep_L(p, layout(p->n, p->m, p->d, prec, TARGET_BLOCKS, p->metric), ws, st);
}

// f(tag) with tag a null pointer to the element type of an explicit cost matrix.
template <typename F>
void by_cost_type(int cost_type, F&& f) {
    if (cost_type == COST_BF16) f(static_cast<__bf16*>(nullptr));
    else if (cost_type == COST_F16) f(static_cast<_Float16*>(nullptr));
    else f(static_cast<float*>(nullptr));
}

// ------------------------------------------------------------------ dispatch by d
#define LAMP_FOR_D(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(16)
template <int V>
using IC = std::integral_constant<int, V>;

// Launches the vector-ALU kernel of metric M and dimension d if one is compiled
// (d in 1..8 and 16 for the squared Euclidean cost, 1..4 for l1 / l_inf):
// launch(IC<D>) issues it.  Returns false for the generic-d kernel.
template <int M, typename F>
bool valu_dispatch(int d, F&& launch) {
    switch (d) {
        case 1: launch(IC<1>{}); return true;
        case 2: launch(IC<2>{}); return true;
        case 3: launch(IC<3>{}); return true;
        case 4: launch(IC<4>{}); return true;
        default: break;
    }
    if constexpr (M == METRIC_SQEUCLID) {
        switch (d) {
            case 5: launch(IC<5>{}); return true;
            case 6: launch(IC<6>{}); return true;
            case 7: launch(IC<7>{}); return true;
            case 8: launch(IC<8>{}); return true;
            case 16: launch(IC<16>{}); return true;
            default: break;
        }
    }
    return false;
}

// The certificate's pair passes: the compiled dimensions of the vector-ALU sweeps and, for the
// squared Euclidean cost, 32 and 64 (the thread's own point in registers and the streamed
// point through scalar loads; the run-time form loads both points' coordinates per pair,
// 6.6 s for a certificate at n = m = 2^16, d = 64).
template <int M, typename F>
bool cert_dispatch(int d, F&& launch) {
    if (valu_dispatch<M>(d, launch)) return true;
    if constexpr (M == METRIC_SQEUCLID) {
        if (d == 32) {
            launch(IC<32>{});
            return true;
        }
        if (d == 64) {
            launch(IC<64>{});
            return true;
        }
    }
    return false;
}

// f(IC<M>) for the run-time metric.
template <typename F>
bool by_metric(int metric, F&& f) {
    if (metric == METRIC_EXPLICIT) return false;   // the run-time (index code) form
    if (metric == METRIC_L1) return f(IC<METRIC_L1>{});
    if (metric == METRIC_LINF) return f(IC<METRIC_LINF>{});
    return f(IC<METRIC_SQEUCLID>{});
}

template <int KP>
void row_extreme64(const Layout& L, Consts kc, void* ws, const double* a, double sgn, hipStream_t st) {
    const int64_t n_waves = L.n_pad64 / 16;
    dim3 g((unsigned)(cdiv(n_waves, 4) * L.P_r64));
    hipLaunchKernelGGL((row_extreme_mfma64<KP>), g, dim3(BLOCK), 0, st, kc, at<double>(ws, L.xop64),
                       at<double>(ws, L.yop64), a, sgn, at<double>(ws, L.rpart), L.tps_r64, (int)L.P_r64,
                       L.m_pad64 / 16, n_waves);
}

// Number of partial minima written by launch_row_extreme.
int extreme_parts(const Layout& L) {
    if (L.cost) return (int)L.P_rx;
    return (int)(L.use64 ? L.P_r64 : L.P_r);
}

void launch_row_extreme(const Layout& L, Consts kc, int d, void* ws, const double* a, double sgn,
                        hipStream_t st) {
    if (L.cost) {
        dim3 g((unsigned)cdiv(kc.n, 4 * COST_ROWS), (unsigned)L.P_rx);
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((row_extreme_cost<T>), g, dim3(BLOCK), 0, st, kc, a, sgn, at<double>(ws, L.rpart), L.split_rx);
        });
        return;
    }
    if (L.use64) {
        switch (L.KP64) {
            case 32: row_extreme64<32>(L, kc, ws, a, sgn, st); return;
            case 64: row_extreme64<64>(L, kc, ws, a, sgn, st); return;
            default: row_extreme64<128>(L, kc, ws, a, sgn, st); return;
        }
    }
    const dim3 g(sweep_grid(kc.n, L.P_r));
    double* part = at<double>(ws, L.rpart);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            hipLaunchKernelGGL((row_extreme<decltype(m)::value, decltype(dd)::value>), g, dim3(BLOCK), 0, st, kc,
                               xc, yc, a, sgn, part, L.split_r);
        });
    });
    if (!done) hipLaunchKernelGGL(row_extreme_dyn, g, dim3(BLOCK), 0, st, kc, d, xc, yc, a, sgn, part, L.split_r);
}

template <typename T, int KP>
void row_mfma(const Layout& L, Consts kc, void* ws, hipStream_t st) {
    const int64_t n_waves = L.n_pad / 32;
    dim3 g((unsigned)(cdiv(n_waves, 4) * L.P_rm));
    hipLaunchKernelGGL((row_sweep_mfma_lds<T, KP>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<T>(ws, L.xop), at<T>(ws, L.yop), at<float2>(ws, L.gtabf), L.m_pad, at<double>(ws, L.H),
                       at<double2>(ws, L.rpart), L.tps_r, (int)L.P_rm, L.m_pad / 32, n_waves);
}

template <typename T, int KP>
void col_mfma(const Layout& L, Consts kc, void* ws, hipStream_t st) {
    const int64_t m_waves = L.m_pad / 32;
    dim3 g((unsigned)(cdiv(m_waves, 4) * L.P_cm));
    hipLaunchKernelGGL((col_sweep_mfma_t_lds<T, KP>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl),
                       at<Sched>(ws, L.sched), kc, at<T>(ws, L.xop), at<T>(ws, L.yop), at<float2>(ws, L.gtabf),
                       L.m_pad, at<float4>(ws, L.rowq), at<double2>(ws, L.cpart), L.tps_c, (int)L.P_cm,
                       L.n_pad / 32, m_waves);
}

template <bool ROW>
void sweep_mfma(const Layout& L, Consts kc, void* ws, hipStream_t st) {
#define MF(T, K) \
    if (ROW) row_mfma<T, K>(L, kc, ws, st); else col_mfma<T, K>(L, kc, ws, st); return;
    if (L.prec == LAMP_FP32_MFMA) {
        switch (L.KP) {
            case 4: MF(float, 4)
            case 16: MF(float, 16)
            case 64: MF(float, 64)
            default: MF(float, 128)
        }
    } else if (L.prec == LAMP_BF16_MFMA) {
        switch (L.KP) {
            case 16: MF(__bf16, 16)
            case 64: MF(__bf16, 64)
            default: MF(__bf16, 128)
        }
    } else {
        switch (L.KP) {
            case 16: MF(_Float16, 16)
            case 64: MF(_Float16, 64)
            case 128: MF(_Float16, 128)
            default: MF(_Float16, 192)
        }
    }
#undef MF
}

template <int KP>
void row_mfma64(const Layout& L, Consts kc, void* ws, hipStream_t st) {
    const int64_t n_waves = L.n_pad64 / 16;
    dim3 g((unsigned)(cdiv(n_waves, 4) * L.P_r64));
    hipLaunchKernelGGL((row_sweep_mfma64_lds<KP>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.xop64), at<double>(ws, L.yop64), at<double2>(ws, L.gtab),
                       at<double>(ws, L.H), at<double2>(ws, L.rpart), L.tps_r64, (int)L.P_r64, L.m_pad64 / 16,
                       n_waves);
}

// The D_t-tracked FP64 matrix-core row sweep: cost sums into tpart ([P_r64][n]).
template <int KP>
void row_mfma64_dt(const Layout& L, Consts kc, void* ws, double* tpart, hipStream_t st) {
    const int64_t n_waves = L.n_pad64 / 16;
    dim3 g((unsigned)(cdiv(n_waves, 4) * L.P_r64));
    hipLaunchKernelGGL((row_sweep_mfma64_dt<KP>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.xop64), at<double>(ws, L.yop64), at<double2>(ws, L.gtab),
                       at<double>(ws, L.H), at<double2>(ws, L.rpart), L.tps_r64, (int)L.P_r64, L.m_pad64 / 16,
                       n_waves, at<double>(ws, L.xn2), at<double>(ws, L.yn2), tpart);
}

template <int KP>
void col_mfma64(const Layout& L, Consts kc, void* ws, hipStream_t st) {
    const int64_t m_waves = L.m_pad64 / 16;
    dim3 g((unsigned)(cdiv(m_waves, 4) * L.P_c64));
    hipLaunchKernelGGL((col_sweep_mfma64_lds<KP>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.xop64), at<double>(ws, L.yop64), at<double2>(ws, L.gtab),
                       at<RowVar>(ws, L.rowvar), at<double2>(ws, L.cpart), L.tps_c64, (int)L.P_c64,
                       L.n_pad64 / 16, m_waves);
}

template <bool ROW>
void sweep_mfma64(const Layout& L, Consts kc, void* ws, hipStream_t st) {
    switch (L.KP64) {
        case 32: if (ROW) row_mfma64<32>(L, kc, ws, st); else col_mfma64<32>(L, kc, ws, st); return;
        case 64: if (ROW) row_mfma64<64>(L, kc, ws, st); else col_mfma64<64>(L, kc, ws, st); return;
        default: if (ROW) row_mfma64<128>(L, kc, ws, st); else col_mfma64<128>(L, kc, ws, st); return;
    }
}

// Number of row / column partials written by the sweeps of this layout.
int row_parts(const Layout& L) {
    if (L.cost) return (int)L.P_rx;
    return (int)(is_mfma(L.prec) ? L.P_rm : (L.use64 ? L.P_r64 : L.P_r));
}
int col_parts(const Layout& L) {
    if (L.cost) return (int)L.P_cx;
    return (int)(is_mfma(L.prec) ? L.P_cm : (L.use64 ? L.P_c64 : L.P_c));
}

void launch_row_sweep(const Layout& L, Consts kc, int d, void* ws, hipStream_t st) {
    if (L.cost) {
        dim3 g((unsigned)cdiv(kc.n, 4 * COST_ROWS), (unsigned)L.P_rx);
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((row_sweep_cost<T>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched), kc,
                           at<double2>(ws, L.gtab), at<double>(ws, L.H), at<double2>(ws, L.rpart), L.split_rx);
        });
        return;
    }
    if (is_mfma(L.prec)) {
        sweep_mfma<true>(L, kc, ws, st);
        return;
    }
    if (L.use64) {
        sweep_mfma64<true>(L, kc, ws, st);
        return;
    }
    const dim3 g(sweep_grid(kc.n, L.P_r));
    const Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
    const Sched* sch = at<Sched>(ws, L.sched);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const double2* gt = at<double2>(ws, L.gtab);
    const double* H = at<double>(ws, L.H);
    double2* part = at<double2>(ws, L.rpart);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            hipLaunchKernelGGL((row_sweep<decltype(m)::value, decltype(dd)::value>), g, dim3(BLOCK), 0, st, ctrl,
                               sch, kc, xc, yc, gt, H, part, L.split_r);
        });
    });
    if (!done)
        hipLaunchKernelGGL(row_sweep_dyn, g, dim3(BLOCK), 0, st, ctrl, sch, kc, d, xc, yc, gt, H, part, L.split_r);
}

void launch_col_sweep(const Layout& L, Consts kc, int d, void* ws, hipStream_t st) {
    if (L.cost) {
        dim3 g((unsigned)cdiv(kc.m, COST_COL_BLOCK), (unsigned)L.P_cx);
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((col_sweep_cost<T>), g, dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched), kc,
                           at<double2>(ws, L.gtab), at<RowVar>(ws, L.rowvar), at<double2>(ws, L.cpart),
                           L.split_cx);
        });
        return;
    }
    if (is_mfma(L.prec)) {
        sweep_mfma<false>(L, kc, ws, st);
        return;
    }
    if (L.use64) {
        sweep_mfma64<false>(L, kc, ws, st);
        return;
    }
    const dim3 g(sweep_grid(kc.m, L.P_c));
    const Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
    const Sched* sch = at<Sched>(ws, L.sched);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const double2* gt = at<double2>(ws, L.gtab);
    const RowVar* rv = at<RowVar>(ws, L.rowvar);
    const double2* ck = at<double2>(ws, L.rowck);
    double2* part = at<double2>(ws, L.cpart);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            hipLaunchKernelGGL((col_sweep<decltype(m)::value, decltype(dd)::value>), g, dim3(BLOCK), 0, st, ctrl,
                               sch, kc, xc, yc, gt, rv, ck, part, L.split_c);
        });
    });
    if (!done)
        hipLaunchKernelGGL(col_sweep_dyn, g, dim3(BLOCK), 0, st, ctrl, sch, kc, d, xc, yc, gt, rv, ck, part, L.split_c);
}

void launch_adjoint(const Layout& L, Consts kc, int d, void* ws, double cA, const double* gA,
                    hipStream_t st) {
    const dim3 g(sweep_grid(kc.n, L.P_r));
    double* part = at<double>(ws, L.rpart);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const float* ycf = at<float>(ws, L.ycf);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            constexpr int D = decltype(dd)::value;
            // the column records follow gA in the scratch region (sized for them in layout())
            auto* cols = reinterpret_cast<AdjCol<D>*>(at<char>(ws, L.scratch) + align256(sizeof(double) * kc.m));
            hipLaunchKernelGGL((adjoint_pack<D>), grid1(kc.m), dim3(BLOCK), 0, st, kc.m, yc, ycf, gA, cols);
            hipLaunchKernelGGL((adjoint_sweep<decltype(m)::value, D>), g, dim3(BLOCK), 0, st, kc, cA, xc,
                               (const AdjCol<D>*)cols, part, L.split_r);
        });
    });
    if (!done)
        hipLaunchKernelGGL(adjoint_sweep_dyn, g, dim3(BLOCK), 0, st, kc, d, cA, xc, yc, ycf, gA, part, L.split_r);
}

// <C, X^t> in one pass over the pairs: per row the split sums (M, Z, S_C), then s r_i S_C / Z
// per row into rows (n doubles) and their fixed-order sum into *out (device).
void launch_cost(const Layout& L, Consts kc, int d, void* ws, double cA, const double* gA, const double* r,
                 double* rows, double* out, hipStream_t st) {
    const dim3 g(sweep_grid(kc.n, L.P_r));
    double* part = at<double>(ws, L.rpart);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const double* xn2 = at<double>(ws, L.xn2);
    const double* yn2 = at<double>(ws, L.yn2);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            constexpr int D = decltype(dd)::value;
            // the column records follow gA in the scratch region (sized for them in layout())
            auto* cols = reinterpret_cast<CostCol<D>*>(at<char>(ws, L.scratch) + align256(sizeof(double) * kc.m));
            hipLaunchKernelGGL((cost_pack<D>), grid1(kc.m), dim3(BLOCK), 0, st, kc.m, yc, yn2, gA, cols);
            hipLaunchKernelGGL((cost_sweep<decltype(m)::value, D>), g, dim3(BLOCK), 0, st, kc, cA, xc, xn2,
                               (const CostCol<D>*)cols, part, L.split_r);
        });
    });
    if (!done)
        hipLaunchKernelGGL(cost_sweep_dyn, g, dim3(BLOCK), 0, st, kc, d, cA, xc, yc, xn2, yn2, gA, part, L.split_r);
    hipLaunchKernelGGL(cost_finish, grid1(kc.n), dim3(BLOCK), 0, st, kc, (int)L.P_r, r, (const double*)part, rows);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, (const double*)rows, kc.n, kc.n, 1, out);
}

__global__ void fill_scaled(int64_t cnt, double f, const double* __restrict__ in, double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = f * in[i];
}

lamp_status max_sqdist_L(const lamp_problem* p, const Layout& L, void* ws, hipStream_t st, double* out_host) {
    Consts kc{};
    kc.n = p->n;
    kc.m = p->m;
    kc.metric = p->metric;
    kc.cost = p->metric == LAMP_EXPLICIT ? p->cost : nullptr;
    kc.cost_type = p->metric == LAMP_EXPLICIT ? p->cost_type : COST_F32;
    double* a = at<double>(ws, L.scratch);
    double* rowmax = a + std::max(p->n, p->m);
    hipLaunchKernelGGL(fill_scaled, grid1(p->m), dim3(BLOCK), 0, st, p->m, -0.5, at<double>(ws, L.yn2), a);
    launch_row_extreme(L, kc, p->d, ws, a, +1.0, st);
    hipLaunchKernelGGL(row_extreme_merge, grid1(p->n), dim3(BLOCK), 0, st, kc, at<double>(ws, L.rpart),
                       extreme_parts(L), at<double>(ws, L.xn2), 1, rowmax);
    hipLaunchKernelGGL(reduce_max, dim3(1), dim3(1024), 0, st, rowmax, p->n, at<double>(ws, L.small));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out_host, at<double>(ws, L.small), sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return LAMP_OK;
}

lamp_status max_sqdist(const lamp_problem* p, void* ws, hipStream_t st, double* out_host, int prec) {
    return max_sqdist_L(p, layout(p->n, p->m, p->d, prec, TARGET_BLOCKS, p->metric), ws, st, out_host);
}

lamp_status resolve_L(const lamp_problem* p, const lamp_params* q, const Layout& L, void* ws, hipStream_t st,
                      Resolved* R) {
    double s = p->cost_scale, cn = p->cost_norm;
    if (!(s > 0.0) || !(cn > 0.0)) {
        double md = 0.0;
        lamp_status e = max_sqdist_L(p, L, ws, st, &md);
        if (e != LAMP_OK) return e;
        if (!(md > 0.0)) return fail(LAMP_EDOMAIN, "all pairwise distances are zero");
        if (!(s > 0.0)) {
            s = 1.0 / md;
            cn = 1.0;
        } else {
            cn = s * md;
        }
    }
    R->s = s;
    R->cnorm = cn;
    R->K = 2.0 * cn;
    R->tau1 = q->tau1 > 0.0 ? q->tau1 : 1.0 / (2.0 * cn);
    R->tau2 = q->tau2 > 0.0 ? q->tau2 : 1.0 / (2.0 * cn);
    R->alpha = q->alpha > 0.0 ? q->alpha : 0.01;
    R->beta = q->beta > 0.0 ? q->beta : 1.1;
    R->kappa = 2.0 * R->tau2 * cn;
    R->clipb = std::tanh(R->beta / 2.0);
    if (R->tau1 * q->eta > 1.0) return fail(LAMP_EINVAL, "tau1 * eta = %g > 1", R->tau1 * q->eta);
    R->dscale = 1.0;
    if (L.prec == LAMP_FP16X3_MFMA) {
        double sc = 0.0;
        HIPCHK(hipMemcpyAsync(&sc, at<double>(ws, L.small) + SPLIT_SCALE_SLOT, sizeof(double), hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipStreamSynchronize(st));
        R->dscale = 1.0 / (sc * sc);
    }
    return LAMP_OK;
}

lamp_status resolve(const lamp_problem* p, const lamp_params* q, void* ws, hipStream_t st, Resolved* R) {
    return resolve_L(p, q, layout(p->n, p->m, p->d, q->precision, TARGET_BLOCKS, p->metric), ws, st, R);
}

Consts make_consts(const lamp_problem* p, const Resolved& R) {
    Consts kc;
    kc.n = p->n;
    kc.m = p->m;
    kc.s = R.s;
    kc.K = R.K;
    kc.kappa = R.kappa;
    kc.alpha_m = R.alpha / (double)p->m;
    kc.clipb = R.clipb;
    kc.metric = p->metric;
    kc.factor_cols = 2.0 * LOG2E * R.K * R.tau1 <= 64.0;
    kc.dscale = R.dscale;
    kc.cost = p->metric == LAMP_EXPLICIT ? p->cost : nullptr;
    kc.cost_type = p->metric == LAMP_EXPLICIT ? p->cost_type : COST_F32;
    return kc;
}

// lam_{t+1} = tau1 + lam_t (1 - tau1 eta): the inverse form of step:eta_update.
#pragma clang fp contract(off)
double next_lam(double lam, double tau1, double eta) { return tau1 + lam * (1.0 - tau1 * eta); }
#pragma clang fp contract(on)

// Fills `cnt` schedule entries of tab[] starting at lam_t0; returns lam_{t0 + cnt}.
double fill_sched(Sched* tab, int cnt, double lam0, double tau1, double eta) {
    double l0 = lam0;
    for (int k = 0; k < cnt; ++k) {
        double l1 = next_lam(l0, tau1, eta);
        double l2 = next_lam(l1, tau1, eta);
        tab[k] = Sched{};
        tab[k].lamA = l0;
        tab[k].lamB = l1;
        tab[k].w = tau1 / l1;
        tab[k].lamC = l2;
        tab[k].w2 = tau1 / l2;
        l0 = l1;
    }
    return l0;
}

template <typename T, int KP>
void extreme_mfma(const Layout& L, Consts kc, void* ws, const Ctrl* ctrl, const Sched* sched, hipStream_t st) {
    const int64_t n_waves = L.n_pad / 32;
    dim3 g((unsigned)(cdiv(n_waves, 4) * L.P_rm));
    hipLaunchKernelGGL((row_extreme_mfma_lds<T, KP>), g, dim3(BLOCK), 0, st, ctrl, sched, kc, at<T>(ws, L.xop),
                       at<T>(ws, L.yop), at<float2>(ws, L.gtabf), L.m_pad, at<double>(ws, L.rpart), L.tps_r,
                       (int)L.P_rm, L.m_pad / 32, n_waves);
}

void launch_extreme_mfma(const Layout& L, Consts kc, void* ws, const Ctrl* ctrl, const Sched* sched,
                         hipStream_t st) {
#define EX(T, K) \
    extreme_mfma<T, K>(L, kc, ws, ctrl, sched, st); return;
    if (L.prec == LAMP_FP32_MFMA) {
        switch (L.KP) {
            case 4: EX(float, 4)
            case 16: EX(float, 16)
            case 64: EX(float, 64)
            default: EX(float, 128)
        }
    } else if (L.prec == LAMP_BF16_MFMA) {
        switch (L.KP) {
            case 16: EX(__bf16, 16)
            case 64: EX(__bf16, 64)
            default: EX(__bf16, 128)
        }
    } else {
        switch (L.KP) {
            case 16: EX(_Float16, 16)
            case 64: EX(_Float16, 64)
            case 128: EX(_Float16, 128)
            default: EX(_Float16, 192)
        }
    }
#undef EX
}

// Offsets for the first row sweep of a call: h_i = min_j(-g^B_j/cfac^B - x~.y~), exact in
// FP64 for the FP64-argument form; for the matrix-core forms from their own operand copies
// and FP32 arithmetic (an offset only has to keep the sums in range).
void launch_offsets(const Layout& L, Consts kc, int d, void* ws, hipStream_t st, const Ctrl* ctrl = nullptr,
                    const Sched* sched = nullptr) {
    if (is_mfma(L.prec)) {
        launch_extreme_mfma(L, kc, ws, ctrl ? ctrl : at<Ctrl>(ws, L.ctrl), sched ? sched : at<Sched>(ws, L.sched),
                            st);
        hipLaunchKernelGGL(row_extreme_merge, grid1(kc.n), dim3(BLOCK), 0, st, kc, at<double>(ws, L.rpart),
                           (int)L.P_rm, (const double*)nullptr, 0, at<double>(ws, L.H));
        return;
    }
    double* a = at<double>(ws, L.scratch);
    hipLaunchKernelGGL(offset_coeffs, grid1(kc.m), dim3(BLOCK), 0, st, ctrl ? ctrl : at<Ctrl>(ws, L.ctrl),
                       sched ? sched : at<Sched>(ws, L.sched), kc, at<double2>(ws, L.gtab), a);
    launch_row_extreme(L, kc, d, ws, a, -1.0, st);
    hipLaunchKernelGGL(row_extreme_merge, grid1(kc.n), dim3(BLOCK), 0, st, kc, at<double>(ws, L.rpart),
                       extreme_parts(L), (const double*)nullptr, 0, at<double>(ws, L.H));
}

// Owns the captured iteration graph of a solve call: destroyed on every return path.
struct GraphGuard {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphGuard() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

struct IterArgs {
    DualBufs buf;
    TraceCols tc;
    double* log_za;
    double* log_zb;
    bool track_dt;
};

// <C, Xbar^{t+1}> of the running iteration into ctrl->dt_cost (D_t tracking); runs after
// the row sweep, with the offsets and column table that sweep used.
void launch_dt_cost(const lamp_problem* p, const Layout& L, Consts kc, void* ws, hipStream_t st) {
    Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
    const Sched* sch = at<Sched>(ws, L.sched);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const double* xn2 = at<double>(ws, L.xn2);
    const double* yn2 = at<double>(ws, L.yn2);
    const double2* gt = at<double2>(ws, L.gtab);
    const double* H = at<double>(ws, L.H);
    double* out = at<double>(ws, L.dtrow);
    const int d = p->d;
    if (L.cost) {
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((dt_cost_rows_cost<T>), dim3((unsigned)cdiv(kc.n, 4 * COST_ROWS)), dim3(BLOCK), 0, st, ctrl, sch,
                           kc, gt, H, p->r, out);
        });
        hipLaunchKernelGGL(dt_cost_total, dim3(1), dim3(1024), 0, st, ctrl, (const double*)out, kc.n);
        return;
    }
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            hipLaunchKernelGGL((dt_cost_rows<decltype(m)::value, decltype(dd)::value>), grid1(kc.n), dim3(BLOCK), 0,
                               st, ctrl, sch, kc, xc, yc, xn2, yn2, gt, H, p->r, out);
        });
    });
    if (!done)
        hipLaunchKernelGGL(dt_cost_rows_dyn, grid1(kc.n), dim3(BLOCK), 0, st, ctrl, sch, kc, d, xc, yc, xn2, yn2, gt,
                           H, p->r, out);
    hipLaunchKernelGGL(dt_cost_total, dim3(1), dim3(1024), 0, st, ctrl, (const double*)out, kc.n);
}

// The row sweep of a D_t-tracked iteration with <C, Xbar^{t+1}> fused into it (FP64
// matrix-core sweeps, and vector-ALU sweeps of a templated dimension): the sweep, then
// dt_rows_finish and dt_cost_total.  The cost partials sit behind the sweep's [P][n] double2
// partials in the row partial buffer (sized for 4 P_r n and 3 P_r64 n doubles).  Returns false,
// launching nothing, for the other sweeps.
bool launch_row_sweep_dt(const lamp_problem* p, const Layout& L, Consts kc, void* ws, hipStream_t st) {
    if (L.cost || is_mfma(L.prec)) return false;
    if (L.use64) {
        double* tpart = at<double>(ws, L.rpart) + 2 * L.P_r64 * kc.n;
        switch (L.KP64) {
            case 32: row_mfma64_dt<32>(L, kc, ws, tpart, st); break;
            case 64: row_mfma64_dt<64>(L, kc, ws, tpart, st); break;
            default: row_mfma64_dt<128>(L, kc, ws, tpart, st); break;
        }
        Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
        double* out = at<double>(ws, L.dtrow);
        hipLaunchKernelGGL(dt_rows_finish_dyn, grid1(kc.n), dim3(BLOCK), 0, st, ctrl, at<Sched>(ws, L.sched), kc,
                           p->d, at<double>(ws, L.xc), at<double>(ws, L.yc), at<double>(ws, L.xn2),
                           at<double>(ws, L.yn2), at<double2>(ws, L.gtab), p->r, at<double2>(ws, L.rpart),
                           (const double*)tpart, (int)L.P_r64, out);
        hipLaunchKernelGGL(dt_cost_total, dim3(1), dim3(1024), 0, st, ctrl, (const double*)out, kc.n);
        return true;
    }
    const dim3 g(sweep_grid(kc.n, L.P_r));
    Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
    const Sched* sch = at<Sched>(ws, L.sched);
    const double* xc = at<double>(ws, L.xc);
    const double* yc = at<double>(ws, L.yc);
    const double* xn2 = at<double>(ws, L.xn2);
    const double* yn2 = at<double>(ws, L.yn2);
    const double2* gt = at<double2>(ws, L.gtab);
    const double* H = at<double>(ws, L.H);
    double2* part = at<double2>(ws, L.rpart);
    double* tpart = at<double>(ws, L.rpart) + 2 * L.P_r * kc.n;
    double* out = at<double>(ws, L.dtrow);
    return by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(p->d, [&](auto dd) {
            constexpr int M = decltype(m)::value, D = decltype(dd)::value;
            hipLaunchKernelGGL((row_sweep_dt<M, D>), g, dim3(BLOCK), 0, st, ctrl, sch, kc, xc, yc, gt, H, part,
                               L.split_r, xn2, yn2, tpart);
            hipLaunchKernelGGL((dt_rows_finish<M, D>), grid1(kc.n), dim3(BLOCK), 0, st, ctrl, sch, kc, xc, yc, xn2,
                               yn2, gt, p->r, (const double2*)part, (const double*)tpart, (int)L.P_r, out);
            hipLaunchKernelGGL(dt_cost_total, dim3(1), dim3(1024), 0, st, ctrl, (const double*)out, kc.n);
        });
    });
}

void launch_iteration(const lamp_problem* p, const Layout& L, Consts kc, void* ws, const IterArgs& ia,
                      hipStream_t st) {
    Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
    const Sched* sch = at<Sched>(ws, L.sched);
    if (!(ia.track_dt && launch_row_sweep_dt(p, L, kc, ws, st))) {
        launch_row_sweep(L, kc, p->d, ws, st);
        if (ia.track_dt) launch_dt_cost(p, L, kc, ws, st);
    }
    RowVarF32 rf{nullptr, 0};
    if (is_mfma(L.prec)) rf = rowvar_f32(L, ws);
    hipLaunchKernelGGL(row_finish, grid1(kc.n), dim3(BLOCK), 0, st, ctrl, sch, kc, p->d, at<double>(ws, L.xc),
                       at<double>(ws, L.yc), at<double2>(ws, L.gtab), p->r, at<double>(ws, L.xn2),
                       at<double2>(ws, L.rpart), row_parts(L), at<double>(ws, L.H), at<RowVar>(ws, L.rowvar),
                       at<double2>(ws, L.rowck), ia.log_za, ia.log_zb, rf);
    launch_col_sweep(L, kc, p->d, ws, st);
    hipLaunchKernelGGL(dual_update, grid1(kc.m), dim3(BLOCK), 0, st, ctrl, sch, kc, at<double2>(ws, L.cpart),
                       col_parts(L), p->c, at<double>(ws, L.yn2), ia.buf, at<double2>(ws, L.gtab),
                       gtabf_ptr(L, ws), L.m_pad, at<double>(ws, L.respart), ia.tc,
                       ia.track_dt ? at<double>(ws, L.dtpart) : (double*)nullptr);
    hipLaunchKernelGGL(dual_finish, dim3(1), dim3(BLOCK), 0, st, ctrl, sch, (const double*)at<double>(ws, L.respart),
                       ia.track_dt ? (const double*)at<double>(ws, L.dtpart) : (const double*)nullptr,
                       cdiv(kc.m, BLOCK));
}

lamp_status upload_ctrl(void* ws, const Layout& L, int64_t t, int64_t t_end, int64_t t_base, double tol,
                        hipStream_t st, Ctrl* host, double dt_acc = 0.0) {
    host->dt_acc = dt_acc;
    host->dt_cost = 0.0;
    host->t = t;
    host->t_end = t_end;
    host->t_base = t_base;
    host->t_done = -1;
    host->done = 0;
    host->err = 0;
    host->fallbacks = 0;
    host->tol = tol;
    host->res_last = -1.0;
    HIPCHK(hipMemcpyAsync(at<Ctrl>(ws, L.ctrl), host, sizeof(Ctrl), hipMemcpyHostToDevice, st));
    return LAMP_OK;
}

lamp_status common_setup(const lamp_problem* p, const lamp_params* q, void* ws, size_t ws_bytes,
                         hipStream_t st, Resolved* R) {
    lamp_status e;
    if ((e = check_problem(p)) != LAMP_OK) return e;
    if ((e = check_params(q)) != LAMP_OK) return e;
    if ((e = check_ws(p, ws, ws_bytes, q->precision)) != LAMP_OK) return e;
    if ((e = check_marginals(p, at<double>(ws, layout(p->n, p->m, p->d, q->precision, TARGET_BLOCKS, p->metric).small),
                             st)) != LAMP_OK)
        return e;
    if ((e = prep(p, ws, st, q->precision)) != LAMP_OK) return e;
    return resolve(p, q, ws, st, R);
}

lamp_status check_state(const lamp_state* s) {
    if (!s || !s->nu || !s->theta) return fail(LAMP_EINVAL, "state or its arrays are NULL");
    if (s->t < 0 || !(s->inv_eta >= 0.0)) return fail(LAMP_EINVAL, "state has t < 0 or inv_eta < 0");
    return LAMP_OK;
}

// Runs an A-only row pass at the state's iterate (lam_t, nu^t): afterwards
// H = -sigma^A / cfac^A and gtab2[t&1] = (g^A, g^A); returns cfac^A.
lamp_status state_normalisers(const lamp_problem* p, const lamp_params* q, const Resolved& R,
                              const lamp_state* s, void* ws, hipStream_t st, double* cA_out) {
    // the workspace is laid out for q->precision; the normalisers always use the FP64-argument sweeps
    Layout L = layout(p->n, p->m, p->d, q->precision, TARGET_BLOCKS, p->metric);
    L.prec = LAMP_FP32;
    const Consts kc = make_consts(p, R);
    Ctrl hc;
    lamp_status e = upload_ctrl(ws, L, s->t, s->t + 1, s->t, 0.0, st, &hc);
    if (e != LAMP_OK) return e;
    Sched sc{};
    sc.lamA = sc.lamB = sc.lamC = s->inv_eta;
    sc.w = sc.w2 = 0.0;   // nubar = nu: both halves evaluate p^{eta_t}(nu^t)
    HIPCHK(hipMemcpyAsync(at<Sched>(ws, L.sched), &sc, sizeof(Sched), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));   // the uploads read host locals of this frame
    hipLaunchKernelGGL(col_table_init, grid1(p->m), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl),
                       at<Sched>(ws, L.sched), kc, at<double>(ws, L.yn2), s->nu, s->theta, at<double2>(ws, L.gtab), (float2*)nullptr, L.m_pad);
    launch_offsets(L, kc, p->d, ws, st);
    launch_row_sweep(L, kc, p->d, ws, st);
    hipLaunchKernelGGL(row_finish, grid1(kc.n), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, p->d, at<double>(ws, L.xc), at<double>(ws, L.yc), at<double2>(ws, L.gtab), p->r,
                       at<double>(ws, L.xn2), at<double2>(ws, L.rpart), row_parts(L), at<double>(ws, L.H),
                       at<RowVar>(ws, L.rowvar), at<double2>(ws, L.rowck), (double*)nullptr, (double*)nullptr,
                       RowVarF32{nullptr, 0});
    HIPCHK(hipGetLastError());
    *cA_out = 2.0 * R.s * s->inv_eta * LOG2E;
    return LAMP_OK;
}

// g^A_j = -lam_t LOG2E (s |y~_j|^2 + K nu_j): the column term of X^t's exponents (base 2).
// mu_i = vals[2 + k][i] / r_i: the row minima of the explicit-cost certificate pass (which
// reports them weighted by r_i > 0), the shifts of the entropic pass.
__global__ void row_minima_of_vals(Consts kc, const double* __restrict__ r, const double* __restrict__ vals,
                                   double* __restrict__ mu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    mu[i] = vals[2 * kc.n + i] / r[i];
    mu[kc.n + i] = vals[3 * kc.n + i] / r[i];
}

__global__ void state_col_term(Consts kc, double lam, const double* __restrict__ yn2,
                               const double* __restrict__ nu, double* __restrict__ gA) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kc.m) gA[j] = -lam * LOG2E * (kc.s * yn2[j] + kc.K * nu[j]);
}

__global__ void gA_extract(int64_t m, int64_t par, const double2* __restrict__ gtab2, double* __restrict__ gA) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) gA[j] = gtab2[par * m + j].x;
}

// r_i log Z_i of X^t from the certificate row pass: with p_ij = 2^(cA (h_i + P_ij) + g^A_j)
// and psum_i = sum_j p_ij,  log Z_i = ln sum_j exp(-lam (C_ij + K nu_j))
//                                  = ln psum_i - ln2 cA h_i - lam s |x~_i|^2.
__global__ void normaliser_terms(Consts kc, double cA, double lam, const double* __restrict__ psum,
                                 const double* __restrict__ H, const double* __restrict__ xn2,
                                 const double* __restrict__ r, double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    out[i] = r[i] * (log(psum[i]) - LN2 * cA * H[i] - lam * kc.s * xn2[i]);
}

__global__ void col_residual(Consts kc, const double2* __restrict__ cpart, int P, const double* __restrict__ c,
                             double* __restrict__ out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kc.m) return;
    double col = 0.0;
    for (int p = 0; p < P; ++p) col += cpart[(int64_t)p * kc.m + j].x;
    out[j] = fabs(col - c[j]);
}


// ------------------------------------------------------------------ batching form
struct BatchCand {
    int64_t target_total;   // sweep blocks per phase over the whole batch
    int grid;               // persistent grid size of the phase kernels
};
constexpr BatchCand kBatchCands[] = {{2048, 1024}, {4096, 1024}, {4096, 2048}, {8192, 2048}, {16384, 2048},
                                 {16384, 4096}};
constexpr int kNumBatchCands = (int)(sizeof(kBatchCands) / sizeof(kBatchCands[0]));

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;   // batch signature -> candidate index

__global__ void set_epoch(const ProbDesc* __restrict__ pd, int count, int64_t t_base, int64_t t_end) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) {
        pd[p].ctrl->t_base = t_base;
        pd[p].ctrl->t_end = t_end;
    }
}

// Rewind every control block to iteration t (used by the autotuner's repeated timing).
__global__ void rewind_ctrl(const ProbDesc* __restrict__ pd, int count, int64_t t, int64_t t_end) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) {
        Ctrl* c = pd[p].ctrl;
        c->t = t;
        c->t_base = t;
        c->t_end = t_end;
        c->done = 0;
        c->err = 0;
    }
}

// The most sweep blocks any candidate spreads over a batch: the capacity of the sweep
// partials and work lists, whatever share of it a problem gets.
constexpr int64_t max_target() {
    int64_t t = 0;
    for (const BatchCand& c : kBatchCands) t = c.target_total > t ? c.target_total : t;
    return t;
}
constexpr int64_t kMaxTarget = max_target();

struct BatchPlan {
    std::vector<Layout> L;                // per-problem buffers and set-up passes
    std::vector<size_t> sub;              // per-problem sub-workspace offsets
    std::vector<size_t> rpartB, cpartB;   // per-problem sweep partials, room for the most splits
    size_t descs, items[4], ctrlv, sched, counters, nact, total;
    int cap_items[4];                     // list capacities; lists 1 and 3 are always full
};

// Relative cost of one pair in the vector-ALU sweeps: d FP64 FMAs for the dot product
// plus about 10 issue slots for the two exponents (assembly, conversion, exp, sum).
double pair_cost(int d) { return (double)(d + 10); }

BatchPlan batch_plan(const lamp_problem* probs, int count) {
    BatchPlan B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int k = 0; k < 4; ++k) B.cap_items[k] = 0;
    B.L.resize(count);
    std::vector<int64_t> pr(count), pc(count);
    for (int p = 0; p < count; ++p) {
        const lamp_problem& q = probs[p];
        B.L[p] = layout(q.n, q.m, q.d, LAMP_FP32);
        pr[p] = cdiv(q.m, choose_split(q.n, q.m, kMaxTarget, false));
        pc[p] = cdiv(q.n, choose_split(q.m, q.n, kMaxTarget, false));
        const int64_t rb = cdiv(q.n, BLOCK), cb = cdiv(q.m, BLOCK);
        B.cap_items[0] += (int)(rb * pr[p]);
        B.cap_items[1] += (int)rb;
        B.cap_items[2] += (int)(cb * pc[p]);
        B.cap_items[3] += (int)cb;
    }
    B.descs = take(sizeof(ProbDesc) * count);
    for (int k = 0; k < 4; ++k) B.items[k] = take(sizeof(Item) * B.cap_items[k]);
    B.counters = take(sizeof(unsigned) * 2);
    B.nact = take(sizeof(int) * 2);
    B.ctrlv = take(sizeof(Ctrl) * count);
    B.sched = take(sizeof(Sched) * (TAB + 2));
    B.rpartB.resize(count);
    B.cpartB.resize(count);
    for (int p = 0; p < count; ++p) {
        B.rpartB[p] = take(sizeof(double2) * probs[p].n * pr[p]);
        B.cpartB[p] = take(sizeof(double2) * probs[p].m * pc[p]);
    }
    B.sub.resize(count);
    for (int p = 0; p < count; ++p) B.sub[p] = take(B.L[p].total);
    B.total = off;
    return B;
}

std::string batch_signature(const lamp_problem* probs, int count) {
    std::string sig = std::to_string(count);
    for (int p = 0; p < count; ++p)
        sig += ":" + std::to_string(probs[p].n) + "x" + std::to_string(probs[p].m) + "x" + std::to_string(probs[p].d);
    return sig;
}

struct BatchRun {
    BatchPlan B;
    std::vector<Item> lists[2];   // row / column sweep items of the running problems, largest first
    std::vector<ProbDesc> desc;
    std::vector<Resolved> R;
    std::vector<double*> nu1, th1;
    int grid;
    int64_t target_total;
    double tau1;
};

void* sub_ws(void* ws, const BatchPlan& B, int p) { return static_cast<char*>(ws) + B.sub[p]; }

// The running problems (active[p] != 0) share the candidate's sweep blocks in proportion to
// their work (n m times the pair cost of the dimension): each gets the splits of its share,
// and the two sweep lists hold all their items, largest first (an item's cost: its rows x
// its columns x the pair cost), so that the persistent sweeps end on small items.
void batch_assign(BatchRun* run, const lamp_problem* probs, const std::vector<char>& active) {
    const int count = (int)run->desc.size();
    double wsum = 0.0;
    for (int p = 0; p < count; ++p)
        if (active[p]) wsum += (double)probs[p].n * (double)probs[p].m * pair_cost(probs[p].d);
    std::vector<double> icost[2];
    for (int h = 0; h < 2; ++h) run->lists[h].clear();
    for (int p = 0; p < count; ++p) {
        if (!active[p]) continue;
        const lamp_problem& q = probs[p];
        const double w = (double)q.n * (double)q.m * pair_cost(q.d);
        const int64_t target = std::max<int64_t>(1, (int64_t)std::llround((double)run->target_total * w / wsum));
        ProbDesc& D = run->desc[p];
        D.split_r = choose_split(q.n, q.m, target, false);
        D.P_r = (int)cdiv(q.m, D.split_r);
        D.split_c = choose_split(q.m, q.n, target, false);
        D.P_c = (int)cdiv(q.n, D.split_c);
        for (int h = 0; h < 2; ++h) {
            const int64_t own = h == 0 ? q.n : q.m, other = h == 0 ? q.m : q.n;
            const int64_t split = h == 0 ? D.split_r : D.split_c;
            const int64_t P = h == 0 ? D.P_r : D.P_c;
            for (int64_t y = 0; y < P; ++y)
                for (int64_t x = 0; x < cdiv(own, BLOCK); ++x) {
                    run->lists[h].push_back(Item{p, (int)x, (int)y, 0});
                    const double rows = (double)std::min<int64_t>(BLOCK, own - x * BLOCK);
                    const double cols = (double)std::min<int64_t>(split, other - y * split);
                    icost[h].push_back(rows * cols * pair_cost(q.d));
                }
        }
    }
    for (int h = 0; h < 2; ++h) {
        std::vector<int> ord(run->lists[h].size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return icost[h][a] > icost[h][b]; });
        std::vector<Item> sorted(ord.size());
        for (size_t i = 0; i < ord.size(); ++i) sorted[i] = run->lists[h][ord[i]];
        run->lists[h].swap(sorted);
    }
}

// Uploads the descriptors (their splits), the two sweep lists and their lengths, which the
// sweep kernels read from device memory (the captured graph's launch arguments stay valid).
// Synchronises the stream: the copies read host vectors of the run.
lamp_status batch_upload(const BatchRun& run, void* ws, hipStream_t st) {
    const BatchPlan& B = run.B;
    HIPCHK(hipMemcpyAsync(at<ProbDesc>(ws, B.descs), run.desc.data(), sizeof(ProbDesc) * run.desc.size(),
                          hipMemcpyHostToDevice, st));
    int nact[2];
    for (int h = 0; h < 2; ++h) {
        nact[h] = (int)run.lists[h].size();
        if (nact[h] > 0)
            HIPCHK(hipMemcpyAsync(at<Item>(ws, B.items[h == 0 ? 0 : 2]), run.lists[h].data(), sizeof(Item) * nact[h],
                                  hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(at<int>(ws, B.nact), nact, sizeof(nact), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return LAMP_OK;
}

// Everything up to the first iteration: per-problem preparation and cost scale, the
// shared schedule, control blocks, column tables, exact offsets, descriptors and work lists.
lamp_status batch_setup(const lamp_problem* probs, int count, const lamp_params* q, const lamp_state* states,
                        void* ws, hipStream_t st, int cand, int64_t t_stop, BatchRun* run) {
    run->B = batch_plan(probs, count);
    const BatchPlan& B = run->B;
    run->grid = kBatchCands[cand].grid;
    run->target_total = kBatchCands[cand].target_total;
    run->desc.resize(count);
    run->R.resize(count);
    run->nu1.resize(count);
    run->th1.resize(count);
    lamp_status e;
    for (int p = 0; p < count; ++p) {
        void* w = sub_ws(ws, B, p);
        if ((e = prep_L(&probs[p], B.L[p], w, st)) != LAMP_OK) return e;
        if ((e = resolve_L(&probs[p], q, B.L[p], w, st, &run->R[p])) != LAMP_OK) return e;
        if (run->R[p].tau1 != run->R[0].tau1)
            return fail(LAMP_EINVAL, "batched problems need a common ||C||_inf (problem %d differs)", p);
    }
    run->tau1 = run->R[0].tau1;
    const int64_t t0 = states[0].t;
    std::vector<Sched> tab(TAB);
    fill_sched(tab.data(), TAB, states[0].inv_eta, run->tau1, q->eta);
    HIPCHK(hipMemcpyAsync(at<Sched>(ws, B.sched), tab.data(), sizeof(Sched) * TAB, hipMemcpyHostToDevice, st));
    std::vector<Ctrl> hc(count);
    std::vector<Item> fin[2];   // row finish / dual update items: one per block of rows / columns
    for (int p = 0; p < count; ++p) {
        const Layout& L = B.L[p];
        void* w = sub_ws(ws, B, p);
        Ctrl& c = hc[p];
        c = Ctrl{};
        c.t = t0;
        c.t_end = std::min(t_stop, t0 + TAB);
        c.t_base = t0;
        c.t_done = -1;
        c.tol = q->tol;
        c.res_last = -1.0;
        const Consts kc = make_consts(&probs[p], run->R[p]);
        ProbDesc& D = run->desc[p];
        D.ctrl = at<Ctrl>(ws, B.ctrlv) + p;
        D.kc = kc;
        D.d = probs[p].d;
        D.n_dual_blocks = (int)cdiv(probs[p].m, BLOCK);
        D.xc = at<double>(w, L.xc);
        D.yc = at<double>(w, L.yc);
        D.xn2 = at<double>(w, L.xn2);
        D.yn2 = at<double>(w, L.yn2);
        D.r = probs[p].r;
        D.c = probs[p].c;
        D.gtab = at<double2>(w, L.gtab);
        D.H = at<double>(w, L.H);
        D.rowvar = at<RowVar>(w, L.rowvar);
        D.rowck = at<double2>(w, L.rowck);
        D.rpart = at<double2>(ws, B.rpartB[p]);
        D.cpart = at<double2>(ws, B.cpartB[p]);
        run->nu1[p] = at<double>(w, L.nu1);
        run->th1[p] = at<double>(w, L.th1);
        D.buf.nu[t0 & 1] = states[p].nu;
        D.buf.theta[t0 & 1] = states[p].theta;
        D.buf.nu[(t0 + 1) & 1] = run->nu1[p];
        D.buf.theta[(t0 + 1) & 1] = run->th1[p];
        D.respart = at<double>(w, L.respart);
        for (int64_t x = 0; x < cdiv(probs[p].n, BLOCK); ++x) fin[0].push_back(Item{p, (int)x, 0, 0});
        for (int64_t x = 0; x < cdiv(probs[p].m, BLOCK); ++x) fin[1].push_back(Item{p, (int)x, 0, 0});
    }
    batch_assign(run, probs, std::vector<char>(count, 1));
    const unsigned zeros[2] = {0u, 0u};
    HIPCHK(hipMemcpyAsync(at<unsigned>(ws, B.counters), zeros, sizeof(zeros), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<Ctrl>(ws, B.ctrlv), hc.data(), sizeof(Ctrl) * count, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<Item>(ws, B.items[1]), fin[0].data(), sizeof(Item) * fin[0].size(), hipMemcpyHostToDevice,
                          st));
    HIPCHK(hipMemcpyAsync(at<Item>(ws, B.items[3]), fin[1].data(), sizeof(Item) * fin[1].size(), hipMemcpyHostToDevice,
                          st));
    if ((e = batch_upload(*run, ws, st)) != LAMP_OK) return e;   // synchronises: the vectors above are read
    for (int p = 0; p < count; ++p) {
        const Layout& L = B.L[p];
        void* w = sub_ws(ws, B, p);
        const ProbDesc& D = run->desc[p];
        // the per-problem set-up kernels read the batch control block and schedule
        hipLaunchKernelGGL(col_table_init, grid1(D.kc.m), dim3(BLOCK), 0, st, D.ctrl, at<Sched>(ws, B.sched), D.kc,
                           D.yn2, states[p].nu, states[p].theta, D.gtab, (float2*)nullptr, (int64_t)0);
        launch_offsets(L, D.kc, probs[p].d, w, st, D.ctrl, at<Sched>(ws, B.sched));
    }
    HIPCHK(hipGetLastError());
    return LAMP_OK;
}

// One iteration of every running problem: the row sweep, the row finish, the column sweep,
// the dual update and its finish, one launch each.
void batch_iteration(const BatchRun& run, void* ws, hipStream_t st) {
    const BatchPlan& B = run.B;
    const int count = (int)run.desc.size();
    const ProbDesc* pd = at<ProbDesc>(ws, B.descs);
    const Sched* sch = at<Sched>(ws, B.sched);
    unsigned* ctr = at<unsigned>(ws, B.counters);
    const int* na = at<int>(ws, B.nact);
    const dim3 gr((unsigned)std::max(1, std::min(run.grid, B.cap_items[0])));
    const dim3 gc((unsigned)std::max(1, std::min(run.grid, B.cap_items[2])));
    hipLaunchKernelGGL(batch_row_sweep, gr, dim3(BLOCK), 0, st, pd, at<Item>(ws, B.items[0]), na, sch, ctr);
    hipLaunchKernelGGL(batch_row_finish, dim3((unsigned)B.cap_items[1]), dim3(BLOCK), 0, st, pd,
                       at<Item>(ws, B.items[1]), B.cap_items[1], sch, ctr);
    hipLaunchKernelGGL(batch_col_sweep, gc, dim3(BLOCK), 0, st, pd, at<Item>(ws, B.items[2]), na + 1, sch, ctr + 1);
    hipLaunchKernelGGL(batch_dual_update, dim3((unsigned)B.cap_items[3]), dim3(BLOCK), 0, st, pd,
                       at<Item>(ws, B.items[3]), B.cap_items[3], sch, ctr + 1);
    hipLaunchKernelGGL(batch_dual_finish, dim3((unsigned)count), dim3(BLOCK), 0, st, pd, sch);
}

// Autotuner: every candidate launch shape runs a few iterations from the callers' start
// state (writes go to workspace buffers only) and the fastest is cached per batch shape.
lamp_status batch_tune(const lamp_problem* probs, int count, const lamp_params* q, const lamp_state* states,
                       void* ws, hipStream_t st, int* best) {
    const std::string sig = batch_signature(probs, count);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return LAMP_OK;
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int best_c = 0;
    for (int c = 0; c < kNumBatchCands; ++c) {
        BatchRun run;
        lamp_status e = batch_setup(probs, count, q, states, ws, st, c, states[0].t + 1, &run);
        if (e != LAMP_OK) return e;
        // the control blocks stop every problem after one iteration: time 3 repetitions of it
        batch_iteration(run, ws, st);   // warm-up (the real iteration)
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) {
            // rerun the same iteration: reset t on the device to the start iteration
            hipLaunchKernelGGL(rewind_ctrl, dim3(cdiv(count, 64)), dim3(64), 0, st, at<ProbDesc>(ws, run.B.descs),
                               count, states[0].t, states[0].t + 1);
            batch_iteration(run, ws, st);
        }
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[sig] = best_c;
    *best = best_c;
    return LAMP_OK;
}
// One iteration on workspace `ws` (lamp_step and lamp_step_noalloc); `prob` is canonical.
lamp_status step_impl(const lamp_problem* prob, const lamp_params* params, lamp_state* state, void* ws,
                      size_t ws_bytes, hipStream_t st, const lamp_trace* trace, double* res_out) {
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    const int64_t t = state->t;
    Sched tab[1];
    fill_sched(tab, 1, state->inv_eta, R.tau1, params->eta);
    HIPCHK(hipMemcpyAsync(at<Sched>(ws, L.sched), tab, sizeof(Sched), hipMemcpyHostToDevice, st));
    Ctrl hc;
    if ((e = upload_ctrl(ws, L, t, t + 1, t, 0.0, st, &hc, state->dt_partial)) != LAMP_OK) return e;
    IterArgs ia{};
    ia.track_dt = params->track_dt != 0;
    ia.buf.nu[t & 1] = state->nu;
    ia.buf.theta[t & 1] = state->theta;
    ia.buf.nu[(t + 1) & 1] = at<double>(ws, L.nu1);
    ia.buf.theta[(t + 1) & 1] = at<double>(ws, L.th1);
    if (trace) {
        ia.tc = TraceCols{trace->col_a, trace->col_b, trace->theta_bar, trace->theta_hat};
        ia.log_za = trace->log_za;
        ia.log_zb = trace->log_zb;
    }
    hipLaunchKernelGGL(col_table_init, grid1(kc.m), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.yn2), state->nu, state->theta, at<double2>(ws, L.gtab), gtabf_ptr(L, ws), L.m_pad);
    launch_offsets(L, kc, prob->d, ws, st);
    launch_iteration(prob, L, kc, ws, ia, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(state->nu, at<double>(ws, L.nu1), sizeof(double) * kc.m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(state->theta, at<double>(ws, L.th1), sizeof(double) * kc.m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(&hc, at<Ctrl>(ws, L.ctrl), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc.err) return fail(LAMP_ENUMERIC, "non-finite value in the dual update at t = %lld", (long long)t);
    if (res_out) *res_out = hc.res_last;
    state->t = t + 1;
    state->inv_eta = tab[0].lamB;
    state->dt_partial = ia.track_dt ? hc.dt_acc : std::numeric_limits<double>::quiet_NaN();
    return LAMP_OK;
}


// Fixed workspace of lamp_step_noalloc: one copy per device, held until the process ends.
// Host code never uses the array's name as an address: scratch_address() returns the
// device address of the current device's copy (hipGetSymbolAddress, once per device).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

lamp_status scratch_address(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LAMP_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LAMP_EDEVICE, "no device address for the scratch array on device %d", dev);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LAMP_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* lamp_last_error(void) { return g_err; }

size_t lamp_workspace_bytes(const lamp_problem* prob, const lamp_params* params) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    if (!prob || prob->n < 1 || prob->m < 1 || prob->d < 1) return 0;
    const int prec = params ? params->precision : LAMP_FP32;
    if (is_mfma(prec) && mfma_kp(prec, prob->d) == 0) return 0;
    return layout(prob->n, prob->m, prob->d, prec, TARGET_BLOCKS, prob->metric).total;
}

lamp_status lamp_cost_scale(const lamp_problem* prob, void* ws, size_t ws_bytes, void* stream,
                            double* s_out, double* max_sqdist_out) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_problem(prob)) != LAMP_OK) return e;
    if ((e = check_ws(prob, ws, ws_bytes)) != LAMP_OK) return e;
    if ((e = prep(prob, ws, st)) != LAMP_OK) return e;
    double md = 0.0;
    if ((e = max_sqdist(prob, ws, st, &md, LAMP_FP32)) != LAMP_OK) return e;
    if (!(md > 0.0)) return fail(LAMP_EDOMAIN, "all pairwise distances are zero");
    if (s_out) *s_out = 1.0 / md;
    if (max_sqdist_out) *max_sqdist_out = md;
    return LAMP_OK;
}

lamp_status lamp_step(const lamp_problem* prob, const lamp_params* params, lamp_state* state, void* ws,
                      size_t ws_bytes, void* stream, const lamp_trace* trace, double* res_out) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    return step_impl(prob, params, state, ws, ws_bytes, (hipStream_t)stream, trace, res_out);
}

lamp_status lamp_step_noalloc(const lamp_problem* prob, const lamp_params* params, lamp_state* state,
                              void* stream, const lamp_trace* trace, double* res_out) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    lamp_status e;
    if ((e = check_problem(prob)) != LAMP_OK) return e;
    if ((e = check_params(params)) != LAMP_OK) return e;
    const size_t need = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric).total;
    if (need > LAMP_NOALLOC_WS_BYTES)
        return fail(LAMP_ENOMEM, "lamp_step_noalloc: this problem needs %zu bytes of workspace, the fixed device "
                    "scratch holds %zu (use lamp_step with a caller workspace)", need, (size_t)LAMP_NOALLOC_WS_BYTES);
    void* ws = nullptr;
    if ((e = scratch_address(&ws)) != LAMP_OK) return e;
    return step_impl(prob, params, state, ws, LAMP_NOALLOC_WS_BYTES, (hipStream_t)stream, trace, res_out);
}

lamp_status lamp_solve(const lamp_problem* prob, const lamp_params* params, lamp_state* state, void* ws,
                       size_t ws_bytes, void* stream, lamp_report* out) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    const auto t_start = std::chrono::steady_clock::now();
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    // graph capture needs a non-default stream: use a private one when given NULL
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!st) {
        HIPCHK(hipStreamSynchronize(nullptr));
        HIPCHK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
        }
    } guard{own};
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    const int64_t t0 = state->t;
    const int64_t t_stop = t0 + params->max_iter;
    const int K = params->check_every > 0 ? params->check_every : 64;

    IterArgs ia{};
    ia.track_dt = params->track_dt != 0;
    ia.buf.nu[t0 & 1] = state->nu;
    ia.buf.theta[t0 & 1] = state->theta;
    ia.buf.nu[(t0 + 1) & 1] = at<double>(ws, L.nu1);
    ia.buf.theta[(t0 + 1) & 1] = at<double>(ws, L.th1);

    std::vector<Sched> tab(TAB);
    double lam_epoch = state->inv_eta;   // lam at t_base of the current epoch
    int64_t t_base = t0;
    double lam_next_epoch = fill_sched(tab.data(), TAB, lam_epoch, R.tau1, params->eta);
    HIPCHK(hipMemcpyAsync(at<Sched>(ws, L.sched), tab.data(), sizeof(Sched) * TAB, hipMemcpyHostToDevice, st));
    Ctrl hc;
    int64_t t_end = std::min(t_stop, t_base + TAB);
    if ((e = upload_ctrl(ws, L, t0, t_end, t_base, params->tol, st, &hc, state->dt_partial)) != LAMP_OK) return e;

    hipLaunchKernelGGL(col_table_init, grid1(kc.m), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.yn2), state->nu, state->theta, at<double2>(ws, L.gtab), gtabf_ptr(L, ws), L.m_pad);
    launch_offsets(L, kc, prob->d, ws, st);
    HIPCHK(hipGetLastError());

    // capture K iterations once; the kernels read t, the schedule and the stop flag
    // from device memory, so the same graph is replayed for every chunk
    GraphGuard gg;
    if (t_stop > t0) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) launch_iteration(prob, L, kc, ws, ia, st);
        hipError_t ce = hipStreamEndCapture(st, &gg.graph);
        if (ce != hipSuccess) return fail(LAMP_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce));
        HIPCHK(hipGraphInstantiate(&gg.exec, gg.graph, nullptr, nullptr, 0));
    }
    int64_t t_cur = t0;
    lamp_status result = LAMP_OK;
    while (t_cur < t_stop) {
        // two chunks in flight: the kernels of a chunk that starts after the stop exit at once
        HIPCHK(hipGraphLaunch(gg.exec, st));
        HIPCHK(hipGraphLaunch(gg.exec, st));
        HIPCHK(hipMemcpyAsync(&hc, at<Ctrl>(ws, L.ctrl), sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hc.err) {
            result = fail(LAMP_ENUMERIC, "non-finite value in the dual update at t = %lld", (long long)hc.t_done);
            t_cur = hc.t_done;
            break;
        }
        if (hc.done) {
            t_cur = hc.t_done;
            break;
        }
        if (hc.t == t_cur && hc.t < hc.t_end) {
            result = fail(LAMP_EDEVICE, "iteration counter did not advance past t = %lld", (long long)t_cur);
            break;
        }
        t_cur = hc.t;
        if (t_cur >= t_stop) break;
        if (t_cur >= hc.t_end) {
            // new schedule epoch
            t_base = t_cur;
            lam_epoch = lam_next_epoch;
            lam_next_epoch = fill_sched(tab.data(), TAB, lam_epoch, R.tau1, params->eta);
            HIPCHK(hipMemcpyAsync(at<Sched>(ws, L.sched), tab.data(), sizeof(Sched) * TAB, hipMemcpyHostToDevice, st));
            hc.t_end = std::min(t_stop, t_base + TAB);
            hc.t_base = t_base;
            HIPCHK(hipMemcpyAsync(at<Ctrl>(ws, L.ctrl), &hc, sizeof(Ctrl), hipMemcpyHostToDevice, st));
        }
    }
    // the iterate of t_cur lives in buffer t_cur & 1
    if (t_cur != t0 && (t_cur & 1) != (t0 & 1)) {
        HIPCHK(hipMemcpyAsync(state->nu, at<double>(ws, L.nu1), sizeof(double) * kc.m, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(state->theta, at<double>(ws, L.th1), sizeof(double) * kc.m, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    // lam at t_cur (continue the recursion from the epoch base)
    double lam = lam_epoch;
    for (int64_t k = t_base; k < t_cur; ++k) lam = next_lam(lam, R.tau1, params->eta);
    state->t = t_cur;
    state->inv_eta = lam;
    if (t_cur != t0) state->dt_partial = ia.track_dt ? hc.dt_acc : std::numeric_limits<double>::quiet_NaN();
    if (out) {
        out->iters = t_cur - t0;
        out->t = t_cur;
        out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        out->final_res = hc.res_last;
        out->cost_scale = R.s;
        out->cost_norm = R.cnorm;
        out->converged = hc.done && !hc.err;
        out->row_fallbacks = hc.fallbacks;
    }
    if (result != LAMP_OK) return result;
    return (hc.done || params->tol == 0.0) ? LAMP_OK : LAMP_NOT_CONVERGED;
}

lamp_status lamp_certificate(const lamp_problem* prob, const lamp_params* params, const lamp_state* state,
                             void* ws, size_t ws_bytes, void* stream, lamp_cert* out) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    if (state->t < 1 || !(state->inv_eta > 0.0)) return fail(LAMP_EINVAL, "the certificate needs t >= 1");
    if (!out) return fail(LAMP_EINVAL, "out is NULL");
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    double cA = 0.0;
    if ((e = state_normalisers(prob, params, R, state, ws, st, &cA)) != LAMP_OK) return e;
    // column marginal col(X^t): the column sweep evaluates both (identical) halves
    Layout LV = L;
    LV.prec = LAMP_FP32;
    launch_col_sweep(LV, kc, prob->d, ws, st);
    double* sc = at<double>(ws, L.scratch);
    const int64_t nm = std::max(kc.n, kc.m);
    double* gA = sc;                 // m
    double* colres = sc + nm;        // m
    double* prods = sc + 2 * nm;     // 2m
    double* part = at<double>(ws, L.rpart);  // per-split partials of the row passes: P_r x n x 4
    double* small = at<double>(ws, L.small);
    double* psum = sc + 4 * nm;      // n
    double* xr = sc + 5 * nm;        // n
    double* colp = sc + 6 * nm;      // m
    double* yf = sc + 7 * nm;        // m
    double* dc = sc + 8 * nm;        // m
    double* dr = sc + 9 * nm;        // n
    double* cpp = sc + 10 * nm;      // n
    double* tr1 = sc + 11 * nm;      // n
    double* absdr = sc + 12 * nm;    // n
    double* vals = sc + 13 * nm;     // 4n
    double* mu = sc + 17 * nm;       // 2n: the row minima of C_ij + K theta_j, C_ij + K nu_j
    double* S = sc + 19 * nm;        // d + 2
    const dim3 split_grid(sweep_grid(kc.n, L.P_r));
    hipLaunchKernelGGL(col_residual, grid1(kc.m), dim3(BLOCK), 0, st, kc, at<double2>(ws, L.cpart), col_parts(LV),
                       prob->c, colres);
    hipLaunchKernelGGL(gA_extract, grid1(kc.m), dim3(BLOCK), 0, st, kc.m, (int64_t)(state->t & 1),
                       at<double2>(ws, L.gtab), gA);
    // pair passes: the kernel of the problem's metric and dimension, coordinates of the
    // thread's own point in registers where compiled (run-time form otherwise)
    auto by_md = [&](auto&& launch) {
        const bool done = by_metric(kc.metric, [&](auto m) {
            return cert_dispatch<decltype(m)::value>(prob->d, [&](auto dd) { launch(m, dd); });
        });
        if (!done) launch(IC<-1>{}, IC<0>{});
    };
    // explicit cost: the row-wise passes in the row sweep's layout (coalesced reads of C)
    const dim3 cost_rows_grid((unsigned)cdiv(kc.n, 4 * COST_ROWS));
    if (L.cost) {
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((cert_rows_cost<T>), cost_rows_grid, dim3(BLOCK), 0, st, kc, cA, gA, at<double>(ws, L.H),
                           prob->r, state->nu, state->theta, vals, psum);
        });
    } else {
        by_md([&](auto m, auto dd) {
            hipLaunchKernelGGL((cert_rows<decltype(m)::value, decltype(dd)::value>), split_grid, dim3(BLOCK), 0,
                               st, kc, prob->d, cA, at<double>(ws, L.xc), at<double>(ws, L.yc),
                               at<double>(ws, L.xn2), at<double>(ws, L.yn2), gA, at<double>(ws, L.H), state->nu,
                               state->theta, part, L.split_r);
        });
        hipLaunchKernelGGL(cert_rows_merge, grid1(kc.n), dim3(BLOCK), 0, st, kc, (int)L.P_r, prob->r,
                           (const double*)part, vals, psum, mu);
    }
    hipLaunchKernelGGL(col_products, grid1(kc.m), dim3(BLOCK), 0, st, kc, prob->c, state->theta, state->nu, prods);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, vals, kc.n, kc.n, 4, small);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, colres, kc.m, kc.m, 1, small + 4);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, prods, kc.m, kc.m, 2, small + 5);
    // Round (Algorithm 3) of the same X and its cost
    hipLaunchKernelGGL(round_row_factors, grid1(kc.n), dim3(BLOCK), 0, st, kc, psum, xr);
    // Round step 2 over row splits; the split partials reuse the (consumed) column partials
    double* rpart = at<double>(ws, L.cpart);
    if (L.cost) {
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((round_cols_cost<T>), dim3((unsigned)cdiv(kc.m, COST_COL_BLOCK), (unsigned)L.P_cx), dim3(BLOCK),
                           0, st, kc, cA, gA, at<double>(ws, L.H), prob->r, xr, rpart, L.split_cx);
        });
    } else {
        by_md([&](auto m, auto dd) {
            hipLaunchKernelGGL((round_cols<decltype(m)::value, decltype(dd)::value>),
                               dim3(sweep_grid(kc.m, L.P_c)), dim3(BLOCK), 0, st, kc, prob->d, cA,
                               at<double>(ws, L.xc), at<double>(ws, L.yc), gA, at<double>(ws, L.H), prob->r, xr,
                               rpart, L.split_c);
        });
    }
    hipLaunchKernelGGL(round_cols_merge, grid1(kc.m), dim3(BLOCK), 0, st, kc, (const double*)rpart,
                       (int)(L.cost ? L.P_cx : L.P_c), colp);
    hipLaunchKernelGGL(round_col_factors, grid1(kc.m), dim3(BLOCK), 0, st, kc, prob->c, colp, yf, dc);
    if (L.cost) {
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((round_rows_cost<T>), cost_rows_grid, dim3(BLOCK), 0, st, kc, cA, gA, at<double>(ws, L.H),
                           prob->r, xr, yf, dr, cpp);
        });
    } else {
        by_md([&](auto m, auto dd) {
            hipLaunchKernelGGL((round_rows<decltype(m)::value, decltype(dd)::value>), split_grid, dim3(BLOCK), 0,
                               st, kc, prob->d, cA, at<double>(ws, L.xc), at<double>(ws, L.yc),
                               at<double>(ws, L.xn2), at<double>(ws, L.yn2), gA, at<double>(ws, L.H), yf, part,
                               L.split_r);
        });
        hipLaunchKernelGGL(round_rows_merge, grid1(kc.n), dim3(BLOCK), 0, st, kc, (int)L.P_r, prob->r, xr,
                           (const double*)part, dr, cpp);
    }
    if (L.cost) {
        by_cost_type(kc.cost_type, [&](auto tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((round_rank_one_cost<T>), cost_rows_grid, dim3(BLOCK), 0, st, kc, dr, dc, tr1, absdr);
        });
    } else if (kc.metric == METRIC_SQEUCLID) {
        hipLaunchKernelGGL(round_col_sums, dim3(prob->d + 2), dim3(BLOCK), 0, st, kc, prob->d,
                           at<double>(ws, L.yc), at<double>(ws, L.yn2), dc, S);
        hipLaunchKernelGGL(round_rank_one, grid1(kc.n), dim3(BLOCK), 0, st, kc, prob->d, at<double>(ws, L.xc),
                           at<double>(ws, L.xn2), dr, S, tr1, absdr);
    } else {
        hipLaunchKernelGGL(round_rank_one_pairs, grid1(kc.n), dim3(BLOCK), 0, st, kc, prob->d,
                           at<double>(ws, L.xc), at<double>(ws, L.yc), dr, dc, tr1, absdr);
    }
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, cpp, kc.n, kc.n, 1, small + 7);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, tr1, kc.n, kc.n, 1, small + 8);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, absdr, kc.n, kc.n, 1, small + 9);
    // <r, log Z^t> for D_t (the telescoped normaliser term of Lemma kl_diff)
    double* rlz = at<double>(ws, L.dtrow);   // n
    hipLaunchKernelGGL(normaliser_terms, grid1(kc.n), dim3(BLOCK), 0, st, kc, cA, state->inv_eta, psum,
                       at<double>(ws, L.H), at<double>(ws, L.xn2), prob->r, rlz);
    hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, rlz, kc.n, kc.n, 1, small + 10);
    // D^eta(theta), D^eta(nu) at the problem's eta (def:dual_spp_e); NaN at eta = 0
    const bool soft = params->eta > 0.0;
    if (soft) {
        double* sv = vals;   // 2n (the row values above are reduced)
        // the minima: from the certificate row pass (recovered from r_i min for the explicit cost)
        if (L.cost) hipLaunchKernelGGL(row_minima_of_vals, grid1(kc.n), dim3(BLOCK), 0, st, kc, prob->r, vals, mu);
        by_md([&](auto m, auto dd) {
            hipLaunchKernelGGL((cert_soft_rows<decltype(m)::value, decltype(dd)::value>), split_grid, dim3(BLOCK),
                               0, st, kc, prob->d, 1.0 / params->eta, at<double>(ws, L.xc), at<double>(ws, L.yc),
                               at<double>(ws, L.xn2), at<double>(ws, L.yn2), state->nu, state->theta,
                               (const double*)mu, part, L.split_r);
        });
        hipLaunchKernelGGL(cert_soft_merge, grid1(kc.n), dim3(BLOCK), 0, st, kc, (int)L.P_r, 1.0 / params->eta,
                           prob->r, (const double*)mu, (const double*)part, sv);
        hipLaunchKernelGGL(reduce_sums, dim3(1), dim3(1024), 0, st, sv, kc.n, kc.n, 2, small + 11);
    }
    HIPCHK(hipGetLastError());
    double h[13];
    HIPCHK(hipMemcpyAsync(h, small, sizeof(double) * (soft ? 13 : 11), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out->row_res = h[0];
    out->cost = h[1];
    out->dual_theta = h[2] - R.K * h[5];
    out->dual_nu = h[3] - R.K * h[6];
    out->col_res = h[4];
    out->primal_penalized = out->cost + R.K * (out->row_res + out->col_res);
    out->gap = out->primal_penalized - std::max(out->dual_theta, out->dual_nu);
    out->prop_bound = 4.0 * R.cnorm * out->col_res + 2.0 * R.cnorm * std::log((double)kc.m) / (double)state->t;
    // <C, Round(X)>; the rank-one correction is skipped when ||dr||_1 = 0 (then dc = 0 too)
    out->rounded_cost = h[7] + (h[9] > 0.0 ? h[8] / h[9] : 0.0);
    // D_t = (summands accumulated by the iterations) + <r, log Z^t> - <r, log Z^0>, log Z^0 = log m
    const double logm = std::log((double)kc.m);
    out->dt = state->dt_partial + h[10] - logm;
    out->midpoint_bound =
        2.0 * R.cnorm * (logm + (1.0 + R.alpha) * std::log(2.0) + out->dt) / (double)state->t;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    out->dual_eta_theta = soft ? h[11] - R.K * h[5] : nan;
    out->dual_eta_nu = soft ? h[12] - R.K * h[6] : nan;
    out->cost_scale = R.s;
    out->cost_norm = R.cnorm;
    out->t = state->t;
    return LAMP_OK;
}

lamp_status lamp_backward(const lamp_problem* prob, const lamp_params* params, const lamp_state* state,
                          double grad_out, float* grad_x, void* ws, size_t ws_bytes, void* stream) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    if (state->t < 1 || !(state->inv_eta > 0.0)) return fail(LAMP_EINVAL, "the gradient needs t >= 1");
    if (!grad_x) return fail(LAMP_EINVAL, "grad_x is NULL");
    if (prob && prob->metric == LAMP_EXPLICIT)
        return fail(LAMP_EINVAL, "the gradient with respect to the points needs point clouds");
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    // one pass: the sweep keeps its own per-row offsets and divides by the row sums at the end
    const double cA = 2.0 * R.s * state->inv_eta * LOG2E;
    double* gA = at<double>(ws, L.scratch);
    hipLaunchKernelGGL(state_col_term, grid1(kc.m), dim3(BLOCK), 0, st, kc, state->inv_eta, at<double>(ws, L.yn2),
                       state->nu, gA);
    launch_adjoint(L, kc, prob->d, ws, cA, gA, st);
    hipLaunchKernelGGL(adjoint_finish, grid1(kc.n), dim3(BLOCK), 0, st, kc, prob->d, (int)L.P_r,
                       grad_out * 2.0 * R.s, at<double>(ws, L.xc), prob->r, at<double>(ws, L.rpart), grad_x);
    HIPCHK(hipGetLastError());
    return LAMP_OK;
}

lamp_status lamp_transport_cost(const lamp_problem* prob, const lamp_params* params, const lamp_state* state,
                                void* ws, size_t ws_bytes, void* stream, double* cost) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    if (state->t < 1 || !(state->inv_eta > 0.0)) return fail(LAMP_EINVAL, "the transport cost needs t >= 1");
    if (!cost) return fail(LAMP_EINVAL, "cost is NULL");
    if (prob && prob->metric == LAMP_EXPLICIT)
        return fail(LAMP_EINVAL, "an explicit cost matrix takes lamp_certificate for <C, X^t>");
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    // the same weights as the adjoint: the sweep keeps its own per-row offsets
    const double cA = 2.0 * R.s * state->inv_eta * LOG2E;
    double* gA = at<double>(ws, L.scratch);
    hipLaunchKernelGGL(state_col_term, grid1(kc.m), dim3(BLOCK), 0, st, kc, state->inv_eta, at<double>(ws, L.yn2),
                       state->nu, gA);
    launch_cost(L, kc, prob->d, ws, cA, gA, prob->r, at<double>(ws, L.dtrow), cost, st);
    HIPCHK(hipGetLastError());
    return LAMP_OK;
}

lamp_status lamp_backward_y(const lamp_problem* prob, const lamp_params* params, const lamp_state* state,
                            double grad_out, float* grad_y, void* ws, size_t ws_bytes, void* stream) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    if (state->t < 1 || !(state->inv_eta > 0.0)) return fail(LAMP_EINVAL, "the gradient needs t >= 1");
    if (!grad_y) return fail(LAMP_EINVAL, "grad_y is NULL");
    if (prob && prob->metric == LAMP_EXPLICIT)
        return fail(LAMP_EINVAL, "the gradient with respect to the points needs point clouds");
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    const int d = prob->d;
    // row offsets k_i and weights w_i = r_i of X^t: one pass of row sums under per-lane integer
    // offsets (templated dimensions), else the normaliser set-up of the certificate
    const double cA = 2.0 * R.s * state->inv_eta * LOG2E;
    double* gA = at<double>(ws, L.scratch);
    hipLaunchKernelGGL(state_col_term, grid1(kc.m), dim3(BLOCK), 0, st, kc, state->inv_eta, at<double>(ws, L.yn2),
                       state->nu, gA);
    const bool one_pass = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            constexpr int D = decltype(dd)::value;
            // the column records follow gA in the scratch region (sized for them in layout())
            auto* cols = reinterpret_cast<CostCol<D>*>(at<char>(ws, L.scratch) + align256(sizeof(double) * kc.m));
            hipLaunchKernelGGL((cost_pack<D>), grid1(kc.m), dim3(BLOCK), 0, st, kc.m, at<double>(ws, L.yc),
                               at<double>(ws, L.yn2), (const double*)gA, cols);
            hipLaunchKernelGGL((norm_sweep<decltype(m)::value, D>), dim3(sweep_grid(kc.n, L.P_r)), dim3(BLOCK), 0,
                               st, kc, cA, at<double>(ws, L.xc), (const CostCol<D>*)cols, at<double>(ws, L.rpart),
                               L.split_r);
            hipLaunchKernelGGL(norm_finish, grid1(kc.n), dim3(BLOCK), 0, st, kc, (int)L.P_r, cA, prob->r,
                               (const double*)at<double>(ws, L.rpart), at<RowVar>(ws, L.rowvar));
        });
    });
    if (!one_pass) {
        double cA2 = 0.0;
        if ((e = state_normalisers(prob, params, R, state, ws, st, &cA2)) != LAMP_OK) return e;
        hipLaunchKernelGGL(gA_extract, grid1(kc.m), dim3(BLOCK), 0, st, kc.m, (int64_t)(state->t & 1),
                           at<double2>(ws, L.gtab), gA);
    }
    const dim3 g(sweep_grid(kc.m, L.P_c));
    double* part = at<double>(ws, L.cpart);
    const double* xc = at<double>(ws, L.xc);
    const float* xcf = at<float>(ws, L.xcf);
    const double* yc = at<double>(ws, L.yc);
    const RowVar* rv = at<RowVar>(ws, L.rowvar);
    const bool done = by_metric(kc.metric, [&](auto m) {
        return valu_dispatch<decltype(m)::value>(d, [&](auto dd) {
            constexpr int D = decltype(dd)::value;
            // the row records follow gA in the scratch region, over the norm pass's column records
            auto* rows = reinterpret_cast<AdjRow<D>*>(at<char>(ws, L.scratch) + align256(sizeof(double) * kc.m));
            hipLaunchKernelGGL((adjoint_y_pack<D>), grid1(kc.n), dim3(BLOCK), 0, st, kc.n, cA, xc, xcf, rv, rows);
            hipLaunchKernelGGL((adjoint_y_sweep<decltype(m)::value, D>), g, dim3(BLOCK), 0, st, kc, cA,
                               (const AdjRow<D>*)rows, yc, (const double*)gA, part, L.split_c);
        });
    });
    if (!done)
        hipLaunchKernelGGL(adjoint_y_sweep_dyn, g, dim3(BLOCK), 0, st, kc, d, cA, xc, xcf, yc, gA, rv, part,
                           L.split_c);
    hipLaunchKernelGGL(adjoint_y_finish, grid1(kc.m), dim3(BLOCK), 0, st, kc, d, (int)L.P_c, grad_out * 2.0 * R.s,
                       yc, part, grad_y);
    HIPCHK(hipGetLastError());
    return LAMP_OK;
}

lamp_status lamp_sweep_times(const lamp_problem* prob, const lamp_params* params, const lamp_state* state,
                             void* ws, size_t ws_bytes, void* stream, int32_t reps, double* row_ms,
                             double* col_ms) {
    lamp_problem canon_buf;
    prob = canonical(prob, &canon_buf);
    hipStream_t st = (hipStream_t)stream;
    lamp_status e;
    if ((e = check_state(state)) != LAMP_OK) return e;
    if (reps < 1) return fail(LAMP_EINVAL, "reps must be >= 1");
    Resolved R;
    if ((e = common_setup(prob, params, ws, ws_bytes, st, &R)) != LAMP_OK) return e;
    const Layout L = layout(prob->n, prob->m, prob->d, params->precision, TARGET_BLOCKS, prob->metric);
    const Consts kc = make_consts(prob, R);
    Sched tab[1];
    fill_sched(tab, 1, state->inv_eta, R.tau1, params->eta);
    HIPCHK(hipMemcpyAsync(at<Sched>(ws, L.sched), tab, sizeof(Sched), hipMemcpyHostToDevice, st));
    Ctrl hc;
    if ((e = upload_ctrl(ws, L, state->t, state->t + 1, state->t, 0.0, st, &hc)) != LAMP_OK) return e;
    hipLaunchKernelGGL(col_table_init, grid1(kc.m), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched),
                       kc, at<double>(ws, L.yn2), state->nu, state->theta, at<double2>(ws, L.gtab), gtabf_ptr(L, ws), L.m_pad);
    launch_offsets(L, kc, prob->d, ws, st);
    launch_row_sweep(L, kc, prob->d, ws, st);
    hipLaunchKernelGGL(row_finish, grid1(kc.n), dim3(BLOCK), 0, st, at<Ctrl>(ws, L.ctrl), at<Sched>(ws, L.sched), kc,
                       prob->d, at<double>(ws, L.xc), at<double>(ws, L.yc), at<double2>(ws, L.gtab), prob->r,
                       at<double>(ws, L.xn2), at<double2>(ws, L.rpart), row_parts(L), at<double>(ws, L.H),
                       at<RowVar>(ws, L.rowvar), at<double2>(ws, L.rowck), (double*)nullptr, (double*)nullptr,
                       is_mfma(L.prec) ? rowvar_f32(L, ws) : RowVarF32{nullptr, 0});
    HIPCHK(hipGetLastError());
    hipEvent_t ev[4];
    for (auto& x : ev) HIPCHK(hipEventCreate(&x));
    HIPCHK(hipEventRecord(ev[0], st));
    for (int k = 0; k < reps; ++k) launch_row_sweep(L, kc, prob->d, ws, st);
    HIPCHK(hipEventRecord(ev[1], st));
    HIPCHK(hipEventRecord(ev[2], st));
    for (int k = 0; k < reps; ++k) launch_col_sweep(L, kc, prob->d, ws, st);
    HIPCHK(hipEventRecord(ev[3], st));
    HIPCHK(hipEventSynchronize(ev[3]));
    float a = 0.f, b = 0.f;
    HIPCHK(hipEventElapsedTime(&a, ev[0], ev[1]));
    HIPCHK(hipEventElapsedTime(&b, ev[2], ev[3]));
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (row_ms) *row_ms = a / reps;
    if (col_ms) *col_ms = b / reps;
    return LAMP_OK;
}

lamp_status lamp_exp_rate(void* stream, int32_t blocks, int32_t iters, int32_t reps, double* exp_per_s) {
    if (blocks < 1 || iters < 1 || reps < 1 || !exp_per_s)
        return fail(LAMP_EINVAL, "blocks, iters and reps must be >= 1 and exp_per_s non-NULL");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } eg{e0, e1};
    hipLaunchKernelGGL(exp_rate_probe, dim3((unsigned)blocks), dim3(256), 0, st, iters, 0.5f, (float*)nullptr);
    HIPCHK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(exp_rate_probe, dim3((unsigned)blocks), dim3(256), 0, st, iters, 0.5f, (float*)nullptr);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    const double exps = (double)reps * blocks * 256.0 * (double)iters * EXP_PROBE_CHAINS;
    *exp_per_s = exps / (ms * 1e-3);
    return LAMP_OK;
}

size_t lamp_batch_workspace_bytes(const lamp_problem* probs, int32_t count, const lamp_params* params) {
    (void)params;
    if (!probs || count < 1) return 0;
    for (int p = 0; p < count; ++p)
        if (probs[p].n < 1 || probs[p].m < 1 || probs[p].d < 1) return 0;
    return batch_plan(probs, count).total + 256;
}

lamp_status lamp_solve_batched(const lamp_problem* probs, int32_t count, const lamp_params* params,
                               lamp_state* states, void* ws, size_t ws_bytes, void* stream, lamp_report* outs) {
    const auto t_start = std::chrono::steady_clock::now();
    lamp_status e;
    if (!probs || !states || count < 1) return fail(LAMP_EINVAL, "empty batch or NULL arrays");
    if ((e = check_params(params)) != LAMP_OK) return e;
    if (params->precision != LAMP_FP32) return fail(LAMP_EINVAL, "the batching form runs the LAMP_FP32 form");
    if (params->track_dt) return fail(LAMP_EINVAL, "D_t tracking is not available in the batching form");
    for (int p = 0; p < count; ++p) {
        if ((e = check_problem(&probs[p])) != LAMP_OK) return e;
        if (probs[p].metric != LAMP_SQEUCLID)
            return fail(LAMP_EINVAL, "the batching form runs the squared Euclidean cost (problem %d)", p);
        if ((e = check_state(&states[p])) != LAMP_OK) return e;
        if (states[p].t != states[0].t || states[p].inv_eta != states[0].inv_eta)
            return fail(LAMP_EINVAL, "batched states must share t and inv_eta (problem %d differs)", p);
    }
    if (!ws) return fail(LAMP_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(LAMP_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = lamp_batch_workspace_bytes(probs, count, params) - 256;
    if (ws_bytes < need) return fail(LAMP_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!st) {
        HIPCHK(hipStreamSynchronize(nullptr));
        HIPCHK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
        }
    } guard{own};
    // the first problem's sub-workspace is laid out at offset 0 of a batch plan's problem region;
    // its small-scalar area is scratch here (every problem's preparation rewrites it later)
    {
        const BatchPlan B0 = batch_plan(probs, count);
        double* dev6 = at<double>(static_cast<char*>(ws) + B0.sub[0], B0.L[0].small);
        for (int p = 0; p < count; ++p)
            if ((e = check_marginals(&probs[p], dev6, st)) != LAMP_OK) return e;
    }

    int cand = 0;
    if ((e = batch_tune(probs, count, params, states, ws, st, &cand)) != LAMP_OK) return e;
    const int64_t t0 = states[0].t;
    const int64_t t_stop = t0 + params->max_iter;
    BatchRun run;
    if ((e = batch_setup(probs, count, params, states, ws, st, cand, t_stop, &run)) != LAMP_OK) return e;
    const BatchPlan& B = run.B;
    const int K = params->check_every > 0 ? params->check_every : 64;
    GraphGuard gg;
    if (t_stop > t0) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) batch_iteration(run, ws, st);
        hipError_t ce = hipStreamEndCapture(st, &gg.graph);
        if (ce != hipSuccess) return fail(LAMP_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce));
        HIPCHK(hipGraphInstantiate(&gg.exec, gg.graph, nullptr, nullptr, 0));
    }
    std::vector<Ctrl> hc(count);
    std::vector<char> active(count, 1);
    Ctrl* hc_dev = at<Ctrl>(ws, B.ctrlv);
    double lam_epoch = states[0].inv_eta;
    int64_t t_base = t0;
    std::vector<Sched> tab(TAB);
    double lam_next_epoch = fill_sched(tab.data(), TAB, lam_epoch, run.tau1, params->eta);
    int64_t t_cur = t0;
    lamp_status result = LAMP_OK;
    while (t_cur < t_stop) {
        HIPCHK(hipGraphLaunch(gg.exec, st));
        HIPCHK(hipGraphLaunch(gg.exec, st));
        HIPCHK(hipMemcpyAsync(hc.data(), hc_dev, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool all_done = true, any_err = false, newly_done = false;
        int64_t tmax = t_cur;
        for (int p = 0; p < count; ++p) {
            if (hc[p].err) any_err = true;
            if (!hc[p].done) {
                all_done = false;
                tmax = std::max(tmax, hc[p].t);
            } else if (active[p]) {
                active[p] = 0;
                newly_done = true;
            }
        }
        if (any_err) {
            result = fail(LAMP_ENUMERIC, "non-finite value in the dual update of a batched problem");
            break;
        }
        if (all_done) break;
        if (tmax == t_cur) {
            result = fail(LAMP_EDEVICE, "batched iteration counter did not advance past %lld", (long long)t_cur);
            break;
        }
        t_cur = tmax;
        if (t_cur >= t_stop) break;
        // problems that stopped leave the sweep work lists and the running ones take over their
        // share of the sweep blocks (no graph change: the kernels read the splits and the item
        // counts from device memory)
        if (newly_done) {
            batch_assign(&run, probs, active);
            if ((e = batch_upload(run, ws, st)) != LAMP_OK) {
                result = e;
                break;
            }
        }
        if (t_cur >= t_base + TAB) {
            t_base = t_cur;
            lam_epoch = lam_next_epoch;
            lam_next_epoch = fill_sched(tab.data(), TAB, lam_epoch, run.tau1, params->eta);
            HIPCHK(hipMemcpyAsync(at<Sched>(ws, B.sched), tab.data(), sizeof(Sched) * TAB, hipMemcpyHostToDevice,
                                  st));
            hipLaunchKernelGGL(set_epoch, dim3(cdiv(count, 64)), dim3(64), 0, st, at<ProbDesc>(ws, B.descs), count,
                               t_base, std::min(t_stop, t_base + TAB));
            HIPCHK(hipStreamSynchronize(st));
        }
    }
    HIPCHK(hipMemcpyAsync(hc.data(), hc_dev, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    bool all_conv = true;
    const double lam0 = states[0].inv_eta;   // every state starts at (t0, lam0); states[0] is rewritten below
    for (int p = 0; p < count; ++p) {
        const int64_t tp = hc[p].done ? hc[p].t_done : hc[p].t;
        if ((tp & 1) != (t0 & 1)) {
            HIPCHK(hipMemcpyAsync(states[p].nu, run.nu1[p], sizeof(double) * probs[p].m, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(states[p].theta, run.th1[p], sizeof(double) * probs[p].m, hipMemcpyDeviceToDevice,
                                  st));
        }
        double lam = lam0;
        for (int64_t k = t0; k < tp; ++k) lam = next_lam(lam, run.tau1, params->eta);
        states[p].t = tp;
        states[p].inv_eta = lam;
        if (tp != t0) states[p].dt_partial = std::numeric_limits<double>::quiet_NaN();
        const bool conv = hc[p].done && !hc[p].err;
        all_conv = all_conv && conv;
        if (outs) {
            outs[p].iters = tp - t0;
            outs[p].t = tp;
            outs[p].seconds = secs;
            outs[p].final_res = hc[p].res_last;
            outs[p].cost_scale = run.R[p].s;
            outs[p].cost_norm = run.R[p].cnorm;
            outs[p].converged = conv;
            outs[p].row_fallbacks = hc[p].fallbacks;
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (result != LAMP_OK) return result;
    return (all_conv || params->tol == 0.0) ? LAMP_OK : LAMP_NOT_CONVERGED;
}

}  // extern "C"
