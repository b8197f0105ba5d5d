// Matrix-core (MFMA) forms of the two marginal sweeps: the dot products
// x~_i . y~_j of a 32 x 32 tile come from v_mfma_f32_32x32x{2f32,16bf16,16f16}
// with FP32 accumulation; the exponent is assembled in FP32 from the tile:
//     e = c * (h_i + x~_i . y~_j) + g_j,
// with h_i entering the MFMA as its accumulator input, so each coupling entry
// costs one FP32 FMA, one v_exp_f32 and one FP32 add (or FMA with the row
// weight).  Operands are FP32, BF16 or FP16 copies of the centred points,
// zero-padded to KP coordinates and to a multiple of 128 points.
//
// Lane layout of the 32x32 MFMA (verified on gfx950): lane l supplies row
// (l mod 32) of A and column (l mod 32) of B; D[row][col] sits in lane
// col + 32 h, register 4a + b, with row = 8a + 4h + b (h = l / 32).  The
// contraction index may be permuted consistently between A and B, so lane half
// h supplies coordinates [h KP/2, (h+1) KP/2) of its point as contiguous vectors.
#pragma once

#include "lamp_kernels.hpp"

namespace lampk {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<float> {
    static constexpr int KSTEP = 2;   // contraction length of one instruction
    using vec = float;                // per-lane operand of one instruction
    __device__ static floatx16 mma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
};

template <>
struct MfmaOp<__bf16> {
    static constexpr int KSTEP = 16;
    using vec = bf16x8;
    __device__ static floatx16 mma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct MfmaOp<_Float16> {
    static constexpr int KSTEP = 16;
    using vec = halfx8;
    __device__ static floatx16 mma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

constexpr float PAD_NEG = -1e30f;   // exponent of padded entries: 2^PAD_NEG = 0

__device__ __forceinline__ int mfma_row(int r, int hf) { return 8 * (r >> 2) + 4 * hf + (r & 3); }

// Operand copies: out[i][k] = T(x~[i][k]) for k < d, 0 for k >= d or i >= cnt.
template <typename T>
__global__ void prep_operands(const double* __restrict__ src, int64_t cnt, int d, int KP, int64_t cnt_pad,
                              T* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cnt_pad * KP) return;
    int64_t i = idx / KP;
    int k = (int)(idx % KP);
    double v = (i < cnt && k < d) ? src[i * d + k] : 0.0;
    out[idx] = (T)v;
}

__global__ void pad_rows(int64_t n, int64_t n_pad, float* __restrict__ kf, float* __restrict__ wa,
                         float* __restrict__ wb) {
    int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    kf[i] = PAD_NEG;
    wa[i] = 0.f;
    wb[i] = 0.f;
}

// Row sweep: wave w of block b owns rows [32 rw, 32 rw + 32), rw = (b / P) * 4 + w,
// and streams column tiles of split p = b mod P (P a multiple of 8 maps each split to
// one XCD, whose L2 then holds that split's operand rows).
template <typename T, int KP>
__global__ __launch_bounds__(BLOCK) void row_sweep_mfma(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                        const T* __restrict__ xop, const T* __restrict__ yop,
                                                        const float2* __restrict__ gtabf, int64_t m_pad,
                                                        const double* __restrict__ H,
                                                        double2* __restrict__ part, int64_t tiles_per_split,
                                                        int P, int64_t m_tiles, int64_t n_waves) {
    if (halted(ctrl)) return;
    using Op = MfmaOp<T>;
    using vec = typename Op::vec;
    constexpr int NS = KP / Op::KSTEP;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const float cA = (float)(2.0 * kc.s * sc.lamA * LOG2E);
    const float cB = (float)(2.0 * kc.s * sc.lamB * LOG2E);
    const float2* __restrict__ g = gtabf + (t & 1) * m_pad;
    const int lane = threadIdx.x & 63;
    const int hf = lane >> 5, c32 = lane & 31;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t rw = (b / P) * 4 + (threadIdx.x >> 6);
    if (rw >= n_waves) return;
    const int64_t i0 = rw * 32;

    vec a[NS];
    {
        const vec* ap = reinterpret_cast<const vec*>(xop + (i0 + c32) * KP + hf * (KP / 2));
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s] = ap[s];
    }
    floatx16 hv;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int64_t ii = i0 + mfma_row(r, hf);
        hv[r] = (float)H[ii < kc.n ? ii : kc.n - 1];
    }
    float accA[16], accB[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accA[r] = accB[r] = 0.f;

    const int64_t jt0 = (int64_t)p * tiles_per_split;
    const int64_t jt1 = min(m_tiles, jt0 + tiles_per_split);
    // software pipeline: operands of tile jt+1 load while tile jt computes
    vec bn[NS];
    float2 gn = make_float2(PAD_NEG, PAD_NEG);
    if (jt0 < jt1) {
        const int64_t j = jt0 * 32 + c32;
        const vec* bp = reinterpret_cast<const vec*>(yop + j * KP + hf * (KP / 2));
#pragma unroll
        for (int s = 0; s < NS; ++s) bn[s] = bp[s];
        gn = g[j];
    }
    for (int64_t jt = jt0; jt < jt1; ++jt) {
        vec bv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) bv[s] = bn[s];
        const float gA = gn.x, gB = gn.y;
        if (jt + 1 < jt1) {
            const int64_t j = (jt + 1) * 32 + c32;
            const vec* bp = reinterpret_cast<const vec*>(yop + j * KP + hf * (KP / 2));
#pragma unroll
            for (int s = 0; s < NS; ++s) bn[s] = bp[s];
            gn = g[j];
        }
        floatx16 d = Op::mma(a[0], bv[0], hv);
#pragma unroll
        for (int s = 1; s < NS; ++s) d = Op::mma(a[s], bv[s], d);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            accA[r] += __builtin_amdgcn_exp2f(fmaf(d[r], cA, gA));
            accB[r] += __builtin_amdgcn_exp2f(fmaf(d[r], cB, gB));
        }
    }
    // sum over the 32 columns held by the 32 lanes of each half
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
            accA[r] += __shfl_xor(accA[r], o, 64);
            accB[r] += __shfl_xor(accB[r], o, 64);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t row = i0 + mfma_row(r, hf);
        if (c32 == r && row < kc.n) part[(int64_t)p * kc.n + row] = make_double2(accA[r], accB[r]);
    }
}

// Operands and row data of one 32-row tile of the column sweep.
template <typename T, int KP>
struct ColTile {
    typename MfmaOp<T>::vec a[KP / MfmaOp<T>::KSTEP];
    floatx16 kv;
    float wa[16], wb[16];
};

template <typename T, int KP>
__device__ __forceinline__ void load_col_tile(ColTile<T, KP>& ct, const T* __restrict__ xop,
                                              const float* __restrict__ kf, const float* __restrict__ wAf,
                                              const float* __restrict__ wBf, int64_t it, int hf, int c32) {
    using vec = typename MfmaOp<T>::vec;
    constexpr int NS = KP / MfmaOp<T>::KSTEP;
    const vec* ap = reinterpret_cast<const vec*>(xop + (it * 32 + c32) * KP + hf * (KP / 2));
#pragma unroll
    for (int s = 0; s < NS; ++s) ct.a[s] = ap[s];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t rbase = it * 32 + 8 * q + 4 * hf;   // rows of registers 4q .. 4q+3
        const float4 k4 = *reinterpret_cast<const float4*>(kf + rbase);
        const float4 a4 = *reinterpret_cast<const float4*>(wAf + rbase);
        const float4 b4 = *reinterpret_cast<const float4*>(wBf + rbase);
        ct.kv[4 * q + 0] = k4.x; ct.kv[4 * q + 1] = k4.y; ct.kv[4 * q + 2] = k4.z; ct.kv[4 * q + 3] = k4.w;
        ct.wa[4 * q + 0] = a4.x; ct.wa[4 * q + 1] = a4.y; ct.wa[4 * q + 2] = a4.z; ct.wa[4 * q + 3] = a4.w;
        ct.wb[4 * q + 0] = b4.x; ct.wb[4 * q + 1] = b4.y; ct.wb[4 * q + 2] = b4.z; ct.wb[4 * q + 3] = b4.w;
    }
}

// Column sweep: wave owns columns [32 cw, 32 cw + 32), streams row tiles of split p.
// The per-row offsets k_i enter as the MFMA accumulator input; the row weights
// w^A_i, w^B_i multiply the exponentials.
template <typename T, int KP>
__global__ __launch_bounds__(BLOCK) void col_sweep_mfma(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                        const T* __restrict__ xop, const T* __restrict__ yop,
                                                        const float2* __restrict__ gtabf, int64_t m_pad,
                                                        const float* __restrict__ kf,
                                                        const float* __restrict__ wAf,
                                                        const float* __restrict__ wBf,
                                                        double2* __restrict__ cpart, int64_t tiles_per_split,
                                                        int P, int64_t n_tiles, int64_t m_waves) {
    if (halted(ctrl)) return;
    using Op = MfmaOp<T>;
    using vec = typename Op::vec;
    constexpr int NS = KP / Op::KSTEP;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const float cA = (float)(2.0 * kc.s * sc.lamA * LOG2E);
    const float cB = (float)(2.0 * kc.s * sc.lamB * LOG2E);
    const int lane = threadIdx.x & 63;
    const int hf = lane >> 5, c32 = lane & 31;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t cw = (b / P) * 4 + (threadIdx.x >> 6);
    if (cw >= m_waves) return;
    const int64_t j = cw * 32 + c32;

    vec bv[NS];
    {
        const vec* bp = reinterpret_cast<const vec*>(yop + j * KP + hf * (KP / 2));
#pragma unroll
        for (int s = 0; s < NS; ++s) bv[s] = bp[s];
    }
    const float2 gg = gtabf[(t & 1) * m_pad + j];
    const float gA = gg.x, gB = gg.y;
    float accA[4] = {0.f, 0.f, 0.f, 0.f}, accB[4] = {0.f, 0.f, 0.f, 0.f};
    const int64_t it0 = (int64_t)p * tiles_per_split;
    const int64_t it1 = min(n_tiles, it0 + tiles_per_split);
    ColTile<T, KP> nx;
    if (it0 < it1) load_col_tile<T, KP>(nx, xop, kf, wAf, wBf, it0, hf, c32);
    for (int64_t it = it0; it < it1; ++it) {
        const ColTile<T, KP> ct = nx;
        if (it + 1 < it1) load_col_tile<T, KP>(nx, xop, kf, wAf, wBf, it + 1, hf, c32);
        floatx16 d = Op::mma(ct.a[0], bv[0], ct.kv);
#pragma unroll
        for (int s = 1; s < NS; ++s) d = Op::mma(ct.a[s], bv[s], d);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            accA[r & 3] = fmaf(ct.wa[r], __builtin_amdgcn_exp2f(fmaf(d[r], cA, gA)), accA[r & 3]);
            accB[r & 3] = fmaf(ct.wb[r], __builtin_amdgcn_exp2f(fmaf(d[r], cB, gB)), accB[r & 3]);
        }
    }
    float sA = (accA[0] + accA[1]) + (accA[2] + accA[3]);
    float sB = (accB[0] + accB[1]) + (accB[2] + accB[3]);
    sA += __shfl_xor(sA, 32, 64);
    sB += __shfl_xor(sB, 32, 64);
    if (hf == 0 && j < kc.m) cpart[(int64_t)p * kc.m + j] = make_double2(sA, sB);
}

// Padded entries of the FP32 column tables (both parities): zero weight in every sum.
__global__ void pad_gtabf(int64_t m, int64_t m_pad, float2* __restrict__ gtabf) {
    int64_t j = m + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_pad) return;
    gtabf[j] = make_float2(PAD_NEG, PAD_NEG);
    gtabf[m_pad + j] = make_float2(PAD_NEG, PAD_NEG);
}

}  // namespace lampk
