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

#include <type_traits>

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
    // one round-to-nearest-even of the FP64 centred coordinate to T (the compiler lowers
    // FP64 -> BF16/FP16 as a single rounding; a cast through FP32 would be folded into it)
    out[idx] = (i < cnt && k < d) ? (T)src[i * d + k] : (T)0.f;
}

// Split FP16 operands: with v the FP64 centred coordinate times the range scale (a power of
// two), hi = fp16(v) and lo = fp16(v - hi), each a single rounding to nearest even.  A point's
// row of KP entries holds [hi, hi, lo] (side 0, the source points) or [hi, lo, hi] (side 1,
// the targets), d entries each, zero padded, so that one FP16 contraction over 3 d entries is
//     x_hi . y_hi + x_hi . y_lo + x_lo . y_hi
// (the dot product of the scaled points but for x_lo . y_lo and the parts below lo).
__global__ void prep_operands_split(const double* __restrict__ src, int64_t cnt, int d, int KP, int64_t cnt_pad,
                                    const double* __restrict__ scale, int side, _Float16* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cnt_pad * KP) return;
    const int64_t i = idx / KP;
    const int k = (int)(idx % KP);
    _Float16 v = (_Float16)0.f;
    if (i < cnt && k < 3 * d) {
        const int part = k / d;   // 0, 1, 2
        const double x = src[i * d + (k - part * d)] * *scale;
        const _Float16 hi = (_Float16)x;
        const bool lo = side == 0 ? part == 2 : part == 1;
        v = lo ? (_Float16)(x - (double)hi) : hi;
    }
    out[idx] = v;
}

// The range scale of the split FP16 operands: *scale = 2^(7 - e) with 2^e <= max |coordinate|
// < 2^(e+1) over both centred clouds, so that every scaled coordinate is below 256 (its hi
// part far from the FP16 limit, its lo part resolved to 2^-24 absolute or better); 1 if all
// coordinates are zero.  Three launches: split_scale_clear zeroes the running maximum,
// split_scale_max (any grid) folds each block's maximum into it with a 64-bit atomic max on
// the bit pattern (non-negative doubles order as their bits do, so the result is the exact
// maximum whatever the order), split_scale_final turns it into the scale.
__global__ void split_scale_clear(unsigned long long* __restrict__ mbits) { *mbits = 0ull; }

__global__ void split_scale_max(const double* __restrict__ xc, int64_t nx, const double* __restrict__ yc,
                                int64_t ny, unsigned long long* __restrict__ mbits) {
    __shared__ double sh[BLOCK / 64];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    double mx = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < nx; k += stride) mx = fmax(mx, fabs(xc[k]));
    for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < ny; k += stride) mx = fmax(mx, fabs(yc[k]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; ++w) mx = fmax(mx, sh[w]);
        if (mx > 0.0) atomicMax(mbits, (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void split_scale_final(const unsigned long long* __restrict__ mbits, double* __restrict__ scale) {
    const double mx = __longlong_as_double((long long)*mbits);
    *scale = mx > 0.0 ? ldexp(1.0, 7 - ilogb(mx)) : 1.0;
}

// Padded entries of the FP32 column tables (both parities): zero weight in every sum.
__global__ void pad_gtabf(int64_t m, int64_t m_pad, float2* __restrict__ gtabf) {
    int64_t j = m + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_pad) return;
    gtabf[j] = make_float2(PAD_NEG, PAD_NEG);
    gtabf[m_pad + j] = make_float2(PAD_NEG, PAD_NEG);
}


// ---------------------------------------------------------------------------
// FP64 matrix-core sweeps (v_mfma_f64_16x16x4f64) for larger d in the reference-
// accuracy form: the dot products and the exponent assembly are FP64, only the
// exponential and the sums are FP32, exactly as in the vector-ALU sweeps.
// Layout (verified on gfx950): lane l supplies row (l mod 16) of A and column
// (l mod 16) of B for contraction slot l / 16; D[row][col] sits in lane
// col + 16 g, register q, with row = 4 q + g (g = l / 16).  Lane group g supplies
// coordinates [g KP/4, (g+1) KP/4) of its point over the KP/4 instructions.
// ---------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ doublex4 mma64(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP64 operand copy padded to KP coordinates (multiple of 4) and to a multiple of 64 points.
__global__ void prep_operands64(const double* __restrict__ src, int64_t cnt, int d, int KP, int64_t cnt_pad,
                                double* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cnt_pad * KP) return;
    int64_t i = idx / KP;
    int k = (int)(idx % KP);
    out[idx] = (i < cnt && k < d) ? src[i * d + k] : 0.0;
}

__global__ void pad_rowq(int64_t n, int64_t n_pad, float4* __restrict__ q) {
    int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pad) q[i] = make_float4(PAD_NEG, 0.f, 0.f, 0.f);
}

// Row extreme sweep on FP64 matrix cores: out_i = min_j (a_j + sgn x~_i . y~_j), exact FP64.
template <int KP>
__global__ __launch_bounds__(BLOCK) void row_extreme_mfma64(Consts kc, const double* __restrict__ xop,
                                                            const double* __restrict__ yop,
                                                            const double* __restrict__ aj, double sgn,
                                                            double* __restrict__ part, int64_t tiles_per_split,
                                                            int P, int64_t m_tiles, int64_t n_waves) {
    constexpr int NS = KP / 4;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, c16 = lane & 15;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t rw = (b / P) * 4 + (threadIdx.x >> 6);
    if (rw >= n_waves) return;
    const int64_t i0 = rw * 16;
    double a[NS];
    {
        const double* ap = xop + (i0 + c16) * KP + grp * NS;
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s] = sgn * ap[s];
    }
    double best[4] = {__builtin_inf(), __builtin_inf(), __builtin_inf(), __builtin_inf()};
    const int64_t jt0 = (int64_t)p * tiles_per_split;
    const int64_t jt1 = min(m_tiles, jt0 + tiles_per_split);
    for (int64_t jt = jt0; jt < jt1; ++jt) {
        const int64_t j = jt * 16 + c16;
        const double* bp = yop + j * KP + grp * NS;
        double bv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) bv[s] = bp[s];
        const double aval = j < kc.m ? aj[j] : __builtin_inf();
        doublex4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s) d = mma64(a[s], bv[s], d);
#pragma unroll
        for (int q = 0; q < 4; ++q) best[q] = fmin(best[q], aval + d[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) best[q] = fmin(best[q], __shfl_xor(best[q], o, 64));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = i0 + 4 * q + grp;
        if (c16 == q && row < kc.n) part[(int64_t)p * kc.n + row] = best[q];
    }
}

// ---------------------------------------------------------------------------
// LDS-shared forms of the matrix-core sweeps.  The four waves of a block own
// 4 x 32 points and stream the same tiles of the other cloud: each tile (32
// points x KP coordinates, plus its per-point scalars) is loaded once per block
// into LDS, double-buffered, instead of once per wave, which cuts the L2 traffic
// of the streamed operand by 4.  LDS rows are padded by 16 bytes so that the 32
// lanes reading 16-byte pieces of 32 different rows hit distinct banks.
//
// Two-stage pipeline per wave: while the exponentials of tile j are evaluated on
// the vector ALU, the matrix core already computes the dot products of tile j+1
// (its result is consumed one iteration later), and the global loads of tile j+2
// are in flight.  At the top of iteration j, LDS buffer (j+1) mod 2 holds tile
// j+1; tile j+2 goes into buffer j mod 2, whose last reader (the matrix-core
// stage of the previous iteration) finished before the previous barrier.  The
// loop body has no branches: past the end of the range the tile index is clamped
// to the last tile, whose repeated load and dot products are discarded.
// ---------------------------------------------------------------------------
template <typename T, int KP>
struct LdsTile {
    static constexpr int ROW_BYTES = KP * (int)sizeof(T);     // one point's operand
    static constexpr int STRIDE = ROW_BYTES + 16;              // padded LDS row
    static constexpr int TILE_BYTES = 32 * ROW_BYTES;          // global bytes per tile
    static constexpr int CHUNKS = TILE_BYTES / 16;             // 16-byte pieces per tile
    static constexpr int PER_THREAD = (CHUNKS + BLOCK - 1) / BLOCK;
    static constexpr int BUF = 32 * STRIDE + 32 * 16;          // operand rows + 32 scalar slots
    static_assert(PER_THREAD <= 4, "tile larger than the prefetch registers");
};

// Registers of one in-flight tile load: up to four 16-byte pieces per thread and one
// per-point scalar slot.  Named members with compile-time access, so that the
// prefetch stays in registers (an indexed array here ends up in scratch memory).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

struct TileRegs {
    i32x4 r0, r1, r2, r3, s;
};

template <int I>
__device__ __forceinline__ i32x4& treg(TileRegs& t) {
    if constexpr (I == 0) return t.r0;
    else if constexpr (I == 1) return t.r1;
    else if constexpr (I == 2) return t.r2;
    else return t.r3;
}

template <int I, int N, typename F>
__device__ __forceinline__ void unroll_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        unroll_for<I + 1, N>(f);
    }
}

// Scheduling fences of the pipelined loops.  loads_done(): every outstanding global
// load has completed (issued once before a loop, so that the loop's own wait counts
// track only its prefetch).  pin(): the value is computed at this point of the program,
// so the exponentials of a tile stay ahead of the LDS store of the prefetched tile,
// which must wait for its global loads.
__device__ __forceinline__ void loads_done() {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt and lgkmcnt at their maxima (no wait)
}

// One tile step of the half-precision sweeps with the matrix chain of the next tile and the
// vector work of the current one interleaved in issue order: the vector work is cut into
// NS + 1 equal shares of ITEMS items (item(q) for each); share s is issued ahead of matrix
// instruction s and runs while instruction s - 1 executes (the first one covers the LDS
// latency of the operands, the last one the final instruction).  A scheduling barrier
// after each share keeps the compiler from regrouping the two phases, which in-order
// issue would then run one after the other.  d enters as the chain's initial value and
// leaves as its result.  Used where the chain is long (NS >= 12): with 4 instructions
// per tile the extra live registers cost more than the overlap gains.
template <int NS, int ITEMS, typename Op, typename Item>
__device__ __forceinline__ void mma_chain_interleaved(const typename Op::vec (&a)[NS],
                                                      const typename Op::vec (&b)[NS], floatx16& d,
                                                      Item&& item) {
    unroll_for<0, NS + 1>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        unroll_for<s * ITEMS / (NS + 1), (s + 1) * ITEMS / (NS + 1)>([&](auto qc) { item(qc); });
        if constexpr (s < NS) d = Op::mma(a[s], b[s], d);
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N>
__device__ __forceinline__ void pin(float (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ void pin(float& a, float& b) {
    asm volatile("" : "+v"(a), "+v"(b));
    asm volatile("" ::: "memory");
}

// Global -> registers part of a tile load of ROWS points of ROW_BYTES bytes each
// (16-byte pieces, PT per thread) and their SB-byte scalars (SB = 8 or 16).  Every
// thread loads the scalar of point row0 + (thread mod ROWS), clamped to the last of
// scal_rows entries: no branch, so no wait on these loads before the LDS store.
// Consumers mask the scalars of points past the end themselves.
template <int ROWS, int ROW_BYTES, int PT, int SB>
__device__ __forceinline__ void fetch_tile(const char* __restrict__ base, const char* __restrict__ scal,
                                           int64_t row0, int64_t scal_rows, TileRegs& R) {
    constexpr int CHUNKS = ROWS * ROW_BYTES / 16;
    unroll_for<0, PT>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int c = threadIdx.x + q * BLOCK;
        constexpr bool full = (q + 1) * BLOCK <= CHUNKS;   // every thread has a piece
        if (full || c < CHUNKS) treg<q>(R) = *reinterpret_cast<const i32x4*>(base + (int64_t)c * 16);
    });
    const int64_t row = min(row0 + (int64_t)(threadIdx.x & (ROWS - 1)), scal_rows - 1);
    const char* sp = scal + row * SB;
    if constexpr (SB == 16) {
        R.s = *reinterpret_cast<const i32x4*>(sp);
    } else {
        const i32x2 v = *reinterpret_cast<const i32x2*>(sp);
        R.s = i32x4{v.x, v.y, 0, 0};
    }
}

// Registers -> LDS part of a tile load (rows padded to STRIDE bytes, scalars after them).
template <int ROWS, int ROW_BYTES, int STRIDE, int PT>
__device__ __forceinline__ void store_tile(char* lds, TileRegs& R) {
    constexpr int CHUNKS = ROWS * ROW_BYTES / 16;
    unroll_for<0, PT>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int c = threadIdx.x + q * BLOCK;
        constexpr bool full = (q + 1) * BLOCK <= CHUNKS;
        if (full || c < CHUNKS) {
            const int row = (c * 16) / ROW_BYTES;
            const int off = (c * 16) % ROW_BYTES;
            *reinterpret_cast<i32x4*>(lds + row * STRIDE + off) = treg<q>(R);
        }
    });
    // every thread writes its scalar; the BLOCK / ROWS threads of one slot write the same value
    *reinterpret_cast<i32x4*>(lds + ROWS * STRIDE + (threadIdx.x & (ROWS - 1)) * 16) = R.s;
}

// Sources of the tile loads of the matrix-core forms as buffer resources: operand rows
// and their per-point scalars (column table or row data, padded to whole tiles).  A load
// is a wave-uniform byte offset of the tile (scalar) plus a fixed lane offset: no
// per-lane address arithmetic in the loop.  Byte offsets are 32-bit (the host limits the
// operand copies to less than 4 GiB); reads past num_bytes return zero.
struct TileSrc {
    __amdgpu_buffer_rsrc_t ops, scal;
};

constexpr int BUFFER_CONFIG = 0x00020000;   // raw buffer, 32-bit data format (gfx9)

__device__ __forceinline__ TileSrc make_tile_src(const void* ops, uint32_t ops_bytes, const void* scal,
                                                 uint32_t scal_bytes) {
    return TileSrc{
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(ops), (short)0, (int)ops_bytes, BUFFER_CONFIG),
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(scal), (short)0, (int)scal_bytes, BUFFER_CONFIG)};
}

// Global -> registers part of the load of tile `tile` (32 points) and its SB-byte scalars.
template <typename T, int KP, int SB>
__device__ __forceinline__ void tile_fetch(const TileSrc& src, int tile, TileRegs& R) {
    using L = LdsTile<T, KP>;
    constexpr int CHUNKS = 32 * L::ROW_BYTES / 16;
    const uint32_t tile_off = (uint32_t)tile * (32u * L::ROW_BYTES);
    unroll_for<0, L::PER_THREAD>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const uint32_t c = threadIdx.x + q * BLOCK;
        constexpr bool full = (q + 1) * BLOCK <= CHUNKS;   // every thread has a piece
        if (full || c < (uint32_t)CHUNKS)
            treg<q>(R) = __builtin_amdgcn_raw_buffer_load_b128(src.ops, c * 16u, tile_off, 0);
    });
    const uint32_t lane_s = (threadIdx.x & 31u) * (uint32_t)SB;
    const uint32_t scal_off = (uint32_t)tile * (32u * SB);
    if constexpr (SB == 16) {
        R.s = __builtin_amdgcn_raw_buffer_load_b128(src.scal, lane_s, scal_off, 0);
    } else {
        const i32x2 v = __builtin_amdgcn_raw_buffer_load_b64(src.scal, lane_s, scal_off, 0);
        R.s = i32x4{v.x, v.y, 0, 0};
    }
}

template <typename T, int KP>
__device__ __forceinline__ void tile_store(char* lds, TileRegs& R) {
    using L = LdsTile<T, KP>;
    store_tile<32, L::ROW_BYTES, L::STRIDE, L::PER_THREAD>(lds, R);
}

// The operand vectors of lane (c32, hf) from an LDS tile.
template <typename T, int KP>
__device__ __forceinline__ void tile_operands(const char* lds, int c32, int hf,
                                              typename MfmaOp<T>::vec (&v)[KP / MfmaOp<T>::KSTEP]) {
    using L = LdsTile<T, KP>;
    using vec = typename MfmaOp<T>::vec;
    const vec* p = reinterpret_cast<const vec*>(lds + c32 * L::STRIDE + hf * (L::ROW_BYTES / 2));
#pragma unroll
    for (int s = 0; s < KP / MfmaOp<T>::KSTEP; ++s) v[s] = p[s];
}

// x~_i . y~_j + C for the 32 x 32 tile held in LDS (B operand) against the wave's rows (A).
template <typename T, int KP>
__device__ __forceinline__ floatx16 tile_dot(const char* lds, int c32, int hf,
                                             const typename MfmaOp<T>::vec (&a)[KP / MfmaOp<T>::KSTEP],
                                             floatx16 c) {
    using Op = MfmaOp<T>;
    constexpr int NS = KP / Op::KSTEP;
    typename Op::vec bv[NS];
    tile_operands<T, KP>(lds, c32, hf, bv);
    floatx16 d = Op::mma(a[0], bv[0], c);
#pragma unroll
    for (int s = 1; s < NS; ++s) d = Op::mma(a[s], bv[s], d);
    return d;
}

// Row sweep: wave w of block b owns rows [32 rw, 32 rw + 32), rw = (b / P) * 4 + w,
// and streams column tiles of split p = b mod P (P a multiple of 8 maps each split to
// one XCD, whose L2 then holds that split's operand rows).
// LDS-shared column tiles (see above).
// Waves per SIMD the register allocation of row_sweep_mfma_lds must allow: three for the
// half-precision forms up to 64 coordinates (their loop fits 168 registers without
// spilling; the compiler's own choice is a few registers above, i.e. two waves).
template <typename T, int KP>
constexpr int row_sweep_min_waves() {
    return (sizeof(T) == 2 && KP <= 64) ? 3 : 1;
}

template <typename T, int KP>
__global__ __launch_bounds__(BLOCK, (row_sweep_min_waves<T, KP>())) void row_sweep_mfma_lds(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                            const T* __restrict__ xop, const T* __restrict__ yop,
                                                            const float2* __restrict__ gtabf, int64_t m_pad,
                                                            const double* __restrict__ H,
                                                            double2* __restrict__ part, int64_t tiles_per_split,
                                                            int P, int64_t m_tiles, int64_t n_waves) {
    using L = LdsTile<T, KP>;
    using Op = MfmaOp<T>;
    using vec = typename Op::vec;
    constexpr int NS = KP / Op::KSTEP;
    constexpr bool INTERLEAVE = sizeof(T) == 2 && NS >= 12;   // measured: +1.5% at NS = 12, -8% at NS = 4
    __shared__ __align__(16) char lds[2][L::BUF];
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    // the products come scaled by 1 / dscale (a power of two): the factors of the products
    // take dscale, the offsets entering the accumulator 1 / dscale (exact scalings)
    const float cA = (float)(2.0 * kc.s * sc.lamA * LOG2E * kc.dscale);
    const float cB = (float)(2.0 * kc.s * sc.lamB * LOG2E * kc.dscale);
    const float2* __restrict__ g = gtabf + (t & 1) * m_pad;
    const int lane = threadIdx.x & 63;
    const int hf = lane >> 5, c32 = lane & 31;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t rw = (b / P) * 4 + (threadIdx.x >> 6);
    const bool active = rw < n_waves;   // whole waves; the block still joins every barrier
    const int64_t i0 = (active ? rw : 0) * 32;

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
        hv[r] = (float)(H[ii < kc.n ? ii : kc.n - 1] / kc.dscale);
    }
    float accA[16], accB[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accA[r] = accB[r] = 0.f;

    const int jt0 = p * (int)tiles_per_split;
    const int jt1 = min((int)m_tiles, jt0 + (int)tiles_per_split);
    const TileSrc src = make_tile_src(yop, (uint32_t)(m_pad * KP * (int64_t)sizeof(T)), g, (uint32_t)(m_pad * 8));
    TileRegs pf;
    if (jt0 < jt1) {
        const int jl = jt1 - 1;
        // prologue: tile jt0 through buffer 0 into the matrix core, tile jt0 + 1 into buffer 1
        tile_fetch<T, KP, 8>(src, jt0, pf);
        tile_store<T, KP>(lds[0], pf);
        __syncthreads();
        floatx16 dc = tile_dot<T, KP>(lds[0], c32, hf, a, hv);
        float2 gc = *reinterpret_cast<const float2*>(lds[0] + 32 * L::STRIDE + c32 * 16);
        tile_fetch<T, KP, 8>(src, min(jt0 + 1, jl), pf);
        tile_store<T, KP>(lds[1], pf);
        __syncthreads();
        loads_done();
#pragma clang loop unroll(disable)
        for (int jt = jt0; jt < jt1; ++jt) {
            const int nxt = (jt + 1 - jt0) & 1;
            tile_fetch<T, KP, 8>(src, min(jt + 2, jl), pf);
            floatx16 dn;
            float2 gn;
            if constexpr (INTERLEAVE) {
                vec bv[NS];
                tile_operands<T, KP>(lds[nxt], c32, hf, bv);
                dn = hv;
                mma_chain_interleaved<NS, 32, Op>(a, bv, dn, [&](auto qc) {
                    constexpr int q = decltype(qc)::value, r = q >> 1;
                    if constexpr (q & 1)
                        accB[r] += __builtin_amdgcn_exp2f(fmaf(dc[r], cB, gc.y));
                    else
                        accA[r] += __builtin_amdgcn_exp2f(fmaf(dc[r], cA, gc.x));
                });
                gn = *reinterpret_cast<const float2*>(lds[nxt] + 32 * L::STRIDE + c32 * 16);
            } else {
                dn = tile_dot<T, KP>(lds[nxt], c32, hf, a, hv);
                gn = *reinterpret_cast<const float2*>(lds[nxt] + 32 * L::STRIDE + c32 * 16);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    accA[r] += __builtin_amdgcn_exp2f(fmaf(dc[r], cA, gc.x));
                    accB[r] += __builtin_amdgcn_exp2f(fmaf(dc[r], cB, gc.y));
                }
            }
            pin(accA);
            pin(accB);
            tile_store<T, KP>(lds[nxt ^ 1], pf);
            __syncthreads();
            dc = dn;
            gc = gn;
        }
    }
    if (!active) return;
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

// Offsets of the matrix-core forms: part[p][i] = -max_j (c^B x~_i . y~_j + g^B_j) / c^B over
// the column tiles of split p, from the same operand copies and the same FP32 arithmetic as
// the row sweep, so that the largest B-half term of the next row sweep is 2^0 up to
// rounding (the merge takes the minimum over splits).
template <typename T, int KP>
__global__ __launch_bounds__(BLOCK) void row_extreme_mfma_lds(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                              const T* __restrict__ xop, const T* __restrict__ yop,
                                                              const float2* __restrict__ gtabf, int64_t m_pad,
                                                              double* __restrict__ part, int64_t tiles_per_split,
                                                              int P, int64_t m_tiles, int64_t n_waves) {
    using L = LdsTile<T, KP>;
    using Op = MfmaOp<T>;
    using vec = typename Op::vec;
    constexpr int NS = KP / Op::KSTEP;
    __shared__ __align__(16) char lds[2][L::BUF];
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const float cB = (float)(2.0 * kc.s * sc.lamB * LOG2E);
    const float cBd = (float)(2.0 * kc.s * sc.lamB * LOG2E * kc.dscale);   // the factor of the scaled products
    const float2* __restrict__ g = gtabf + (t & 1) * m_pad;
    const int lane = threadIdx.x & 63;
    const int hf = lane >> 5, c32 = lane & 31;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t rw = (b / P) * 4 + (threadIdx.x >> 6);
    const bool active = rw < n_waves;
    const int64_t i0 = (active ? rw : 0) * 32;
    vec a[NS];
    {
        const vec* ap = reinterpret_cast<const vec*>(xop + (i0 + c32) * KP + hf * (KP / 2));
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s] = ap[s];
    }
    floatx16 zero;
#pragma unroll
    for (int r = 0; r < 16; ++r) zero[r] = 0.f;
    float mx[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) mx[r] = -__builtin_inff();
    const int jt0 = p * (int)tiles_per_split;
    const int jt1 = min((int)m_tiles, jt0 + (int)tiles_per_split);
    const TileSrc src = make_tile_src(yop, (uint32_t)(m_pad * KP * (int64_t)sizeof(T)), g, (uint32_t)(m_pad * 8));
    TileRegs pf;
    if (jt0 < jt1) {
        tile_fetch<T, KP, 8>(src, jt0, pf);
        tile_store<T, KP>(lds[0], pf);
    }
    __syncthreads();
    for (int jt = jt0; jt < jt1; ++jt) {
        const int cur = (jt - jt0) & 1;
        if (jt + 1 < jt1) tile_fetch<T, KP, 8>(src, jt + 1, pf);
        const floatx16 d = tile_dot<T, KP>(lds[cur], c32, hf, a, zero);
        const float2 gg = *reinterpret_cast<const float2*>(lds[cur] + 32 * L::STRIDE + c32 * 16);
#pragma unroll
        for (int r = 0; r < 16; ++r) mx[r] = fmaxf(mx[r], fmaf(d[r], cBd, gg.y));
        if (jt + 1 < jt1) tile_store<T, KP>(lds[cur ^ 1], pf);
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) mx[r] = fmaxf(mx[r], __shfl_xor(mx[r], o, 64));
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t row = i0 + mfma_row(r, hf);
        if (c32 == r && row < kc.n) part[(int64_t)p * kc.n + row] = -(double)mx[r] / (double)cB;
    }
}

// Column sweep of the matrix-core forms with the roles of the operands swapped, LDS-shared
// row tiles: the wave's 32 columns y_j are the MFMA rows (fixed A operand) and the
// streamed points x_i the MFMA columns, so the per-row data (k_i, w^A_i, w^B_i) is one
// value per lane per tile instead of sixteen.  The column offsets enter as the
// accumulator input G_j = g_j / c (per register), so that
//     e = c (G_j + x~_i . y~_j) + c k_i,
// one FP32 FMA per entry with the per-lane c k_i.  G differs between the couplings:
// with one matrix-core step per tile (d <= 16) each coupling gets its own chain; with
// NS >= 4 steps the second chain costs more than one add per term, and one chain
// (accumulator G^B) serves both:
//     e^A = c^A (d^B + k_i) + CA_j,   d^B = x~_i . y~_j + G^B_j,   CA_j = g^A_j - c^A G^B_j
// (measured: column sweep 1.49 -> 1.30 ms at n = m = 2^16, d = 64; at d = 3 the two
// chains are 7% faster than one).  CA_j does not depend on the streamed row, so the
// column's sum is accumulated without it and multiplied by 2^CA_j once at the end,
// which saves the add per term (kc.factor_cols; 1.23 -> 1.17 ms at d = 64).  The unscaled sums stay in FP32 range:
// by the column tables of iteration t, CA_j = LOG2E K tau1 (lam_t / lam_{t+1})
// (theta_j - nu_j), so |CA_j| <= 2 LOG2E K tau1 (2.9 with the default tau1); the host
// keeps the per-term add when that bound exceeds 64.
template <typename T, int KP>
__global__ __launch_bounds__(BLOCK) void col_sweep_mfma_t_lds(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                              const T* __restrict__ xop, const T* __restrict__ yop,
                                                              const float2* __restrict__ gtabf, int64_t m_pad,
                                                              const float4* __restrict__ rowq,
                                                              double2* __restrict__ cpart, int64_t tiles_per_split,
                                                              int P, int64_t n_tiles, int64_t m_waves) {
    using L = LdsTile<T, KP>;
    using Op = MfmaOp<T>;
    using vec = typename Op::vec;
    constexpr int NS = KP / Op::KSTEP;
    __shared__ __align__(16) char lds[2][L::BUF];
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const float cA = (float)(2.0 * kc.s * sc.lamA * LOG2E);
    const float cB = (float)(2.0 * kc.s * sc.lamB * LOG2E);
    // factors of the products, which come scaled by 1 / dscale (a power of two); the column
    // terms G below are in the same scaled units, the row offsets k_i are not
    const float cAd = (float)(2.0 * kc.s * sc.lamA * LOG2E * kc.dscale);
    const float cBd = (float)(2.0 * kc.s * sc.lamB * LOG2E * kc.dscale);
    const int lane = threadIdx.x & 63;
    const int hf = lane >> 5, c32 = lane & 31;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t cw = (b / P) * 4 + (threadIdx.x >> 6);
    const bool active = cw < m_waves;
    const int64_t j0 = (active ? cw : 0) * 32;
    vec a[NS];
    {
        const vec* ap = reinterpret_cast<const vec*>(yop + (j0 + c32) * KP + hf * (KP / 2));
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s] = ap[s];
    }
    constexpr bool ONE_CHAIN = NS >= 4;
    constexpr bool INTERLEAVE = sizeof(T) == 2 && NS >= 12;   // as in the row sweep
    const float2* __restrict__ g = gtabf + (t & 1) * m_pad;
    floatx16 GA, GB;
    float CA[16];   // g^A_j - c^A G^B_j (one-chain form)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float2 gg = g[j0 + mfma_row(r, hf)];
        GA[r] = cAd > 0.f ? gg.x / cAd : 0.f;
        GB[r] = gg.y / cBd;
        if (gg.x <= PAD_NEG) GA[r] = PAD_NEG;
        if (gg.y <= PAD_NEG) GB[r] = PAD_NEG;
        CA[r] = gg.x <= PAD_NEG ? PAD_NEG : gg.x - cAd * GB[r];
    }
    float accA[16], accB[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accA[r] = accB[r] = 0.f;
    const int it0 = p * (int)tiles_per_split;
    const int it1 = min((int)n_tiles, it0 + (int)tiles_per_split);
    const int64_t n_rows = n_tiles * 32;
    const TileSrc src = make_tile_src(xop, (uint32_t)(n_rows * KP * (int64_t)sizeof(T)), rowq,
                                      (uint32_t)(n_rows * 16));
    TileRegs pf;
    if (it0 < it1) {
        const int il = it1 - 1;
        auto dots = [&](const char* buf, floatx16& dA, floatx16& dB) {
            typename Op::vec bv[NS];
            tile_operands<T, KP>(buf, c32, hf, bv);
            dB = Op::mma(a[0], bv[0], GB);
            if constexpr (!ONE_CHAIN) dA = Op::mma(a[0], bv[0], GA);
#pragma unroll
            for (int s = 1; s < NS; ++s) {
                if constexpr (!ONE_CHAIN) dA = Op::mma(a[s], bv[s], dA);
                dB = Op::mma(a[s], bv[s], dB);
            }
            if constexpr (ONE_CHAIN) dA = dB;
        };
        tile_fetch<T, KP, 16>(src, it0, pf);
        tile_store<T, KP>(lds[0], pf);
        __syncthreads();
        floatx16 dcA, dcB;
        dots(lds[0], dcA, dcB);
        float4 qc = *reinterpret_cast<const float4*>(lds[0] + 32 * L::STRIDE + c32 * 16);
        tile_fetch<T, KP, 16>(src, min(it0 + 1, il), pf);
        tile_store<T, KP>(lds[1], pf);
        __syncthreads();
        loads_done();
        auto stream_tiles = [&](auto factor_tag) {
            constexpr bool FACTOR = decltype(factor_tag)::value;
#pragma clang loop unroll(disable)
            for (int it = it0; it < it1; ++it) {
                const int nxt = (it + 1 - it0) & 1;
                tile_fetch<T, KP, 16>(src, min(it + 2, il), pf);
                floatx16 dnA, dnB;
                float4 qn;
                if constexpr (INTERLEAVE) {
                    const float ckA = cA * qc.x, ckB = cB * qc.x;
                    typename Op::vec bv[NS];
                    tile_operands<T, KP>(lds[nxt], c32, hf, bv);
                    dnB = GB;
                    mma_chain_interleaved<NS, 32, Op>(a, bv, dnB, [&](auto qi) {
                        constexpr int q = decltype(qi)::value, r = q >> 1;
                        if constexpr (q & 1) {
                            accB[r] = fmaf(qc.z, __builtin_amdgcn_exp2f(fmaf(dcB[r], cBd, ckB)), accB[r]);
                        } else {
                            const float eA = FACTOR ? fmaf(dcB[r], cAd, ckA) : fmaf(dcB[r], cAd, ckA) + CA[r];
                            accA[r] = fmaf(qc.y, __builtin_amdgcn_exp2f(eA), accA[r]);
                        }
                    });
                    dnA = dnB;
                    qn = *reinterpret_cast<const float4*>(lds[nxt] + 32 * L::STRIDE + c32 * 16);
                } else {
                    dots(lds[nxt], dnA, dnB);
                    qn = *reinterpret_cast<const float4*>(lds[nxt] + 32 * L::STRIDE + c32 * 16);
                    const float ckA = cA * qc.x, ckB = cB * qc.x;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float eA = !ONE_CHAIN ? fmaf(dcA[r], cAd, ckA)
                                                    : (FACTOR ? fmaf(dcB[r], cAd, ckA) : fmaf(dcB[r], cAd, ckA) + CA[r]);
                        accA[r] = fmaf(qc.y, __builtin_amdgcn_exp2f(eA), accA[r]);
                        accB[r] = fmaf(qc.z, __builtin_amdgcn_exp2f(fmaf(dcB[r], cBd, ckB)), accB[r]);
                    }
                }
                pin(accA);
                pin(accB);
                tile_store<T, KP>(lds[nxt ^ 1], pf);
                __syncthreads();
                dcA = dnA;
                dcB = dnB;
                qc = qn;
            }
        };
        if constexpr (ONE_CHAIN) {
            if (kc.factor_cols) {
                stream_tiles(std::true_type{});
#pragma unroll
                for (int r = 0; r < 16; ++r) accA[r] *= __builtin_amdgcn_exp2f(CA[r]);
            } else {
                stream_tiles(std::false_type{});
            }
        } else {
            stream_tiles(std::false_type{});
        }
    }
    if (!active) return;
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
        const int64_t j = j0 + mfma_row(r, hf);
        if (c32 == r && j < kc.m) cpart[(int64_t)p * kc.m + j] = make_double2(accA[r], accB[r]);
    }
}

// FP64 matrix-core sweeps with LDS-shared tiles of 16 points (see the LDS-shared
// half-precision sweeps above; the 16x16x4 FP64 layout is described with mma64).
// Row sweep: wave owns 16 rows, a block 64 rows (4 waves) of split p = b mod P;
// column sweep: wave owns 16 columns and streams 16-row tiles of split p.
template <int KP>
struct LdsTile64 {
    static constexpr int ROW_BYTES = KP * 8;
    static constexpr int STRIDE = ROW_BYTES + 16;
    static constexpr int TILE_BYTES = 16 * ROW_BYTES;
    static constexpr int CHUNKS = TILE_BYTES / 16;
    static constexpr int PER_THREAD = (CHUNKS + BLOCK - 1) / BLOCK;
    static constexpr int BUF = 16 * STRIDE + 16 * 16;
    static_assert(PER_THREAD <= 4, "tile larger than the prefetch registers");
};

// Global -> registers part of the load of tile `tile` (16 points) and their 16-byte scalars,
// as buffer loads: a wave-uniform tile offset plus a fixed lane offset (the host keeps the
// operand copies below 4 GiB).  Scalars past the end of their table read as zero; the
// consumers mask the points past the end on the last tile of the range.
template <int KP>
__device__ __forceinline__ void tile64_fetch(const TileSrc& src, int tile, TileRegs& R) {
    using L = LdsTile64<KP>;
    const uint32_t tile_off = (uint32_t)tile * (uint32_t)L::TILE_BYTES;
    unroll_for<0, L::PER_THREAD>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const uint32_t c = threadIdx.x + q * BLOCK;
        constexpr bool full = (q + 1) * BLOCK <= L::CHUNKS;   // every thread has a piece
        if (full || c < (uint32_t)L::CHUNKS)
            treg<q>(R) = __builtin_amdgcn_raw_buffer_load_b128(src.ops, c * 16u, tile_off, 0);
    });
    R.s = __builtin_amdgcn_raw_buffer_load_b128(src.scal, (threadIdx.x & 15u) * 16u, (uint32_t)tile * 256u, 0);
}

template <int KP>
__device__ __forceinline__ void tile64_store(char* lds, TileRegs& R) {
    using L = LdsTile64<KP>;
    store_tile<16, L::ROW_BYTES, L::STRIDE, L::PER_THREAD>(lds, R);
}

// x~ . y~ + C for a 16 x 16 tile: A operand in registers, B operand (16 points) from LDS.
template <int KP>
__device__ __forceinline__ doublex4 tile_dot64(const char* lds, int c16, int grp, const double (&a)[KP / 4],
                                               doublex4 c) {
    using L = LdsTile64<KP>;
    constexpr int NS = KP / 4;
    const double* bp = reinterpret_cast<const double*>(lds + c16 * L::STRIDE) + grp * NS;
    double bv[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) bv[s] = bp[s];
    doublex4 d = mma64(a[0], bv[0], c);
#pragma unroll
    for (int s = 1; s < NS; ++s) d = mma64(a[s], bv[s], d);
    return d;
}

// The tile loop of both FP64 sweeps is software-pipelined over two LDS buffers: iteration
// `it` prefetches tile it + 2, computes the products of tile it + 1 from buffer NXT and the
// exponentials of tile it, then stores the prefetch into the other buffer.  Pairs of
// iterations run with NXT fixed at compile time (constant LDS offsets, the pipeline's values
// kept in place instead of copied); only the iterations whose next tile reaches past the end
// of the points (at most the last three of a range) mask the scalars of those points, with
// NXT at run time.
template <typename Step>
__device__ __forceinline__ void pipelined_tiles(int it0, int it1, int it_mask, Step&& step) {
    int it = it0;
#pragma clang loop unroll(disable)
    for (; it + 2 <= it_mask; it += 2) {
        step(it, std::integral_constant<int, 1>{}, std::false_type{});
        step(it + 1, std::integral_constant<int, 0>{}, std::false_type{});
    }
    for (; it < it1; ++it) step(it, (it + 1 - it0) & 1, std::true_type{});
}

// Body of the FP64 matrix-core row sweep; with DT it also sums the B coupling's cost terms
// for D_t tracking, 2^eB C_ij / s with C_ij / s = (|x~_i|^2 + 2 h_i) + |y~_j|^2 - 2 dot from the
// accumulator dot = h_i + x~_i . y~_j (tpart[p][i], under the row offset of the B sums).
template <int KP, bool DT>
__device__ __forceinline__ void row_sweep_mfma64_body(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                      const double* __restrict__ xop,
                                                      const double* __restrict__ yop,
                                                      const double2* __restrict__ gtab2,
                                                      const double* __restrict__ H,
                                                      double2* __restrict__ part, int64_t tiles_per_split,
                                                      int P, int64_t m_tiles, int64_t n_waves,
                                                      const double* __restrict__ xn2, const double* __restrict__ yn2,
                                                      double* __restrict__ tpart) {
    using L = LdsTile64<KP>;
    constexpr int NS = KP / 4;
    __shared__ __align__(16) char lds[2][L::BUF];
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const double2* __restrict__ g = gtab2 + (t & 1) * kc.m;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, c16 = lane & 15;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t rw = (b / P) * 4 + (threadIdx.x >> 6);
    const bool active = rw < n_waves;
    const int64_t i0 = (active ? rw : 0) * 16;
    double a[NS];
    {
        const double* ap = xop + (i0 + c16) * KP + grp * NS;
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s] = ap[s];
    }
    doublex4 hv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t ii = i0 + 4 * q + grp;
        hv[q] = H[ii < kc.n ? ii : kc.n - 1];
    }
    float accA[4] = {0.f, 0.f, 0.f, 0.f}, accB[4] = {0.f, 0.f, 0.f, 0.f};
    double sumA[4] = {0.0, 0.0, 0.0, 0.0}, sumB[4] = {0.0, 0.0, 0.0, 0.0};
    [[maybe_unused]] float accT[4] = {0.f, 0.f, 0.f, 0.f};
    [[maybe_unused]] double sumT[4] = {0.0, 0.0, 0.0, 0.0};
    [[maybe_unused]] doublex4 xa;
    if constexpr (DT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t ii = i0 + 4 * q + grp;
            xa[q] = xn2[ii < kc.n ? ii : kc.n - 1] + 2.0 * hv[q];
        }
    }
    // |y~_j|^2 of this lane's column in tile jt (clamped past m: those columns weigh 0)
    [[maybe_unused]] auto ycol = [&](int jt) {
        const int64_t j = (int64_t)jt * 16 + c16;
        return yn2[j < kc.m ? j : kc.m - 1];
    };
    const int jt0 = (int)((int64_t)p * tiles_per_split);
    const int jt1 = (int)min(m_tiles, (int64_t)jt0 + tiles_per_split);
    const TileSrc src = make_tile_src(yop, (uint32_t)(m_tiles * L::TILE_BYTES), g, (uint32_t)(kc.m * 16));
    TileRegs pf;
    // column j's table entry; columns past m (padding) never contribute
    auto scal = [&](const char* buf, int jt, auto check) {
        double2 gg = *reinterpret_cast<const double2*>(buf + 16 * L::STRIDE + c16 * 16);
        if constexpr (decltype(check)::value)
            if ((int64_t)jt * 16 + c16 >= kc.m) gg = make_double2(-1e300, -1e300);
        return gg;
    };
    if (jt0 < jt1) {
        const int jl = jt1 - 1;
        tile64_fetch<KP>(src, jt0, pf);
        tile64_store<KP>(lds[0], pf);
        __syncthreads();
        doublex4 dc = tile_dot64<KP>(lds[0], c16, grp, a, hv);
        double2 gc = scal(lds[0], jt0, std::true_type{});
        [[maybe_unused]] double yc = 0.0;
        if constexpr (DT) yc = ycol(jt0);
        tile64_fetch<KP>(src, min(jt0 + 1, jl), pf);
        tile64_store<KP>(lds[1], pf);
        __syncthreads();
        loads_done();
        int cnt = 0;
        auto step = [&](int jt, auto nxtc, auto check) {
            const int nxt = nxtc;   // a constant in the paired iterations
            tile64_fetch<KP>(src, min(jt + 2, jl), pf);
            const doublex4 dn = tile_dot64<KP>(lds[nxt], c16, grp, a, hv);
            const double2 gn = scal(lds[nxt], min(jt + 1, jl), check);
            [[maybe_unused]] double yn = 0.0;
            if constexpr (DT) {
                yn = ycol(min(jt + 1, jl));
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    accA[q] += fexp2(fma(dc[q], cA, gc.x));
                    const float pB = fexp2(fma(dc[q], cB, gc.y));
                    accB[q] += pB;
                    accT[q] = fmaf(pB, (float)fma(-2.0, dc[q], xa[q] + yc), accT[q]);
                }
                pin(accT);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    accA[q] += fexp2(fma(dc[q], cA, gc.x));
                    accB[q] += fexp2(fma(dc[q], cB, gc.y));
                }
            }
            pin(accA);
            pin(accB);
            if (++cnt == 8) {   // carry in FP64 every 8 terms
                cnt = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sumA[q] += (double)accA[q];
                    sumB[q] += (double)accB[q];
                    accA[q] = accB[q] = 0.f;
                    if constexpr (DT) {
                        sumT[q] += (double)accT[q];
                        accT[q] = 0.f;
                    }
                }
            }
            tile64_store<KP>(lds[nxt ^ 1], pf);
            __syncthreads();
            dc = dn;
            gc = gn;
            if constexpr (DT) yc = yn;
        };
        // iteration jt reads the scalars of tile jt + 1: whole tiles (16 columns below m) for jt < m / 16 - 1
        pipelined_tiles(jt0, jt1, max(jt0, min(jt1, (int)(kc.m / 16) - 1)), step);
    }
    if (!active) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sumA[q] += (double)accA[q];
        sumB[q] += (double)accB[q];
        if constexpr (DT) sumT[q] += (double)accT[q];
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            sumA[q] += __shfl_xor(sumA[q], o, 64);
            sumB[q] += __shfl_xor(sumB[q], o, 64);
            if constexpr (DT) sumT[q] += __shfl_xor(sumT[q], o, 64);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = i0 + 4 * q + grp;
        if (c16 == q && row < kc.n) {
            part[(int64_t)p * kc.n + row] = make_double2(sumA[q], sumB[q]);
            if constexpr (DT) tpart[(int64_t)p * kc.n + row] = sumT[q];
        }
    }
}

template <int KP>
__global__ __launch_bounds__(BLOCK) void row_sweep_mfma64_lds(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                              const double* __restrict__ xop,
                                                              const double* __restrict__ yop,
                                                              const double2* __restrict__ gtab2,
                                                              const double* __restrict__ H,
                                                              double2* __restrict__ part, int64_t tiles_per_split,
                                                              int P, int64_t m_tiles, int64_t n_waves) {
    row_sweep_mfma64_body<KP, false>(ctrl, sched, kc, xop, yop, gtab2, H, part, tiles_per_split, P, m_tiles, n_waves,
                                     nullptr, nullptr, nullptr);
}

// The FP64 matrix-core row sweep of a D_t-tracked iteration, tpart: [P][n].
template <int KP>
__global__ __launch_bounds__(BLOCK) void row_sweep_mfma64_dt(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                             const double* __restrict__ xop,
                                                             const double* __restrict__ yop,
                                                             const double2* __restrict__ gtab2,
                                                             const double* __restrict__ H,
                                                             double2* __restrict__ part, int64_t tiles_per_split,
                                                             int P, int64_t m_tiles, int64_t n_waves,
                                                             const double* __restrict__ xn2,
                                                             const double* __restrict__ yn2,
                                                             double* __restrict__ tpart) {
    row_sweep_mfma64_body<KP, true>(ctrl, sched, kc, xop, yop, gtab2, H, part, tiles_per_split, P, m_tiles, n_waves,
                                    xn2, yn2, tpart);
}

// Four waves per SIMD for KP <= 64 (128 VGPRs, no spills): 10.59 -> 10.35 ms at
// n = m = 2^16, d = 64 (the row sweep spills at that bound and gains nothing).
template <int KP>
constexpr int col64_min_waves() { return KP <= 64 ? 4 : 2; }

template <int KP>
__global__ __launch_bounds__(BLOCK, (col64_min_waves<KP>())) void col_sweep_mfma64_lds(const Ctrl* ctrl, const Sched* sched, Consts kc,
                                                              const double* __restrict__ xop,
                                                              const double* __restrict__ yop,
                                                              const double2* __restrict__ gtab2,
                                                              const RowVar* __restrict__ rowvar,
                                                              double2* __restrict__ cpart, int64_t tiles_per_split,
                                                              int P, int64_t n_tiles, int64_t m_waves) {
    using L = LdsTile64<KP>;
    constexpr int NS = KP / 4;
    __shared__ __align__(16) char lds[2][L::BUF];
    if (halted(ctrl)) return;
    const int64_t t = ctrl->t;
    const Sched sc = sched[t - ctrl->t_base];
    const double cA = 2.0 * kc.s * sc.lamA * LOG2E;
    const double cB = 2.0 * kc.s * sc.lamB * LOG2E;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, c16 = lane & 15;
    const int64_t b = blockIdx.x;
    const int p = (int)(b % P);
    const int64_t cw = (b / P) * 4 + (threadIdx.x >> 6);
    const bool active = cw < m_waves;
    const int64_t j = (active ? cw : 0) * 16 + c16;
    // B operand: the wave's 16 columns y_j (lane c16 holds column j of D); the streamed
    // row tile is the A operand, read from LDS
    double bv[NS];
    {
        const double* bp = yop + j * KP + grp * NS;
#pragma unroll
        for (int s = 0; s < NS; ++s) bv[s] = bp[s];
    }
    double gA = -1e300, gB = -1e300;
    if (j < kc.m) {
        const double2 gg = gtab2[(t & 1) * kc.m + j];
        gA = gg.x;
        gB = gg.y;
    }
    float accA = 0.f, accB = 0.f;
    double sumA = 0.0, sumB = 0.0;
    const int it0 = (int)((int64_t)p * tiles_per_split);
    const int it1 = (int)min(n_tiles, (int64_t)it0 + tiles_per_split);
    const TileSrc src = make_tile_src(xop, (uint32_t)(n_tiles * L::TILE_BYTES), rowvar, (uint32_t)(kc.n * 16));
    // rows of the tile: offsets k (accumulator input of the dot products) and weights
    struct RowTerms {
        doublex4 k;
        float wa[4], wb[4];
    };
    auto row_terms = [&](const char* buf, int it, auto check) {
        RowTerms rt;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + grp;
            const RowVar rv = *reinterpret_cast<const RowVar*>(buf + 16 * L::STRIDE + r * 16);
            if constexpr (decltype(check)::value) {
                const bool valid = (int64_t)it * 16 + r < kc.n;
                rt.k[q] = valid ? rv.k : -1e300;
                rt.wa[q] = valid ? rv.wA : 0.f;
                rt.wb[q] = valid ? rv.wB : 0.f;
            } else {
                rt.k[q] = rv.k;
                rt.wa[q] = rv.wA;
                rt.wb[q] = rv.wB;
            }
        }
        return rt;
    };
    auto dot = [&](const char* buf, doublex4 k) {
        const double* ap = reinterpret_cast<const double*>(buf + c16 * L::STRIDE) + grp * NS;
        double av[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) av[s] = ap[s];
        doublex4 d = mma64(av[0], bv[0], k);
#pragma unroll
        for (int s = 1; s < NS; ++s) d = mma64(av[s], bv[s], d);
        return d;
    };
    TileRegs pf;
    if (it0 < it1) {
        const int il = it1 - 1;
        tile64_fetch<KP>(src, it0, pf);
        tile64_store<KP>(lds[0], pf);
        __syncthreads();
        RowTerms rc = row_terms(lds[0], it0, std::true_type{});
        doublex4 dc = dot(lds[0], rc.k);
        tile64_fetch<KP>(src, min(it0 + 1, il), pf);
        tile64_store<KP>(lds[1], pf);
        __syncthreads();
        loads_done();
        auto step = [&](int it, auto nxtc, auto check) {
            const int nxt = nxtc;   // a constant in the paired iterations
            tile64_fetch<KP>(src, min(it + 2, il), pf);
            const RowTerms rn = row_terms(lds[nxt], min(it + 1, il), check);
            const doublex4 dn = dot(lds[nxt], rn.k);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                accA = fmaf(rc.wa[q], fexp2(fma(dc[q], cA, gA)), accA);
                accB = fmaf(rc.wb[q], fexp2(fma(dc[q], cB, gB)), accB);
            }
            pin(accA, accB);
            // carry in FP64 after every second tile of the range (nxt = 0 on those)
            if (nxt == 0) {
                sumA += (double)accA;
                sumB += (double)accB;
                accA = accB = 0.f;
            }
            tile64_store<KP>(lds[nxt ^ 1], pf);
            __syncthreads();
            dc = dn;
            rc = rn;
        };
        // iteration it reads the row data of tile it + 1: whole tiles (16 rows below n) for it < n / 16 - 1
        pipelined_tiles(it0, it1, max(it0, min(it1, (int)(kc.n / 16) - 1)), step);
    }
    if (!active) return;
    sumA += (double)accA;
    sumB += (double)accB;
    sumA += __shfl_xor(sumA, 16, 64);
    sumB += __shfl_xor(sumB, 16, 64);
    sumA += __shfl_xor(sumA, 32, 64);
    sumB += __shfl_xor(sumB, 32, 64);
    if (grp == 0 && j < kc.m) cpart[(int64_t)p * kc.m + j] = make_double2(sumA, sumB);
}

}  // namespace lampk
