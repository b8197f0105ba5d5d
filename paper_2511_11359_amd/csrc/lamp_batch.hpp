// Batching form: many independent problems advance together, each phase of the
// iteration launched once for all of them.  Each sweep is a persistent loop of a
// machine-sized grid over one work list of (problem, tile) items of every dimension; an
// item runs the same device body as the single-problem kernels, compiled for its problem's
// dimension, with that problem's descriptor.  Sweep items are handed out by an atomic
// counter, largest first.  Every problem keeps its own control block, so a problem that
// meets its tolerance stops (its items exit at once) while the others continue; the host
// then hands its share of the sweep blocks to the problems still running.
#pragma once

#include "lamp_kernels.hpp"

namespace lampk {

struct ProbDesc {
    Ctrl* ctrl;
    Consts kc;
    int32_t d, P_r, P_c, n_dual_blocks;
    int64_t split_r, split_c;
    const double *xc, *yc, *xn2, *yn2, *r, *c;
    double2* gtab;
    double* H;
    RowVar* rowvar;
    double2* rowck;
    double2* rpart;
    double2* cpart;
    DualBufs buf;
    double* respart;
};

struct Item {
    int32_t prob, bx, by, pad;
};

#define LAMP_BATCH_D(X) X(1) X(2) X(3) X(4) X(8) X(16)

// The descriptor's pointers are loaded from memory, so the compiler cannot tell their
// address space (it would use flat loads) nor that the column data are read-only during
// the sweep.  Re-typing them restores what the single-problem kernels get from their
// arguments: the streamed column data go through the constant address space (scalar
// loads when the address is wave-uniform), per-lane data through the global one.
// (Through an integer: a direct generic -> specific -> generic cast is folded away.)
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ const T* as_const(const T* p) {
    return (const T*)(const __attribute__((address_space(4))) T*)(uintptr_t)p;
}

// Next work item of a persistent sweep kernel: one atomic increment per block on the
// phase's counter (largest items come first in the list, so the tail is short).  The
// counter is returned to zero by the next phase kernel of the iteration.
__device__ __forceinline__ int next_item(unsigned* counter) {
    __shared__ int k_sh;
    if (threadIdx.x == 0) k_sh = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(k_sh);   // block-uniform
    __syncthreads();
    return k;
}

__device__ __forceinline__ void reset_counter(unsigned* counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
}

// Row sweep items of every running problem; each item runs the body compiled for its
// problem's dimension (the run-time form for any other dimension).
__global__ __launch_bounds__(BLOCK) void batch_row_sweep(const ProbDesc* __restrict__ pd,
                                                         const Item* __restrict__ items,
                                                         const int* __restrict__ n_active,
                                                         const Sched* sched, unsigned* counter) {
    const int n_items = *n_active;   // items of problems still running (rewritten by the host)
    if ((int)blockIdx.x >= n_items) return;   // more blocks than items: the surplus leaves at once
    for (;;) {
        const int k = next_item(counter);
        if (k >= n_items) break;
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        const Ctrl* ctrl = as_const(P.ctrl);
        const double* xc = as_global(P.xc);
        const double* yc = as_const(P.yc);
        const double2* gtab = as_const(P.gtab);
        const double* H = as_global(P.H);
        double2* rpart = as_global(P.rpart);
        switch (P.d) {
#define CASE(D)                                                                                                  \
    case D:                                                                                                      \
        row_sweep_body<METRIC_SQEUCLID, D>(ctrl, sched, P.kc, xc, yc, gtab, H, rpart, P.split_r, it.bx, it.by, 0); \
        break;
            LAMP_BATCH_D(CASE)
#undef CASE
            default:
                row_sweep_dyn_body(ctrl, sched, P.kc, P.d, xc, yc, gtab, H, rpart, P.split_r, it.bx, it.by, 0);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void batch_row_finish(const ProbDesc* __restrict__ pd,
                                                          const Item* __restrict__ items, int n_items,
                                                          const Sched* sched, unsigned* counter) {
    reset_counter(counter);   // the row sweep of this iteration is complete
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        row_finish_body(P.ctrl, sched, P.kc, P.d, P.xc, P.yc, P.gtab, P.r, P.xn2, P.rpart, P.P_r, P.H, P.rowvar,
                        P.rowck, nullptr, nullptr, RowVarF32{nullptr, 0}, it.bx, it.by, 0);
    }
}

// Column sweep items of every running problem, as the row sweep.
__global__ __launch_bounds__(BLOCK) void batch_col_sweep(const ProbDesc* __restrict__ pd,
                                                         const Item* __restrict__ items,
                                                         const int* __restrict__ n_active,
                                                         const Sched* sched, unsigned* counter) {
    const int n_items = *n_active;   // items of problems still running (rewritten by the host)
    if ((int)blockIdx.x >= n_items) return;   // more blocks than items: the surplus leaves at once
    for (;;) {
        const int k = next_item(counter);
        if (k >= n_items) break;
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        const Ctrl* ctrl = as_const(P.ctrl);
        const double* xc = as_const(P.xc);
        const double* yc = as_global(P.yc);
        const double2* gtab = as_global(P.gtab);
        const RowVar* rowvar = as_const(P.rowvar);
        const double2* rowck = as_const(P.rowck);
        double2* cpart = as_global(P.cpart);
        switch (P.d) {
#define CASE(D)                                                                                                 \
    case D:                                                                                                     \
        col_sweep_body<METRIC_SQEUCLID, D>(ctrl, sched, P.kc, xc, yc, gtab, rowvar, rowck, cpart, P.split_c, it.bx, \
                                           it.by, 0);                                                           \
        break;
            LAMP_BATCH_D(CASE)
#undef CASE
            default:
                col_sweep_dyn_body(ctrl, sched, P.kc, P.d, xc, yc, gtab, rowvar, rowck, cpart, P.split_c, it.bx, it.by,
                                   0);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void batch_dual_update(const ProbDesc* __restrict__ pd,
                                                           const Item* __restrict__ items, int n_items,
                                                           const Sched* sched, unsigned* counter) {
    reset_counter(counter);   // the column sweep of this iteration is complete
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        dual_update_body(P.ctrl, sched, P.kc, P.cpart, P.P_c, P.c, P.yn2, P.buf, P.gtab, nullptr, 0, P.respart,
                         TraceCols{nullptr, nullptr, nullptr, nullptr}, nullptr, it.bx);
    }
}

// Block p completes the iteration of problem p (residual, stop decision, t + 1).
__global__ __launch_bounds__(BLOCK) void batch_dual_finish(const ProbDesc* __restrict__ pd, const Sched* sched) {
    const ProbDesc& P = pd[blockIdx.x];
    dual_finish_body(P.ctrl, sched, P.respart, nullptr, P.n_dual_blocks);
}

}  // namespace lampk
