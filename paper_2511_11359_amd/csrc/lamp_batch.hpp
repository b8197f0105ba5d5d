// Batching form: many independent problems advance together, one launch per phase of
// the iteration for all of them.  Each phase kernel is a persistent loop of a
// machine-sized grid over a work list of (problem, tile) items; an item runs the same
// device body as the single-problem kernels, with that problem's descriptor.  Every
// problem keeps its own control block, so a problem that meets its tolerance stops
// (its items exit at once) while the others continue.
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
    double2* rpart;
    double2* cpart;
    DualBufs buf;
    double* respart;
};

struct Item {
    int32_t prob, bx, by, pad;
};

#define LAMP_BATCH_D(X) X(1) X(2) X(3) X(4) X(8) X(16)

__global__ __launch_bounds__(BLOCK) void batch_row_sweep(const ProbDesc* __restrict__ pd,
                                                         const Item* __restrict__ items, int n_items,
                                                         const Sched* sched) {
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        switch (P.d) {
#define CASE(D)                                                                                         \
    case D:                                                                                             \
        row_sweep_body<D>(P.ctrl, sched, P.kc, P.xc, P.yc, P.gtab, P.H, P.rpart, P.split_r, it.bx, it.by, \
                          0);                                                                            \
        break;
            LAMP_BATCH_D(CASE)
#undef CASE
            default:
                row_sweep_dyn_body(P.ctrl, sched, P.kc, P.d, P.xc, P.yc, P.gtab, P.H, P.rpart, P.split_r, it.bx,
                                   it.by, 0);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void batch_row_finish(const ProbDesc* __restrict__ pd,
                                                          const Item* __restrict__ items, int n_items,
                                                          const Sched* sched) {
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        row_finish_body(P.ctrl, sched, P.kc, P.d, P.xc, P.yc, P.gtab, P.r, P.xn2, P.rpart, P.P_r, P.H, P.rowvar,
                        nullptr, nullptr, RowVarF32{nullptr, nullptr, nullptr, nullptr, 0}, it.bx, it.by, 0);
    }
}

__global__ __launch_bounds__(BLOCK) void batch_col_sweep(const ProbDesc* __restrict__ pd,
                                                         const Item* __restrict__ items, int n_items,
                                                         const Sched* sched) {
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        switch (P.d) {
#define CASE(D)                                                                                          \
    case D:                                                                                              \
        col_sweep_body<D>(P.ctrl, sched, P.kc, P.xc, P.yc, P.gtab, P.rowvar, P.cpart, P.split_c, it.bx, it.by, \
                          0);                                                                             \
        break;
            LAMP_BATCH_D(CASE)
#undef CASE
            default:
                col_sweep_dyn_body(P.ctrl, sched, P.kc, P.d, P.xc, P.yc, P.gtab, P.rowvar, P.cpart, P.split_c,
                                   it.bx, it.by, 0);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void batch_dual_update(const ProbDesc* __restrict__ pd,
                                                           const Item* __restrict__ items, int n_items,
                                                           const Sched* sched) {
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const Item it = items[k];
        const ProbDesc& P = pd[it.prob];
        dual_update_body(P.ctrl, sched, P.kc, P.cpart, P.P_c, P.c, P.yn2, P.buf, P.gtab, nullptr, 0, P.respart,
                         TraceCols{nullptr, nullptr, nullptr, nullptr}, it.bx, 0, P.n_dual_blocks);
    }
}

}  // namespace lampk
