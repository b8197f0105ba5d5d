// Measurement support (not part of the method): a throughput probe of the
// transcendental unit.  Each lane runs CHAINS independent chains x <- 2^(-x) of
// v_exp_f32 (the values stay in [1/2, 1]); the chains are independent, so the
// probe measures issue rate rather than latency once enough waves are resident.
#pragma once

#include <hip/hip_runtime.h>

namespace lampk {

constexpr int EXP_PROBE_CHAINS = 8;

__global__ __launch_bounds__(256) void exp_rate_probe(int iters, float seed, float* __restrict__ sink) {
    float x[EXP_PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < EXP_PROBE_CHAINS; ++c) x[c] = seed + 0.01f * (float)(c + (threadIdx.x & 7));
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int c = 0; c < EXP_PROBE_CHAINS; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
    }
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < EXP_PROBE_CHAINS; ++c) acc += x[c];
    // one store per block keeps the chains live without measurable memory traffic
    if (acc == 12345.f) sink[blockIdx.x] = acc;
}

}  // namespace lampk
