// frt_rates.hip -- issue-rate probes of the FP32 vector unit: the sustained
// rate of plain FMA and of each hardware transcendental the distance
// estimators use, over the whole device, with the build's code-generation
// flags (packed FP32 instructions off).  They give the ceilings the march
// kernels are measured against: the FMA rate is the arithmetic ceiling, and
// the transcendental rate a second one for the real-power Mandelbulb, whose
// orbit body calls about ten elementary functions.
//
// Every lane runs kChains independent dependency chains of one operation, so
// latency is hidden by the chains and by the resident waves; the final sum of
// the chains is stored so that nothing is dead code.
#include <hip/hip_runtime.h>

#include "frt_internal.hpp"
#include "frt_math.hpp"

namespace frt {
namespace {

constexpr int kChains = 8;

// One link of a chain for each probed operation.  The negations and
// absolute values are free source modifiers and keep the chains finite
// where that is easy; the rate does not depend on the values.
template <int OP>
__device__ __forceinline__ float link(float v, float a, float b) {
    if constexpr (OP == kRateFma) return fmaf(v, a, b);
    else if constexpr (OP == kRateExp2) return hw_exp2(-fabsf(v));
    else if constexpr (OP == kRateLog2) return hw_log2(fabsf(v));
    else if constexpr (OP == kRateRsq) return hw_rsq(fabsf(v));
    else if constexpr (OP == kRateRcp) return hw_rcp(v);
    else if constexpr (OP == kRateSqrt) return hw_sqrt(fabsf(v));
    else if constexpr (OP == kRateFAdd) return v + b;
    else if constexpr (OP == kRateFMul) return v * a;
    else if constexpr (OP == kRateIntShiftAdd) {
        // two integer operations (shift, add) on the bits of the chain
        const unsigned u = __float_as_uint(v);
        return __uint_as_float(u + (u >> 3));
    } else return hw_sin_rev(v);
}

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(float* __restrict__ sink, int iters, float a, float b) {
    const int gid = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    float v[kChains];
    float w[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        v[i] = 0.25f + 1e-4f * static_cast<float>((gid + 37 * i) & 1023);
        w[i] = 0.5f + 1e-4f * static_cast<float>((gid + 11 * i) & 511);
    }
#pragma unroll 4
    for (int k = 0; k < iters; ++k) {
        if constexpr (OP == kRateMix) {
            // four dependent FMAs per exp2 in each chain pair
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                v[i] = fmaf(fmaf(fmaf(fmaf(v[i], a, b), a, b), a, b), a, b);
                w[i] = hw_exp2(-fabsf(w[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < kChains; ++i) v[i] = link<OP>(v[i], a, b);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += v[i] + w[i];
    sink[gid] = s;
}

}  // namespace

int rate_ops_per_iter(int op) {
    return op == kRateMix ? 5 * kChains : op == kRateIntShiftAdd ? 2 * kChains : kChains;
}

hipError_t launch_rate(int op, int iters, float* sink, int blocks, hipStream_t stream) {
    // a and b keep the FMA chains bounded (|a| < 1) and unknown to the compiler
    const float a = 0.999f, b = 1e-3f;
    const dim3 grid(blocks), block(kRateBlock);
    switch (op) {
        case kRateFma: hipLaunchKernelGGL(rate_kernel<kRateFma>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateExp2: hipLaunchKernelGGL(rate_kernel<kRateExp2>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateLog2: hipLaunchKernelGGL(rate_kernel<kRateLog2>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateRsq: hipLaunchKernelGGL(rate_kernel<kRateRsq>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateRcp: hipLaunchKernelGGL(rate_kernel<kRateRcp>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateSqrt: hipLaunchKernelGGL(rate_kernel<kRateSqrt>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateSin: hipLaunchKernelGGL(rate_kernel<kRateSin>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateFAdd: hipLaunchKernelGGL(rate_kernel<kRateFAdd>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateFMul: hipLaunchKernelGGL(rate_kernel<kRateFMul>, grid, block, 0, stream, sink, iters, a, b); break;
        case kRateIntShiftAdd:
            hipLaunchKernelGGL(rate_kernel<kRateIntShiftAdd>, grid, block, 0, stream, sink, iters, a, b);
            break;
        default: hipLaunchKernelGGL(rate_kernel<kRateMix>, grid, block, 0, stream, sink, iters, a, b); break;
    }
    return hipGetLastError();
}

}  // namespace frt
