// frt_query.hip -- point queries: the distance estimate and the normal at
// arbitrary points (the same orbit and normal code the renderer uses) and an
// evaluator of the library's fast float32 transcendentals, for accuracy
// checks.
#include <hip/hip_runtime.h>

#include "frt_fractal.hpp"
#include "frt_internal.hpp"
#include "frt_job.hpp"
#include "frt_normal.hpp"

namespace frt {

template <class O>
__global__ void __launch_bounds__(256) distance_kernel(OrbitParams P, const float* __restrict__ pts, long long n,
                                                       float* __restrict__ d, int* __restrict__ it) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    O o;
    const DEResult r = de_once(o, P, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
    d[i] = r.d;
    if (it) it[i] = r.it;
}

hipError_t launch_distance(int variant, const OrbitParams& P, const float* pts, long long n, float* d, int* it,
                           hipStream_t stream) {
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    switch (variant) {
        case kVarJulia:
            hipLaunchKernelGGL(distance_kernel<JuliaOrbit>, dim3(grid), dim3(block), 0, stream, P, pts, n, d, it);
            break;
        case kVarBulbReal:
            hipLaunchKernelGGL(distance_kernel<BulbOrbit<0>>, dim3(grid), dim3(block), 0, stream, P, pts, n, d, it);
            break;
        case kVarBulbInt:
            hipLaunchKernelGGL(distance_kernel<BulbOrbit<-1>>, dim3(grid), dim3(block), 0, stream, P, pts, n, d, it);
            break;
        case kVarBulb8:
            hipLaunchKernelGGL(distance_kernel<BulbOrbit<8>>, dim3(grid), dim3(block), 0, stream, P, pts, n, d, it);
            break;
        default:
            hipLaunchKernelGGL(distance_kernel<JuliaDegOrbit>, dim3(grid), dim3(block), 0, stream, P, pts, n, d, it);
            break;
    }
    return hipGetLastError();
}

template <int VAR>
__global__ void __launch_bounds__(256) normal_query_kernel(OrbitParams P, int mode, const float* __restrict__ pts,
                                                           const float* __restrict__ eps, long long n,
                                                           float* __restrict__ out) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gx, gy, gz, nx = 0.0f, ny = 0.0f, nz = 0.0f;
    unsigned evals, bodies;
    estimate_normal<VAR>(P, mode, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], eps ? eps[i] : 0.0f, gx, gy, gz,
                         evals, bodies);
    if (!unit_normal(gx, gy, gz, nx, ny, nz)) nx = ny = nz = 0.0f;
    out[3 * i] = nx;
    out[3 * i + 1] = ny;
    out[3 * i + 2] = nz;
}

hipError_t launch_normal_query(int variant, const OrbitParams& P, int mode, const float* pts, const float* eps,
                               long long n, float* out, hipStream_t stream) {
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    switch (variant) {
        case kVarJulia:
            hipLaunchKernelGGL(normal_query_kernel<kVarJulia>, dim3(grid), dim3(block), 0, stream, P, mode, pts, eps,
                               n, out);
            break;
        case kVarBulbReal:
            hipLaunchKernelGGL(normal_query_kernel<kVarBulbReal>, dim3(grid), dim3(block), 0, stream, P, mode, pts,
                               eps, n, out);
            break;
        case kVarBulbInt:
            hipLaunchKernelGGL(normal_query_kernel<kVarBulbInt>, dim3(grid), dim3(block), 0, stream, P, mode, pts,
                               eps, n, out);
            break;
        case kVarBulb8:
            hipLaunchKernelGGL(normal_query_kernel<kVarBulb8>, dim3(grid), dim3(block), 0, stream, P, mode, pts, eps,
                               n, out);
            break;
        default:
            hipLaunchKernelGGL(normal_query_kernel<kVarJuliaDeg>, dim3(grid), dim3(block), 0, stream, P, mode, pts,
                               eps, n, out);
            break;
    }
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) math_kernel(int func, const float* __restrict__ x, const float* __restrict__ y,
                                                   float* __restrict__ out, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a = x[i];
    float r;
    switch (func) {
        case 0: r = fast_acos(fminf(fmaxf(a, -1.0f), 1.0f)); break;
        case 1: r = fast_atan2(a, y[i]); break;
        case 2: r = hw_sin_rev(a); break;
        case 3: r = hw_cos_rev(a); break;
        case 4: r = hw_log2(a); break;
        case 5: r = hw_exp2(a); break;
        case 6: r = hw_rsq(a); break;
        default: r = hw_rcp(a); break;
    }
    out[i] = r;
}

hipError_t launch_math(int func, const float* x, const float* y, float* out, long long n, hipStream_t stream) {
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    hipLaunchKernelGGL(math_kernel, dim3(grid), dim3(block), 0, stream, func, x, y, out, n);
    return hipGetLastError();
}

}  // namespace frt
