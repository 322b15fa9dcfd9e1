// frt_math.hpp -- fast float32 math for gfx950 used by the distance estimators.
//
// Hardware transcendentals of the CDNA vector unit (quarter rate):
//   v_log_f32 (log2), v_exp_f32 (exp2), v_rsq_f32, v_sqrt_f32, v_rcp_f32,
//   v_sin_f32 / v_cos_f32 (argument in revolutions: sin(2 pi x)).
// acos and atan are the library's own minimax polynomials, fitted by
// csrc/fit_fastmath.py (Lawson-refined least squares on Chebyshev nodes):
//   acos(x) = sqrt(1 - x) P(x) on [0, 1], max error 6.8e-8 rad (double eval)
//   atan(s) = s Q(s^2)      on [0, 1], max error 2.2e-8 rad (double eval)
#pragma once

#include <hip/hip_runtime.h>

namespace frt {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kInv2Pi = 0.15915494309189533577f;
constexpr float kLn2 = 0.69314718055994530942f;

__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// sin / cos of 2*pi*x (x in revolutions)
__device__ __forceinline__ float hw_sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float hw_cos_rev(float x) { return __builtin_amdgcn_cosf(x); }

// natural log via log2
__device__ __forceinline__ float fast_ln(float x) { return hw_log2(x) * kLn2; }

// acos on [-1, 1] (argument must already be clamped)
__device__ __forceinline__ float fast_acos(float x) {
    const float ax = fabsf(x);
    float p = -1.441480010e-03f;
    p = fmaf(p, ax, 7.245448418e-03f);
    p = fmaf(p, ax, -1.780898497e-02f);
    p = fmaf(p, ax, 3.133546934e-02f);
    p = fmaf(p, ax, -5.031278357e-02f);
    p = fmaf(p, ax, 8.899926394e-02f);
    p = fmaf(p, ax, -2.145998925e-01f);
    p = fmaf(p, ax, 1.570796371e+00f);
    const float r = hw_sqrt(1.0f - ax) * p;
    return x < 0.0f ? kPi - r : r;
}

// atan2(y, x) with atan2(0, 0) = 0
__device__ __forceinline__ float fast_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float s = mx > 0.0f ? mn * hw_rcp(mx) : 0.0f;
    const float s2 = s * s;
    float q = 2.456725342e-03f;
    q = fmaf(q, s2, -1.440136135e-02f);
    q = fmaf(q, s2, 3.978123143e-02f);
    q = fmaf(q, s2, -7.234857976e-02f);
    q = fmaf(q, s2, 1.049894616e-01f);
    q = fmaf(q, s2, -1.416122913e-01f);
    q = fmaf(q, s2, 1.998590678e-01f);
    q = fmaf(q, s2, -3.333259821e-01f);
    q = fmaf(q, s2, 9.999998808e-01f);
    float r = s * q;
    r = ay > ax ? kHalfPi - r : r;
    r = x < 0.0f ? kPi - r : r;
    return copysignf(r, y);
}

// x^k for integer k >= 1 by left-to-right binary exponentiation
__device__ __forceinline__ float ipow(float x, int k) {
    float r = x;
    const int top = 31 - __builtin_clz(k);
    for (int bit = top - 1; bit >= 0; --bit) {
        r = r * r;
        if ((k >> bit) & 1) r = r * x;
    }
    return r;
}

// x^K and (re + i im)^K for a compile-time K >= 1: the exponentiation chain
// is unrolled with no run-time bit tests.
template <int K>
__device__ __forceinline__ float ipow_c(float x) {
    if constexpr (K == 1) {
        return x;
    } else {
        const float h = ipow_c<K / 2>(x);
        return (K & 1) ? h * h * x : h * h;
    }
}

template <int K>
__device__ __forceinline__ void cpow_c(float& re, float& im) {
    if constexpr (K > 1) {
        const float br = re, bi = im;
        cpow_c<K / 2>(re, im);
        // the doubling applies to the product, where it can fold into the
        // multiply as an output modifier; the value is the same
        const float sr = fmaf(re, re, -im * im);
        const float si = (re * im) * 2.0f;
        re = sr;
        im = si;
        if constexpr (K & 1) {
            const float mr = fmaf(re, br, -im * bi);
            const float mi = fmaf(re, bi, im * br);
            re = mr;
            im = mi;
        }
    }
}

// (re + i im)^k for integer k >= 1, same scheme as ipow
__device__ __forceinline__ void cpow_int(float& re, float& im, int k) {
    const float br = re, bi = im;
    const int top = 31 - __builtin_clz(k);
    for (int bit = top - 1; bit >= 0; --bit) {
        const float sr = fmaf(re, re, -im * im);
        const float si = (re * im) * 2.0f;
        re = sr;
        im = si;
        if ((k >> bit) & 1) {
            const float mr = fmaf(re, br, -im * bi);
            const float mi = fmaf(re, bi, im * br);
            re = mr;
            im = mi;
        }
    }
}

}  // namespace frt
