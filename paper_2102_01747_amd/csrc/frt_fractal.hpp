// frt_fractal.hpp -- orbit-derivative distance estimators, one lane per point.
//
// Sec. 2 of the paper: with f^k the k-th iterate and (f^k)' its derivative,
// d = 0.5 |f^k| ln|f^k| / |(f^k)'| (Eq. 2 with the factor the listings use),
// the orbit and derivative advancing by Eq. 3-4.  An orbit stops after
// max_iter bodies or when |z|^2 exceeds bailout2; `it` counts the bodies whose
// result stayed within the bailout (it == max_iter: no escape).
//
// The estimators are written as resumable orbit states (init / step / result)
// so that the persistent kernel can advance every lane by a few bodies per
// trip and let lanes whose orbit has ended move on to their next sample
// without waiting for the slowest lane of the wave.
#pragma once

#include "frt_math.hpp"

namespace frt {

struct DEResult {
    float d;
    int it;      // non-escaping bodies
    int bodies;  // bodies executed
};

// 0.25 ln(m) folded into the log2 hardware op
constexpr float kQuarterLn2 = 0.25f * kLn2;

// Parameters the orbit bodies read.
struct OrbitParams {
    float c0, c1, c2, c3;   // Julia constant
    float n;                // Mandelbulb power
    float nm1_half;         // (n - 1) / 2
    float n_rev;            // n / (2 pi)
    int ipow;               // integer power (0: not an integer)
    int kind;
    int max_iter;
    float bail2;
};

// ---------------------------------------------------------------------------
// Quaternion Julia z^2 + c on the slice z0 = (x, y, z, 0), component 0 real
// (Listing 4 at degree 2).  The squared running derivative gains 4|z_k|^2 per
// body (Eq. 4 with p = 2, |2 z z'| = 2 |z| |z'|); the 4^k factor is applied
// once at the end with ldexp so the body holds one multiply for it.
// ---------------------------------------------------------------------------
struct JuliaOrbit {
    float a, b, e, w, m2, prod;
    int k;
    bool esc;

    __device__ __forceinline__ void init(float x, float y, float z) {
        a = x; b = y; e = z; w = 0.0f;
        m2 = fmaf(a, a, fmaf(b, b, e * e));
        prod = 1.0f;
        k = 0;
        esc = false;
    }
    __device__ __forceinline__ bool done(const OrbitParams& P) const { return esc || k >= P.max_iter; }
    __device__ __forceinline__ void body(const OrbitParams& P) {
        prod *= m2;
        const float vv = fmaf(b, b, fmaf(e, e, w * w));
        const float a2 = a + a;
        const float na = fmaf(a, a, -vv) + P.c0;
        b = fmaf(a2, b, P.c1);
        e = fmaf(a2, e, P.c2);
        w = fmaf(a2, w, P.c3);
        a = na;
        m2 = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
        if (m2 > P.bail2) esc = true; else ++k;
    }
    __device__ __forceinline__ DEResult result() const {
        DEResult r;
        r.bodies = esc ? k + 1 : k;
        r.it = k;
        const float dz2 = ldexpf(prod, 2 * r.bodies);
        r.d = m2 > 0.0f ? kQuarterLn2 * hw_log2(m2) * (m2 * hw_rsq(m2)) * hw_rsq(dz2) : 0.0f;
        return r;
    }
};

// ---------------------------------------------------------------------------
// White-Nylander Mandelbulb (Listing 7 generalised to any n >= 2): y is the
// polar axis, theta = acos(y/r), phi = atan2(x, z);
//   dr <- n r^(n-1) dr + 1,  w <- r^n (sin n th sin n ph, cos n th, sin n th cos n ph) + p.
// MODE 0, real n: r^(n-1) = exp2((n-1)/2 log2 m); angles to the hardware
//   sin/cos in revolutions (n_rev = n / 2pi); acos / atan2 are the library's
//   own polynomials.
// MODE > 0, integer n fixed at compile time (MODE = n), and MODE < 0, integer
//   n read at run time: no trigonometry.  With rho = |(x, z)|,
//   (y + i rho)^n = r^n e^(i n theta) and ((z + i x)/rho)^n = e^(i n phi)
//   by binary powering, so w^n = (Im Y Im Z, Re Y, Im Y Re Z).  On the polar
//   axis (rho = 0) the azimuth factor is 1, matching atan2(0, 0) = 0.
// r = 0 maps to w = p, dr = 1 in every mode.
// ---------------------------------------------------------------------------
template <int MODE>
struct BulbOrbit {
    float wx, wy, wz, m, dr, px, py, pz;
    int k;
    bool esc;

    __device__ __forceinline__ void init(float x, float y, float z) {
        wx = x; wy = y; wz = z;
        px = x; py = y; pz = z;
        m = fmaf(x, x, fmaf(y, y, z * z));
        dr = 1.0f;
        k = 0;
        esc = false;
    }
    __device__ __forceinline__ bool done(const OrbitParams& P) const { return esc || k >= P.max_iter; }
    __device__ __forceinline__ void body(const OrbitParams& P) {
        if constexpr (MODE == 0) {
            const float rn1 = hw_exp2(P.nm1_half * hw_log2(m));
            dr = fmaf(P.n * rn1, dr, 1.0f);
            const float rinv = m > 0.0f ? hw_rsq(m) : 0.0f;
            const float r = m * rinv;
            const float u = fminf(fmaxf(wy * rinv, -1.0f), 1.0f);
            const float bt = fast_acos(u) * P.n_rev;
            const float at = fast_atan2(wx, wz) * P.n_rev;
            const float rn = rn1 * r;
            const float rsb = rn * hw_sin_rev(bt);
            const float ny = fmaf(rn, hw_cos_rev(bt), py);
            const float nx = fmaf(rsb, hw_sin_rev(at), px);
            const float nz = fmaf(rsb, hw_cos_rev(at), pz);
            wx = nx; wy = ny; wz = nz;
        } else {
            const float rinv = m > 0.0f ? hw_rsq(m) : 0.0f;
            const float r = m * rinv;
            const float rho2 = fmaf(wx, wx, wz * wz);
            const float irho = rho2 > 0.0f ? hw_rsq(rho2) : 0.0f;
            float yr = wy, yi = rho2 * irho;
            float zr = rho2 > 0.0f ? wz * irho : 1.0f, zi = wx * irho;
            if constexpr (MODE > 0) {
                dr = fmaf(static_cast<float>(MODE) * ipow_c<MODE - 1>(r), dr, 1.0f);
                cpow_c<MODE>(yr, yi);
                cpow_c<MODE>(zr, zi);
            } else {
                dr = fmaf(P.n * ipow(r, P.ipow - 1), dr, 1.0f);
                cpow_int(yr, yi, P.ipow);
                cpow_int(zr, zi, P.ipow);
            }
            wx = fmaf(yi, zi, px);
            wy = yr + py;
            wz = fmaf(yi, zr, pz);
        }
        m = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
        if (m > P.bail2) esc = true; else ++k;
    }
    __device__ __forceinline__ DEResult result() const {
        DEResult r;
        r.bodies = esc ? k + 1 : k;
        r.it = k;
        r.d = m > 0.0f ? kQuarterLn2 * hw_log2(m) * (m * hw_rsq(m)) * hw_rcp(dr) : 0.0f;
        return r;
    }
};

// Julia or any Mandelbulb mode chosen per lane (batches that mix kinds).
struct MixedOrbit {
    JuliaOrbit j;
    BulbOrbit<0> br;
    BulbOrbit<-1> bi;
    int sel;   // 0 Julia, 1 real power, 2 integer power

    __device__ __forceinline__ void set_kind(const OrbitParams& P) {
        sel = P.kind == 0 ? 0 : (P.ipow > 0 ? 2 : 1);
    }
    __device__ __forceinline__ void init(float x, float y, float z) {
        if (sel == 0) j.init(x, y, z); else if (sel == 1) br.init(x, y, z); else bi.init(x, y, z);
    }
    __device__ __forceinline__ bool done(const OrbitParams& P) const {
        return sel == 0 ? j.done(P) : (sel == 1 ? br.done(P) : bi.done(P));
    }
    __device__ __forceinline__ void body(const OrbitParams& P) {
        if (sel == 0) j.body(P); else if (sel == 1) br.body(P); else bi.body(P);
    }
    __device__ __forceinline__ DEResult result() const {
        return sel == 0 ? j.result() : (sel == 1 ? br.result() : bi.result());
    }
};

// One-shot estimate (all bodies at once) with any orbit type.
template <class O>
__device__ __forceinline__ DEResult de_once(O& o, const OrbitParams& P, float x, float y, float z) {
    o.init(x, y, z);
    while (!o.done(P)) o.body(P);
    return o.result();
}

}  // namespace frt
