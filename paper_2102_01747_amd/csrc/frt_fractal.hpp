// frt_fractal.hpp -- orbit-derivative distance estimators, one lane per point.
//
// Sec. 2 of the paper: with f^k the k-th iterate and (f^k)' its derivative,
// d = 0.5 |f^k| ln|f^k| / |(f^k)'| (Eq. 2 with the factor the listings use),
// the orbit and derivative advancing by Eq. 3-4.  An orbit stops after
// max_iter bodies or when |z|^2 exceeds bailout2; `it` counts the bodies whose
// result stayed within the bailout (it == max_iter: no escape).
//
// The estimators are written as resumable orbit states (init / body /
// result) so that the persistent kernel can advance every lane by a few
// bodies per trip and let lanes whose orbit has ended move on to their next
// sample without waiting for the slowest lane of the wave.  body() returns
// whether the orbit is still within the bailout; the caller stops a lane when
// it returns false or after max_iter bodies (k counts the bodies run).
// step(P, live) is the same body for a loop that runs whole waves with no
// per-lane branch: `live` is the wave's mask of iterating lanes, every lane
// computes the body, and only the values the estimate reads (|z|^2, the
// derivative and k) are kept in live lanes -- a stopped lane's other
// coordinates run on unused until its next init.  It returns the mask of
// lanes still iterating.
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
// floor under |w|^2 and rho^2 before a reciprocal square root (keeps rsq finite)
constexpr float kTinyFloor = 1e-30f;

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

    __device__ __forceinline__ void init(float x, float y, float z) {
        a = x; b = y; e = z; w = 0.0f;
        m2 = fmaf(a, a, fmaf(b, b, e * e));
        prod = 1.0f;
        k = 0;
    }
    // current orbit point (first three components) and |z|^2
    __device__ __forceinline__ void point(float& x, float& y, float& z, float& m) const {
        x = a; y = b; z = e; m = m2;
    }
    __device__ __forceinline__ bool body(const OrbitParams& P) {
        prod *= m2;
        const float vv = fmaf(b, b, fmaf(e, e, w * w));
        const float a2 = a + a;
        const float na = fmaf(a, a, -vv) + P.c0;
        b = fmaf(a2, b, P.c1);
        e = fmaf(a2, e, P.c2);
        w = fmaf(a2, w, P.c3);
        a = na;
        m2 = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
        ++k;
        return !(m2 > P.bail2);
    }
    __device__ __forceinline__ unsigned long long step(const OrbitParams& P, unsigned long long live_mask) {
        // The body is short, so stopped lanes run it too and keep their
        // estimate's inputs by three selects: cheaper here than switching
        // the exec mask around it (the longer bodies below do that).
        const bool live = __builtin_amdgcn_inverse_ballot_w64(live_mask);
        const float pn = prod * m2;
        const float vv = fmaf(b, b, fmaf(e, e, w * w));
        const float a2 = a + a;
        const float na = fmaf(a, a, -vv) + P.c0;
        b = fmaf(a2, b, P.c1);
        e = fmaf(a2, e, P.c2);
        w = fmaf(a2, w, P.c3);
        a = na;
        const float mn = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
        const int kn = k + 1;
        prod = live ? pn : prod;
        m2 = live ? mn : m2;
        k = live ? kn : k;
        return live_mask & __builtin_amdgcn_ballot_w64(!(mn > P.bail2)) & __builtin_amdgcn_ballot_w64(kn < P.max_iter);
    }
    __device__ __forceinline__ DEResult result(const OrbitParams& P) const {
        DEResult r;
        const bool esc = m2 > P.bail2;
        r.bodies = k;
        r.it = esc ? k - 1 : k;
        const float dz2 = ldexpf(prod, 2 * k);
        r.d = m2 > 0.0f ? kQuarterLn2 * hw_log2(m2) * (m2 * hw_rsq(m2)) * hw_rsq(dz2) : 0.0f;
        return r;
    }
};

// ---------------------------------------------------------------------------
// Quaternion Julia z^p + c for an integer degree p >= 2 read at run time
// (Eq. 3-4; Listing 4 is the cubic).  Powers of one quaternion z = a + v stay
// in the plane span{1, v}: z^j = R_j + Q_j v with R_1 = a, Q_1 = 1 and, since
// v v = -|v|^2,
//   R_(j+1) = a R_j - |v|^2 Q_j,   Q_(j+1) = R_j + a Q_j,
// three operations per degree and no square root (z^2 = a^2 - |v|^2 + 2a v
// is the first step).  The squared running derivative gains
// p^2 |z|^(2(p-1)) per body (Eq. 4 taken in norm; the quaternion norm is
// multiplicative).
// ---------------------------------------------------------------------------
struct JuliaDegOrbit {
    // dz2 is kept as dm * 2^de with dm in [0.5, 1): a body multiplies it by
    // p^2 |z|^(2(p-1)), up to about 2^120 at the largest accepted degree and
    // bailout, so the product of a few bodies leaves float range long before
    // the estimate it feeds stops mattering.
    float a, b, e, w, m2, dm;
    int k, de;

    __device__ __forceinline__ void init(float x, float y, float z) {
        a = x; b = y; e = z; w = 0.0f;
        m2 = fmaf(a, a, fmaf(b, b, e * e));
        dm = 0.5f;
        de = 1;
        k = 0;
    }
    // current orbit point (first three components) and |z|^2
    __device__ __forceinline__ void point(float& x, float& y, float& z, float& m) const {
        x = a; y = b; z = e; m = m2;
    }
    // z^p + c into (na, nb, ne, nw) and the body's derivative factor
    __device__ __forceinline__ void map(const OrbitParams& P, float& na, float& nb, float& ne, float& nw,
                                        float& fac) const {
        const float vv = fmaf(b, b, fmaf(e, e, w * w));
        float R = fmaf(a, a, -vv), Q = a + a, mp = m2;
        for (int j = 2; j < P.ipow; ++j) {
            const float nR = fmaf(a, R, -vv * Q);
            Q = fmaf(a, Q, R);
            R = nR;
            mp *= m2;
        }
        na = R + P.c0;
        nb = fmaf(Q, b, P.c1);
        ne = fmaf(Q, e, P.c2);
        nw = fmaf(Q, w, P.c3);
        fac = (P.n * P.n) * mp;
    }
    __device__ __forceinline__ bool body(const OrbitParams& P) {
        float na, nb, ne, nw, fac;
        map(P, na, nb, ne, nw, fac);
        a = na; b = nb; e = ne; w = nw;
        const float prod = dm * fac;
        dm = __builtin_amdgcn_frexp_mantf(prod);
        de += __builtin_amdgcn_frexp_expf(prod);
        m2 = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
        ++k;
        return !(m2 > P.bail2);
    }
    __device__ __forceinline__ unsigned long long step(const OrbitParams& P, unsigned long long live_mask) {
        // the body runs under the live lanes' exec mask: stopped lanes keep
        // their state without selects
        if (__builtin_amdgcn_inverse_ballot_w64(live_mask)) {
            float na, nb, ne, nw, fac;
            map(P, na, nb, ne, nw, fac);
            a = na; b = nb; e = ne; w = nw;
            const float prod = dm * fac;
            dm = __builtin_amdgcn_frexp_mantf(prod);
            de += __builtin_amdgcn_frexp_expf(prod);
            m2 = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
            ++k;
        }
        return live_mask & __builtin_amdgcn_ballot_w64(!(m2 > P.bail2)) & __builtin_amdgcn_ballot_w64(k < P.max_iter);
    }
    __device__ __forceinline__ DEResult result(const OrbitParams& P) const {
        DEResult r;
        const bool esc = m2 > P.bail2;
        r.bodies = k;
        r.it = esc ? k - 1 : k;
        // 1 / sqrt(dm 2^de) = rsq(dm 2^(de & 1)) 2^-(de >> 1), the odd power folded into the mantissa
        const float inv = ldexpf(hw_rsq(ldexpf(dm, de & 1)), -(de >> 1));
        r.d = m2 > 0.0f ? kQuarterLn2 * hw_log2(m2) * (m2 * hw_rsq(m2)) * inv : 0.0f;
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
// r^(K-1) from m = r^2 for a compile-time integer power K >= 2: m^((K-1)/2)
// for odd K, m^(K/2-1) sqrt(m) for even K (sqrt(0) = 0 needs no floor).
template <int K>
__device__ __forceinline__ float bulb_rpow(float m) {
    if constexpr (K & 1) return ipow_c<(K - 1) / 2>(m);
    else if constexpr (K == 2) return hw_sqrt(m);
    else return ipow_c<K / 2 - 1>(m) * hw_sqrt(m);
}

// The derivative step dr' = K r^(K-1) dr + 1.  For K = 8 it is taken as
// 2 (4 r^7 dr + 0.5): scalings by powers of two are exact, so the value is
// the same, and both fold into the output modifiers of the multiply and the
// fma that precede them instead of costing a multiply of their own.
template <int K>
__device__ __forceinline__ float bulb_dr_step(float m, float dr) {
    if constexpr (K == 8) return 2.0f * fmaf(4.0f * bulb_rpow<8>(m), dr, 0.5f);
    else return fmaf(static_cast<float>(K) * bulb_rpow<K>(m), dr, 1.0f);
}

template <int MODE>
struct BulbOrbit {
    float wx, wy, wz, m, dr, px, py, pz;
    int k;

    __device__ __forceinline__ void init(float x, float y, float z) {
        wx = x; wy = y; wz = z;
        px = x; py = y; pz = z;
        m = fmaf(x, x, fmaf(y, y, z * z));
        dr = 1.0f;
        k = 0;
    }
    // current orbit point and |w|^2
    __device__ __forceinline__ void point(float& x, float& y, float& z, float& mm) const {
        x = wx; y = wy; z = wz; mm = m;
    }
    // one body from (w, m, dr): the new point and derivative
    __device__ __forceinline__ void map(const OrbitParams& P, float& nx, float& ny, float& nz, float& ndr) const {
        if constexpr (MODE == 0) {
            const float rn1 = hw_exp2(P.nm1_half * hw_log2(m));
            ndr = fmaf(P.n * rn1, dr, 1.0f);
            const float rinv = m > 0.0f ? hw_rsq(m) : 0.0f;
            const float r = m * rinv;
            const float u = fminf(fmaxf(wy * rinv, -1.0f), 1.0f);
            const float bt = fast_acos(u) * P.n_rev;
            const float at = fast_atan2(wx, wz) * P.n_rev;
            const float rn = rn1 * r;
            const float rsb = rn * hw_sin_rev(bt);
            ny = fmaf(rn, hw_cos_rev(bt), py);
            nx = fmaf(rsb, hw_sin_rev(at), px);
            nz = fmaf(rsb, hw_cos_rev(at), pz);
        } else {
            const float rho2 = fmaxf(fmaf(wx, wx, wz * wz), kTinyFloor);
            const float irho = hw_rsq(rho2);
            float yr = wy, yi = rho2 * irho;
            float zr = wz * irho, zi = wx * irho;
            if constexpr (MODE > 0) {
                ndr = bulb_dr_step<MODE>(m, dr);
                cpow_c<MODE>(yr, yi);
                cpow_c<MODE>(zr, zi);
            } else {
                ndr = fmaf(P.n * ipow(hw_sqrt(m), P.ipow - 1), dr, 1.0f);
                cpow_int(yr, yi, P.ipow);
                cpow_int(zr, zi, P.ipow);
            }
            nx = fmaf(yi, zi, px);
            ny = yr + py;
            nz = fmaf(yi, zr, pz);
        }
    }
    __device__ __forceinline__ unsigned long long step(const OrbitParams& P, unsigned long long live_mask) {
        // the body runs under the live lanes' exec mask: stopped lanes keep
        // their state without selects
        if (__builtin_amdgcn_inverse_ballot_w64(live_mask)) {
            float nx, ny, nz, ndr;
            map(P, nx, ny, nz, ndr);
            wx = nx; wy = ny; wz = nz;
            m = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
            dr = ndr;
            ++k;
        }
        return live_mask & __builtin_amdgcn_ballot_w64(!(m > P.bail2)) & __builtin_amdgcn_ballot_w64(k < P.max_iter);
    }
    __device__ __forceinline__ bool body(const OrbitParams& P) {
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
            // tiny floors instead of branches: at r = 0 or rho = 0 the
            // factors they scale are zero (r^(n-1) dr, and Im Y = 0 on the
            // polar axis), so the floor changes no result
            const float rho2 = fmaxf(fmaf(wx, wx, wz * wz), kTinyFloor);
            const float irho = hw_rsq(rho2);
            float yr = wy, yi = rho2 * irho;
            float zr = wz * irho, zi = wx * irho;
            if constexpr (MODE > 0) {
                dr = bulb_dr_step<MODE>(m, dr);
                cpow_c<MODE>(yr, yi);
                cpow_c<MODE>(zr, zi);
            } else {
                dr = fmaf(P.n * ipow(hw_sqrt(m), P.ipow - 1), dr, 1.0f);
                cpow_int(yr, yi, P.ipow);
                cpow_int(zr, zi, P.ipow);
            }
            wx = fmaf(yi, zi, px);
            wy = yr + py;
            wz = fmaf(yi, zr, pz);
        }
        m = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
        ++k;
        return !(m > P.bail2);
    }
    __device__ __forceinline__ DEResult result(const OrbitParams& P) const {
        DEResult r;
        const bool esc = m > P.bail2;
        r.bodies = k;
        r.it = esc ? k - 1 : k;
        r.d = m > 0.0f ? kQuarterLn2 * hw_log2(m) * (m * hw_rsq(m)) * hw_rcp(dr) : 0.0f;
        return r;
    }
};

// One-shot estimate (all bodies at once) with any orbit type; max_iter >= 1.
template <class O>
__device__ __forceinline__ DEResult de_once(O& o, const OrbitParams& P, float x, float y, float z) {
    o.init(x, y, z);
    while (o.body(P) && o.k < P.max_iter) {
    }
    return o.result(P);
}

}  // namespace frt
