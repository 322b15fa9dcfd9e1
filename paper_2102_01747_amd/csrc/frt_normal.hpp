// frt_normal.hpp -- the normal of the estimate at a point, shared by the
// renderer's normal stage and the point query: distance taps (Eq. 5 /
// Listing 5: tetrahedral with h = 0.5773 eps, or central differences with
// h = eps) or the analytic gradient (frt_gradient.hpp), for each kernel
// variant's orbit type.
#pragma once

#include "frt_fractal.hpp"
#include "frt_gradient.hpp"
#include "frt_job.hpp"

namespace frt {

// orbit type of each kernel variant
template <int VAR> struct OrbitOf;
template <> struct OrbitOf<kVarJulia> { using T = JuliaOrbit; };
template <> struct OrbitOf<kVarBulbReal> { using T = BulbOrbit<0>; };
template <> struct OrbitOf<kVarBulbInt> { using T = BulbOrbit<-1>; };
template <> struct OrbitOf<kVarBulb8> { using T = BulbOrbit<8>; };
template <> struct OrbitOf<kVarJuliaDeg> { using T = JuliaDegOrbit; };

// gradient of the estimate with the variant's map form
template <int VAR>
__device__ __forceinline__ int analytic_gradient(const OrbitParams& P, float x, float y, float z, float& gx,
                                                 float& gy, float& gz) {
    if constexpr (VAR == kVarJulia || VAR == kVarJuliaDeg) return julia_gradient(P, x, y, z, gx, gy, gz);
    else if constexpr (VAR == kVarBulbReal) return bulb_gradient<0>(P, x, y, z, gx, gy, gz);
    else if constexpr (VAR == kVarBulbInt) return bulb_gradient<-1>(P, x, y, z, gx, gy, gz);
    else return bulb_gradient<8>(P, x, y, z, gx, gy, gz);
}

// Unnormalised normal at (sx, sy, sz) for normal mode 0 (tetrahedral),
// 1 (central) or 2 (analytic); evals and bodies count the estimates and
// orbit bodies it ran.
template <int VAR>
__device__ __forceinline__ void estimate_normal(const OrbitParams& P, int mode, float sx, float sy, float sz,
                                                float eps, float& gx, float& gy, float& gz, unsigned& evals,
                                                unsigned& bodies) {
    using Orbit = typename OrbitOf<VAR>::T;
    Orbit orb;
    gx = gy = gz = 0.0f;
    bodies = 0;
    if (mode == 0) {
        const float h = 0.5773f * eps;
        for (int k = 0; k < 4; ++k) {
            const float vx = (k == 0 || k == 3) ? 1.0f : -1.0f;
            const float vy = (k >= 2) ? 1.0f : -1.0f;
            const float vz = (k == 1 || k == 3) ? 1.0f : -1.0f;
            const DEResult r = de_once(orb, P, fmaf(h, vx, sx), fmaf(h, vy, sy), fmaf(h, vz, sz));
            gx = fmaf(vx, r.d, gx);
            gy = fmaf(vy, r.d, gy);
            gz = fmaf(vz, r.d, gz);
            bodies += static_cast<unsigned>(r.bodies);
        }
        evals = 4;
    } else if (mode == 2) {
        bodies = static_cast<unsigned>(analytic_gradient<VAR>(P, sx, sy, sz, gx, gy, gz));
        evals = 1;
    } else {
        const float h = eps;
        for (int k = 0; k < 6; ++k) {
            const float sg = (k & 1) ? -h : h;
            const int ax = k >> 1;
            const DEResult r = de_once(orb, P, ax == 0 ? sx + sg : sx, ax == 1 ? sy + sg : sy,
                                       ax == 2 ? sz + sg : sz);
            const float sd = (k & 1) ? -r.d : r.d;
            if (ax == 0) gx += sd; else if (ax == 1) gy += sd; else gz += sd;
            bodies += static_cast<unsigned>(r.bodies);
        }
        evals = 6;
    }
}

// Orbit trap at a point: the minima of |x|, |y|, |z| and of the squared
// norm over the start point and the result of every body of the estimate's
// orbit (the colour parameters of the Mandelbulb distance listing).
template <int VAR>
__device__ __forceinline__ void orbit_trap(const OrbitParams& P, float x, float y, float z, float (&tr)[4]) {
    typename OrbitOf<VAR>::T o;
    o.init(x, y, z);
    float px, py, pz, m;
    o.point(px, py, pz, m);
    tr[0] = fabsf(px);
    tr[1] = fabsf(py);
    tr[2] = fabsf(pz);
    tr[3] = m;
    while (o.k < P.max_iter) {
        const bool in = o.body(P);
        o.point(px, py, pz, m);
        tr[0] = fminf(tr[0], fabsf(px));
        tr[1] = fminf(tr[1], fabsf(py));
        tr[2] = fminf(tr[2], fabsf(pz));
        tr[3] = fminf(tr[3], m);
        if (!in) break;
    }
}

// Unit vector along (gx, gy, gz), scaled by the largest component first
// (analytic gradients carry the orbit's derivative magnitude, whose square
// may exceed float range).  Returns false for a zero or non-finite gradient.
__device__ __forceinline__ bool unit_normal(float gx, float gy, float gz, float& nx, float& ny, float& nz) {
    const float gm = fmaxf(fabsf(gx), fmaxf(fabsf(gy), fabsf(gz)));
    if (!(gm > 0.0f && gm <= 3.4e38f)) return false;
    const float sc = 1.0f / gm;
    gx *= sc;
    gy *= sc;
    gz *= sc;
    const float inv = hw_rsq(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
    nx = gx * inv;
    ny = gy * inv;
    nz = gz * inv;
    return true;
}

}  // namespace frt
