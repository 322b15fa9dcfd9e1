// frt_gradient.hpp -- analytic normals: the gradient of the distance
// estimate at a point, by forward-mode differentiation of the orbit with the
// three spatial tangents carried beside it, in float32.
//
// Sec. 2 observes that on the set the gradient of d = G / |grad G| is
// grad G / |grad G|, and then approximates it with distance taps (Eq. 5).
// Here the gradient of the estimate itself (running derivative included) is
// taken at the hit point, with no tap spacing.  A normal needs only the
// direction, so positive factors common to the three components are dropped:
//
// Julia, d = A sqrt(m2 / dz2) with A = 0.25 ln m2:
//   grad d ~ (0.25 + 0.5 A) grad(m2) / m2 - 0.5 A grad(ln dz2),
//   grad(ln dz2) = sum over bodies of 2 (p - 1) z . z' / |z|^2
//   (each body multiplies dz2 by p^2 |z|^(2(p-1))).
// Mandelbulb, d = 0.25 ln m sqrt(m) / dr:
//   grad d ~ (1 + 0.5 ln m) grad(m) / m - ln m grad(dr) / dr,
//   with the relative tangent rho = dr' / dr advancing, from
//   dr_new = n r^(n-1) dr + 1, as rho <- (1 - 1/dr_new) ((n - 1) r'/r + rho).
// The spatial tangent of the Mandelbulb gains e_i every body (the point is
// also the additive constant).  Each function returns the bodies it ran.
#pragma once

#include "frt_fractal.hpp"

namespace frt {

// Quaternion Julia z^p + c, any degree p >= 2 (P.ipow): the power recurrence
// of JuliaDegOrbit with its tangents, z^j = R_j + Q_j v,
//   R'_(j+1) = a' R_j + a R'_j - (|v|^2)' Q_j - |v|^2 Q'_j,
//   Q'_(j+1) = R'_j + a' Q_j + a Q'_j.
__device__ __forceinline__ int julia_gradient(const OrbitParams& P, float x, float y, float z, float& gx,
                                              float& gy, float& gz) {
    float a = x, b = y, e = z, w = 0.0f;
    float ta[3] = {1.0f, 0.0f, 0.0f}, tb[3] = {0.0f, 1.0f, 0.0f}, te[3] = {0.0f, 0.0f, 1.0f};
    float tw[3] = {0.0f, 0.0f, 0.0f}, L[3] = {0.0f, 0.0f, 0.0f};
    float m2 = fmaf(a, a, fmaf(b, b, e * e));
    const float lfac = 2.0f * static_cast<float>(P.ipow - 1);
    int k = 0;
    while (k < P.max_iter) {
        const float il = lfac * hw_rcp(fmaxf(m2, kTinyFloor));
        const float vv = fmaf(b, b, fmaf(e, e, w * w));
        float R = fmaf(a, a, -vv), Q = a + a;
        float dR[3], dQ[3], dvv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float bt = fmaf(b, tb[i], fmaf(e, te[i], w * tw[i]));
            L[i] = fmaf(fmaf(a, ta[i], bt), il, L[i]);
            dvv[i] = bt + bt;
            dR[i] = 2.0f * fmaf(a, ta[i], -bt);
            dQ[i] = ta[i] + ta[i];
        }
        for (int j = 2; j < P.ipow; ++j) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float nr = fmaf(ta[i], R, fmaf(a, dR[i], -fmaf(dvv[i], Q, vv * dQ[i])));
                dQ[i] = fmaf(ta[i], Q, fmaf(a, dQ[i], dR[i]));
                dR[i] = nr;
            }
            const float nR = fmaf(a, R, -vv * Q);
            Q = fmaf(a, Q, R);
            R = nR;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float nb = fmaf(dQ[i], b, Q * tb[i]);
            const float ne = fmaf(dQ[i], e, Q * te[i]);
            const float nw = fmaf(dQ[i], w, Q * tw[i]);
            ta[i] = dR[i];
            tb[i] = nb;
            te[i] = ne;
            tw[i] = nw;
        }
        a = R + P.c0;
        b = fmaf(Q, b, P.c1);
        e = fmaf(Q, e, P.c2);
        w = fmaf(Q, w, P.c3);
        m2 = fmaf(a, a, fmaf(b, b, fmaf(e, e, w * w)));
        ++k;
        if (m2 > P.bail2) break;
    }
    const float A = kQuarterLn2 * hw_log2(fmaxf(m2, kTinyFloor));
    const float c1 = 2.0f * fmaf(0.5f, A, 0.25f) * hw_rcp(fmaxf(m2, kTinyFloor));
    const float c2 = 0.5f * A;
    float g[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float zt = fmaf(a, ta[i], fmaf(b, tb[i], fmaf(e, te[i], w * tw[i])));
        g[i] = fmaf(c1, zt, -c2 * L[i]);
    }
    gx = g[0];
    gy = g[1];
    gz = g[2];
    return k;
}

// White-Nylander Mandelbulb with the map forms of BulbOrbit<MODE>: MODE 0
// real n (angles theta = atan2(rho, y), phi = atan2(x, z) differentiated as
// theta' = (y rho' - rho y') / r^2, phi' = (z x' - x z') / rho^2); MODE > 0
// compile-time and MODE < 0 run-time integer n (Y = y + i rho and
// U = (z + i x) / rho raised to the n-th power, d(Y^n) = n Y^(n-1) dY).
template <int MODE>
__device__ __forceinline__ int bulb_gradient(const OrbitParams& P, float x, float y, float z, float& gx,
                                             float& gy, float& gz) {
    float wx = x, wy = y, wz = z;
    float tx[3] = {1.0f, 0.0f, 0.0f}, ty[3] = {0.0f, 1.0f, 0.0f}, tz[3] = {0.0f, 0.0f, 1.0f};
    float rho[3] = {0.0f, 0.0f, 0.0f};
    float m = fmaf(x, x, fmaf(y, y, z * z));
    float dr = 1.0f;
    const float n = P.n;
    int k = 0;
    while (k < P.max_iter) {
        const float mf = fmaxf(m, kTinyFloor);
        const float mi = hw_rcp(mf);
        const float rinv = hw_rsq(mf);
        // r^(n-1)
        float rn1;
        if constexpr (MODE == 0) {
            rn1 = hw_exp2(P.nm1_half * hw_log2(mf));
        } else if constexpr (MODE > 0) {
            if constexpr ((MODE & 1) == 0) rn1 = ipow_c<MODE / 2>(m) * rinv;
            else rn1 = ipow_c<(MODE - 1) / 2>(m);
        } else {
            rn1 = ipow(m * rinv, P.ipow - 1);
        }
        const float ndr = fmaf(n * rn1, dr, 1.0f);
        const float q = 1.0f - hw_rcp(ndr);
        float s[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s[i] = fmaf(wx, tx[i], fmaf(wy, ty[i], wz * tz[i])) * mi;
            rho[i] = q * fmaf(n - 1.0f, s[i], rho[i]);
        }
        const float rho2 = fmaxf(fmaf(wx, wx, wz * wz), kTinyFloor);
        const float irho = hw_rsq(rho2);
        float nx, ny, nz;
        if constexpr (MODE == 0) {
            const float rr = m * rinv;
            const float u = fminf(fmaxf(wy * rinv, -1.0f), 1.0f);
            const float bt = fast_acos(u) * P.n_rev;
            const float at = fast_atan2(wx, wz) * P.n_rev;
            const float sB = hw_sin_rev(bt), cB = hw_cos_rev(bt);
            const float sA = hw_sin_rev(at), cA = hw_cos_rev(at);
            const float rn = rn1 * rr;
            const float rh = rho2 * irho;
            const float irho2 = irho * irho;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float drh = fmaf(wx, tx[i], wz * tz[i]) * irho;
                const float Bp = n * fmaf(wy, drh, -rh * ty[i]) * mi;
                const float Ap = n * fmaf(wz, tx[i], -wx * tz[i]) * irho2;
                const float rnp = n * rn * s[i];
                const float ntx = fmaf(rnp, sB * sA, rn * fmaf(cB * Bp, sA, sB * cA * Ap));
                const float nty = fmaf(rnp, cB, -rn * sB * Bp);
                const float ntz = fmaf(rnp, sB * cA, rn * fmaf(cB * Bp, cA, -sB * sA * Ap));
                tx[i] = ntx + (i == 0 ? 1.0f : 0.0f);
                ty[i] = nty + (i == 1 ? 1.0f : 0.0f);
                tz[i] = ntz + (i == 2 ? 1.0f : 0.0f);
            }
            const float rsb = rn * sB;
            nx = fmaf(rsb, sA, x);
            ny = fmaf(rn, cB, y);
            nz = fmaf(rsb, cA, z);
        } else {
            const float Yr = wy, Yi = rho2 * irho;
            const float Ur = wz * irho, Ui = wx * irho;
            float y1r = Yr, y1i = Yi, u1r = Ur, u1i = Ui;   // Y^(n-1), U^(n-1)
            if constexpr (MODE > 0) {
                if constexpr (MODE > 2) {
                    cpow_c<MODE - 1>(y1r, y1i);
                    cpow_c<MODE - 1>(u1r, u1i);
                }
            } else {
                if (P.ipow > 2) {
                    cpow_int(y1r, y1i, P.ipow - 1);
                    cpow_int(u1r, u1i, P.ipow - 1);
                }
            }
            const float ynr = fmaf(y1r, Yr, -y1i * Yi), yni = fmaf(y1r, Yi, y1i * Yr);
            const float unr = fmaf(u1r, Ur, -u1i * Ui), uni = fmaf(u1r, Ui, u1i * Ur);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float drh = fmaf(wx, tx[i], wz * tz[i]) * irho;
                const float dyr = ty[i], dyi = drh;
                const float dur = fmaf(-Ur, drh, tz[i]) * irho, dui = fmaf(-Ui, drh, tx[i]) * irho;
                const float dynr = n * fmaf(y1r, dyr, -y1i * dyi), dyni = n * fmaf(y1r, dyi, y1i * dyr);
                const float dunr = n * fmaf(u1r, dur, -u1i * dui), duni = n * fmaf(u1r, dui, u1i * dur);
                const float ntx = fmaf(dyni, uni, yni * duni);
                const float ntz = fmaf(dyni, unr, yni * dunr);
                tx[i] = ntx + (i == 0 ? 1.0f : 0.0f);
                ty[i] = dynr + (i == 1 ? 1.0f : 0.0f);
                tz[i] = ntz + (i == 2 ? 1.0f : 0.0f);
            }
            nx = fmaf(yni, uni, x);
            ny = ynr + y;
            nz = fmaf(yni, unr, z);
        }
        wx = nx;
        wy = ny;
        wz = nz;
        m = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
        dr = ndr;
        ++k;
        if (m > P.bail2) break;
    }
    const float mf = fmaxf(m, kTinyFloor);
    const float lnm = kLn2 * hw_log2(mf);
    const float c1 = 2.0f * fmaf(0.5f, lnm, 1.0f) * hw_rcp(mf);
    float g[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float wt = fmaf(wx, tx[i], fmaf(wy, ty[i], wz * tz[i]));
        g[i] = fmaf(c1, wt, -lnm * rho[i]);
    }
    gx = g[0];
    gy = g[1];
    gz = g[2];
    return k;
}

}  // namespace frt
