// frt_adjoint.hip -- gradient of a batch render with respect to the fractal
// parameters (Julia c, Mandelbulb power n) and the cut planes, by implicit
// differentiation at the hit points.  One lane per pixel, FP64 arithmetic.
//
// The rendered depth of a refined hit is the root t* of
//   g(t, theta) = d(o + t dir; theta) - eps_abs - eps_rel t,
// so by the implicit function theorem
//   dt*/dtheta = -(dd/dtheta) / (grad d . dir - eps_rel).
// Both derivatives of d come out of one orbit evaluation that carries
// forward-mode tangents (the derivative of the orbit-derivative estimate of
// Sec. 2, Eq. 2-4, with respect to each parameter and to one spatial
// direction).  The normal taps of Eq. 5 / Listing 5 sit at
//   q_a = o + t* dir + k eps(t*) nu_a,
// which move with t*: dq_a/dt* = dir + k eps_rel nu_a, so each tap needs the
// parameter tangents plus one directional tangent along that vector.  The
// normal is the normalised tap sum and the colour Lambert's term of it, so
// their derivatives follow by the chain rule.  Cut-face hits have closed
// forms: t* = (d - n_hat . o) / (n_hat . dir) and normal n_hat, with
// n_hat = n / |n| for the raw plane normal n.  Exhausted and unrefined hits,
// misses and the shadow visibility contribute nothing (the visibility is
// piecewise constant).  Nothing from the forward orbits is stored: the
// kernel reads depth and status and recomputes.
//
// Work distribution: persistent waves claim 64-ray tiles (8x8 pixels of one
// job) from a counter in the workspace header, accumulate per-lane partial
// gradients while the job stays the same, and on a change of job reduce
// across the wave and add the 13 sums into the job's gradient with one
// atomic per slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "frt_fractal.hpp"
#include "frt_internal.hpp"
#include "frt_job.hpp"
#include "frt_ray.hpp"

namespace frt {

// All adjoint arithmetic is FP64.  The normal's parameter derivative is a
// difference of tap tangents of size O(1) taken over taps 2h ~ 1e-3 apart,
// so float32 tangents would lose ~1e-3 of relative accuracy to that
// cancellation alone; in FP64 the loss is ~1e-12.  The adjoint runs a few
// orbit evaluations per hit pixel (no march), and the CDNA4 FP64 vector rate
// equals the non-packed FP32 rate, so the cost stays a fraction of the
// forward pass.  The transcendentals are the device library's FP64 ones.

// ---------------------------------------------------------------------------
// Julia z^p + c (same loop as JuliaOrbit / JuliaDegOrbit) with NP + 1
// tangents: slots 0..NP-1 the constant c (z'_0 = 0, +e_s every body; NP = 4
// or 0), slot NP the spatial direction v (z'_0 = (v, 0)).  z^p comes from
// the recurrence on z^j = R_j + Q_j v (R_1 = a, Q_1 = 1,
// R_(j+1) = a R_j - |v|^2 Q_j, Q_(j+1) = R_j + a Q_j), differentiated term
// by term.  The running derivative product (p^2 |z|^(2(p-1)) per body)
// enters only through its logarithm, so its tangent is carried as
// L = d ln(dz2) = sum 2 (p-1) z.z'/|z|^2.  d = A S with A = 0.25 ln m2,
// S = sqrt(m2 / dz2):
//   d' = S (m2'/m2) (0.25 + 0.5 A) - 0.5 A S L.
// ---------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void julia_de_tan(const OrbitParams& P, double x, double y, double z, double vx,
                                             double vy, double vz, double& d, double (&dp)[NP > 0 ? NP : 1],
                                             double& dv) {
    constexpr int K = NP + 1;
    const double c0 = P.c0, c1 = P.c1, c2 = P.c2, c3 = P.c3;
    const int deg = P.ipow;
    const double lfac = 2.0 * (deg - 1);
    const double p2 = static_cast<double>(deg) * deg;
    double a = x, b = y, e = z, w = 0.0;
    double ta[K], tb[K], te[K], tw[K], L[K];
#pragma unroll
    for (int s = 0; s < NP; ++s) { ta[s] = tb[s] = te[s] = tw[s] = L[s] = 0.0; }
    ta[NP] = vx; tb[NP] = vy; te[NP] = vz; tw[NP] = 0.0; L[NP] = 0.0;
    double m2 = fma(a, a, fma(b, b, e * e));
    double prod = 1.0;
    for (int i = 0; i < P.max_iter; ++i) {
        const double im2 = m2 > 0.0 ? 1.0 / m2 : 0.0;
        const double vv = fma(b, b, fma(e, e, w * w));
        // primal z^p = R + Q v and |z|^(2(p-1))
        double R = a, Q = 1.0, mp = 1.0;
        for (int j = 1; j < deg; ++j) {
            const double nR = fma(a, R, -vv * Q);
            Q = fma(a, Q, R);
            R = nR;
            mp *= m2;
        }
        prod *= mp * p2;
        // tangents one slot at a time (the primal recurrence is rerun per
        // slot rather than holding every slot's (R', Q') at once)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const double dot = fma(a, ta[s], fma(b, tb[s], fma(e, te[s], w * tw[s])));
            L[s] = fma(lfac * dot, im2, L[s]);
            const double dvv = 2.0 * fma(b, tb[s], fma(e, te[s], w * tw[s]));
            double r = a, q = 1.0, dr = ta[s], dq = 0.0;
            for (int j = 1; j < deg; ++j) {
                const double ndr = fma(ta[s], r, fma(a, dr, -fma(dvv, q, vv * dq)));
                dq = fma(ta[s], q, fma(a, dq, dr));
                dr = ndr;
                const double nr = fma(a, r, -vv * q);
                q = fma(a, q, r);
                r = nr;
            }
            const double nb = fma(dq, b, Q * tb[s]);
            const double ne = fma(dq, e, Q * te[s]);
            const double nw = fma(dq, w, Q * tw[s]);
            ta[s] = dr + ((s < NP && s == 0) ? 1.0 : 0.0);
            tb[s] = nb + ((s < NP && s == 1) ? 1.0 : 0.0);
            te[s] = ne + ((s < NP && s == 2) ? 1.0 : 0.0);
            tw[s] = nw + ((s < NP && s == 3) ? 1.0 : 0.0);
        }
        a = R + c0;
        b = fma(Q, b, c1);
        e = fma(Q, e, c2);
        w = fma(Q, w, c3);
        m2 = fma(a, a, fma(b, b, fma(e, e, w * w)));
        if (m2 > P.bail2) break;
    }
    if (!(m2 > 0.0)) {
        d = 0.0;
#pragma unroll
        for (int s = 0; s < NP; ++s) dp[s] = 0.0;
        dv = 0.0;
        return;
    }
    const double dz2 = prod;
    const double S = sqrt(m2 / dz2);
    const double A = 0.25 * log(m2);
    d = A * S;
    const double c1s = S * fma(0.5, A, 0.25) / m2;
    const double c2s = 0.5 * A * S;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const double m2p = 2.0 * fma(a, ta[s], fma(b, tb[s], fma(e, te[s], w * tw[s])));
        const double o = fma(c1s, m2p, -c2s * L[s]);
        if (s < NP) dp[s] = o; else dv = o;
    }
}

// ---------------------------------------------------------------------------
// Mandelbulb (Listing 7 with real n, same axes as BulbOrbit) with two
// tangents: slot 0 the power n, slot 1 the spatial direction v (the point p
// is also the additive constant, so p' = v is added every body).  With
// r = |w|, rho = |(x, z)|, theta = atan2(rho, y) (= acos(y / r), better
// conditioned near the polar axis), phi = atan2(x, z), B = n theta, A = n phi:
//   w <- r^n (sin B sin A, cos B, sin B cos A) + p,  dr <- n r^(n-1) dr + 1,
// differentiated term by term (theta' = (y rho' - rho y') / r^2,
// phi' = (z x' - x z') / rho^2); d = 0.25 ln m sqrt(m) / dr with m = |w|^2:
//   d' = (sqrt(m) / dr) (m'/m) (0.25 + 0.5 * 0.25 ln m) - d dr'/dr.
// The integer powers use the same trigonometric form here: it is the same
// function of (p, n), and its n-derivative needs the angles anyway.
// ---------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void bulb_de_tan(const OrbitParams& P, double x, double y, double z, double vx,
                                            double vy, double vz, double& d, double (&dp)[NP > 0 ? NP : 1],
                                            double& dv) {
    constexpr int K = NP + 1;   // slot 0 the power (if NP = 1), slot NP the direction
    const double n = P.n;
    double wx = x, wy = y, wz = z;
    double tx[K], ty[K], tz[K], px[K], py[K], pz[K], tdr[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const bool sp = s == NP;
        px[s] = sp ? vx : 0.0;
        py[s] = sp ? vy : 0.0;
        pz[s] = sp ? vz : 0.0;
        tx[s] = px[s]; ty[s] = py[s]; tz[s] = pz[s];
        tdr[s] = 0.0;
    }
    double m = fma(wx, wx, fma(wy, wy, wz * wz));
    double dr = 1.0;
    for (int i = 0; i < P.max_iter; ++i) {
        if (m == 0.0) {
            wx = x; wy = y; wz = z;
            dr = 1.0;
#pragma unroll
            for (int s = 0; s < K; ++s) { tx[s] = px[s]; ty[s] = py[s]; tz[s] = pz[s]; tdr[s] = 0.0; }
        } else {
            const double lr = 0.5 * log(m);                  // ln r
            const double rn1 = exp((n - 1.0) * lr);          // r^(n-1)
            const double r = sqrt(m);
            const double rinv = 1.0 / r;
            const double rho2 = fma(wx, wx, wz * wz);
            const double rho = sqrt(rho2);
            const double th = atan2(rho, wy);
            const double ph = atan2(wx, wz);
            double sb, cb, sa, ca;
            sincos(n * th, &sb, &cb);
            sincos(n * ph, &sa, &ca);
            const double rn = rn1 * r;
            const double irho = rho > 0.0 ? 1.0 / rho : 0.0;
            const double irho2 = irho * irho;
            const double im = 1.0 / m;
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const double np = s < NP ? 1.0 : 0.0;
                const double rp = fma(wx, tx[s], fma(wy, ty[s], wz * tz[s])) * rinv;
                const double rn1p = rn1 * fma(np, lr, (n - 1.0) * rp * rinv);
                tdr[s] = fma(np * rn1, dr, n * fma(rn1p, dr, rn1 * tdr[s]));
                const double rhop = fma(wx, tx[s], wz * tz[s]) * irho;
                const double thp = fma(wy, rhop, -rho * ty[s]) * im;
                const double php = fma(wz, tx[s], -wx * tz[s]) * irho2;
                const double Bp = fma(np, th, n * thp);
                const double Ap = fma(np, ph, n * php);
                const double rnp = fma(rn1p, r, rn1 * rp);
                const double ntx = fma(rnp, sb * sa, rn * fma(cb * Bp, sa, sb * ca * Ap)) + px[s];
                const double nty = fma(rnp, cb, -rn * sb * Bp) + py[s];
                const double ntz = fma(rnp, sb * ca, rn * fma(cb * Bp, ca, -sb * sa * Ap)) + pz[s];
                tx[s] = ntx; ty[s] = nty; tz[s] = ntz;
            }
            dr = fma(n * rn1, dr, 1.0);
            const double rsb = rn * sb;
            wx = fma(rsb, sa, x);
            wy = fma(rn, cb, y);
            wz = fma(rsb, ca, z);
        }
        m = fma(wx, wx, fma(wy, wy, wz * wz));
        if (m > P.bail2) break;
    }
    if (!(m > 0.0)) {
        d = 0.0;
#pragma unroll
        for (int s = 0; s < NP; ++s) dp[s] = 0.0;
        dv = 0.0;
        return;
    }
    const double sq = sqrt(m);
    const double A = 0.25 * log(m);
    d = A * sq / dr;
    const double c1s = sq / dr * fma(0.5, A, 0.25) / m;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const double mp = 2.0 * fma(wx, tx[s], fma(wy, ty[s], wz * tz[s]));
        const double o = fma(c1s, mp, -d * tdr[s] / dr);
        if (s < NP) dp[s] = o; else dv = o;
    }
}

// Estimate with the tangents of kind KIND: NP parameter slots (Julia 4 / 0,
// Mandelbulb 1 / 0) plus the direction (vx, vy, vz).
template <int KIND, int NP>
__device__ __forceinline__ void de_tan(const OrbitParams& P, double x, double y, double z, double vx, double vy,
                                       double vz, double& d, double (&dp)[NP > 0 ? NP : 1], double& dv) {
    if constexpr (KIND == kJulia) julia_de_tan<NP>(P, x, y, z, vx, vy, vz, d, dp, dv);
    else bulb_de_tan<NP>(P, x, y, z, vx, vy, vz, d, dp, dv);
}

// Upstream weights of one pixel: w = g_normal + [lit] k_d (g_colour . albedo) L
// (the derivative of the colour is albedo k_d (L . N') where N . L > 0).
__device__ __forceinline__ void normal_weights(const JobDev& J, const AdjointJob& A, long long p, long long NP,
                                               bool lit, double nx, double ny, double nz, double (&w)[3]) {
    w[0] = w[1] = w[2] = 0.0;
    if (A.g_normal) {
        w[0] = A.g_normal[p];
        w[1] = A.g_normal[NP + p];
        w[2] = A.g_normal[2 * NP + p];
    }
    if (A.g_colour && lit) {
        const double ndl = fma(nx, double(J.light[0]), fma(ny, double(J.light[1]), nz * J.light[2]));
        if (ndl > 0.0) {
            const double gca = fma(double(A.g_colour[p]), J.albedo[0],
                                   fma(double(A.g_colour[NP + p]), J.albedo[1],
                                       double(A.g_colour[2 * NP + p]) * J.albedo[2]));
            const double k = J.k_d * gca;
            w[0] = fma(k, double(J.light[0]), w[0]);
            w[1] = fma(k, double(J.light[1]), w[1]);
            w[2] = fma(k, double(J.light[2]), w[2]);
        }
    }
}

// Contribution of one refined surface hit to the NPAR parameter slots.  The
// ray is rebuilt in FP64 from the FP64 camera basis, and the float32 depth
// is polished by one FP64 Newton step on g(t) = d - eps_abs - eps_rel t
// (skipped when the step would exceed eps/8 or the crossing is not
// descending), so that the derivatives are those at the root itself rather
// than at its float32 rounding -- on fine detail the derivatives of the
// normal change measurably over 1e-7.
template <int KIND, int NPAR>
__device__ __forceinline__ void surface_hit_grad(const JobDev& J, const AdjointJob& A, const OrbitParams& P,
                                                 long long p, long long NP, bool lit, int px, int py, float tsf,
                                                 float gdf, float (&acc)[NPAR]) {
    double dx, dy, dz;
    primary_dir_f64(J, px, py, dx, dy, dz);
    const double gd = gdf;
    const double er = J.eps_rel, ea = J.eps_abs;
    const double ox = J.eye[0], oy = J.eye[1], oz = J.eye[2];
    double ts = tsf;
    {
        double dn, dpn[1], dvn;
        de_tan<KIND, 0>(P, fma(ts, dx, ox), fma(ts, dy, oy), fma(ts, dz, oz), dx, dy, dz, dn, dpn, dvn);
        const double gt = dvn - er;
        const double step = (dn - fma(er, ts, ea)) / gt;
        if (gt < 0.0 && fabs(step) <= 0.125 * fma(er, ts, ea)) ts -= step;
    }
    const double sx = fma(ts, dx, ox), sy = fma(ts, dy, oy), sz = fma(ts, dz, oz);
    double d0, dp0[NPAR], dv0;
    de_tan<KIND, NPAR>(P, sx, sy, sz, dx, dy, dz, d0, dp0, dv0);
    const double den = dv0 - er;
    if (!(den != 0.0)) return;
    const double iden = -1.0 / den;
    double dT[NPAR];
#pragma unroll
    for (int s = 0; s < NPAR; ++s) dT[s] = dp0[s] * iden;

    // taps around p* moving with t*
    const double eps = fma(er, ts, ea);
    double G[3] = {0.0, 0.0, 0.0};
    double dG[NPAR][3];
#pragma unroll
    for (int s = 0; s < NPAR; ++s) dG[s][0] = dG[s][1] = dG[s][2] = 0.0;
    const int taps = J.normal_mode == 0 ? 4 : 6;
    const double ks = J.normal_mode == 0 ? double(0.5773f) : 1.0;
    const double h = ks * eps;
    const double hr = ks * er;
    for (int k = 0; k < taps; ++k) {
        double nu[3];
        if (J.normal_mode == 0) {
            nu[0] = (k == 0 || k == 3) ? 1.0 : -1.0;
            nu[1] = (k >= 2) ? 1.0 : -1.0;
            nu[2] = (k == 1 || k == 3) ? 1.0 : -1.0;
        } else {
            const double sg = (k & 1) ? -1.0 : 1.0;
            const int ax = k >> 1;
            nu[0] = ax == 0 ? sg : 0.0;
            nu[1] = ax == 1 ? sg : 0.0;
            nu[2] = ax == 2 ? sg : 0.0;
        }
        double da, dpa[NPAR], dva;
        de_tan<KIND, NPAR>(P, fma(h, nu[0], sx), fma(h, nu[1], sy), fma(h, nu[2], sz), fma(hr, nu[0], dx),
                     fma(hr, nu[1], dy), fma(hr, nu[2], dz), da, dpa, dva);
        // Eq. 5 weights: tetrahedral nu_a, central +-e_k (the same signs)
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c] = fma(nu[c], da, G[c]);
#pragma unroll
        for (int s = 0; s < NPAR; ++s) {
            const double Da = fma(dva, dT[s], dpa[s]);
#pragma unroll
            for (int c = 0; c < 3; ++c) dG[s][c] = fma(nu[c], Da, dG[s][c]);
        }
    }
    const double gl2 = fma(G[0], G[0], fma(G[1], G[1], G[2] * G[2]));
    double w[3] = {0.0, 0.0, 0.0};
    double inv = 0.0, N[3] = {0.0, 0.0, 0.0};
    if (gl2 > 0.0) {   // else the forward normal is -dir, a constant
        inv = 1.0 / sqrt(gl2);
        N[0] = G[0] * inv;
        N[1] = G[1] * inv;
        N[2] = G[2] * inv;
        normal_weights(J, A, p, NP, lit, N[0], N[1], N[2], w);
    }
    // dN = (dG - N (N . dG)) / |G|, contribution w . dN
    const double wn = fma(w[0], N[0], fma(w[1], N[1], w[2] * N[2]));
#pragma unroll
    for (int s = 0; s < NPAR; ++s) {
        const double wdg = fma(w[0], dG[s][0], fma(w[1], dG[s][1], w[2] * dG[s][2]));
        const double ndg = fma(N[0], dG[s][0], fma(N[1], dG[s][1], N[2] * dG[s][2]));
        const double vn = (wdg - wn * ndg) * inv;
        acc[s] += static_cast<float>(fma(gd, dT[s], vn));
    }
}

// Contribution of one cut-face hit to the 4 slots of its entry plane (raw
// normal n xyz, offset d; the plane is n_hat . x = d).  With q = o + t* dir
// the hit point:
//   dt/dn = -(I - n_hat n_hat^T) q / (|n| n_hat . dir),  dt/dd = 1 / (n_hat . dir),
//   dN/dn = (I - n_hat n_hat^T) / |n|,  dN/dd = 0.
__device__ __forceinline__ void cut_face_grad(const JobDev& J, const AdjointJob& A, long long p, long long NP,
                                              bool lit, int e, int px, int py, float gdf, float (&acc)[4]) {
    double dx, dy, dz;
    primary_dir_f64(J, px, py, dx, dy, dz);
    const double gd = gdf;
    const double rx = A.raw_n[e][0], ry = A.raw_n[e][1], rz = A.raw_n[e][2];
    const double ilen = 1.0 / sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
    const double nx = rx * ilen, ny = ry * ilen, nz = rz * ilen;
    const double nd = fma(nx, dx, fma(ny, dy, nz * dz));
    if (!(nd != 0.0)) return;
    const double ind = 1.0 / nd;
    const double ox = J.eye[0], oy = J.eye[1], oz = J.eye[2];
    const double ts = (double(J.pd[e]) - fma(nx, ox, fma(ny, oy, nz * oz))) * ind;   // exact crossing
    const double qx = fma(ts, dx, ox), qy = fma(ts, dy, oy), qz = fma(ts, dz, oz);
    const double nq = fma(nx, qx, fma(ny, qy, nz * qz));
    double w[3];
    normal_weights(J, A, p, NP, lit, nx, ny, nz, w);
    const double wn = fma(w[0], nx, fma(w[1], ny, w[2] * nz));
    const double kt = -gd * ilen * ind;
    acc[0] += static_cast<float>(fma(kt, qx - nq * nx, (w[0] - wn * nx) * ilen));
    acc[1] += static_cast<float>(fma(kt, qy - nq * ny, (w[1] - wn * ny) * ilen));
    acc[2] += static_cast<float>(fma(kt, qz - nq * nz, (w[2] - wn * nz) * ilen));
    acc[3] += static_cast<float>(gd * ind);
}

// A pixel whose tangents overflowed (an orbit that grows without escaping
// within the iteration budget) contributes nothing rather than a NaN/inf
// that would swamp its job's whole gradient.
template <int K>
__device__ __forceinline__ void drop_nonfinite(float (&v)[K]) {
    bool ok = true;
#pragma unroll
    for (int s = 0; s < K; ++s) ok = ok && isfinite(v[s]);
    if (!ok) {
#pragma unroll
        for (int s = 0; s < K; ++s) v[s] = 0.0f;
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce the wave's partial gradients for job j and add them to its outputs.
// j: the job's index in the caller's arrays
__device__ __forceinline__ void flush(const AdjointArgs& a, int j, float (&acc)[kGradSlots]) {
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int s = 0; s < kGradSlots; ++s) {
        const float v = wave_sum(acc[s]);
        acc[s] = 0.0f;
        if (lead && v != 0.0f) {
            float* dst = s < 4 ? a.grad_c + 4ll * j + s : (s == 4 ? a.grad_power + j : a.grad_plane + 8ll * j + (s - 5));
            unsafeAtomicAdd(dst, v);
        }
    }
}

// Tiles per claim of the adjoint's counter.
constexpr unsigned kAdjTiles = 4;

// The surface-hit gradient of one queued pixel of job J (its index in the
// job's planes); adds into acc and writes the per-pixel slots of its kind.
template <int KIND>
__device__ __forceinline__ void surface_item(const JobDev& J, const AdjointJob& A, long long p,
                                             float (&acc)[kGradSlots]) {
    const long long NP = J.npix;
    const int py = static_cast<int>(p / J.width), px = static_cast<int>(p - static_cast<long long>(py) * J.width);
    const bool lit = !(J.status[p] & kFlagShadowed);
    const float gd = A.g_depth ? A.g_depth[p] : 0.0f;
    const OrbitParams P = orbit_params(J);
    if constexpr (KIND == kJulia) {
        float pa[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        surface_hit_grad<kJulia, 4>(J, A, P, p, NP, lit, px, py, J.depth[p], gd, pa);
        drop_nonfinite(pa);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s] += pa[s];
        if (A.g_pixel) {
            for (int s = 0; s < 4; ++s) A.g_pixel[s * NP + p] = pa[s];
        }
    } else {
        float pa[1] = {0.0f};
        surface_hit_grad<kBulb, 1>(J, A, P, p, NP, lit, px, py, J.depth[p], gd, pa);
        drop_nonfinite(pa);
        acc[4] += pa[0];
        if (A.g_pixel) A.g_pixel[4 * NP + p] = pa[0];
    }
}

// One instantiation per fractal kind (the two tangent sets differ in size);
// each drains the 64-ray tiles of its kind's jobs, [range[KIND][0],
// range[KIND][1]) of the ray index space, kAdjTiles at a time.  A wave's
// first group is the one of its index in the grid; the kind's counter hands
// out the groups after the grid's first n_waves (one address serves about 80
// device-scope atomics per microsecond, so a claim per tile, and all waves
// claiming at the start, would queue on it).  A tile lies inside one job,
// found through the wave's job cursor.
//
// A tile's cut-face pixels take their closed form at once.  Its surface hits,
// the FP64 orbit with tangents that holds most of the work, are queued in a
// per-wave LDS list instead and evaluated 64 at a time, one per lane, so
// misses and background pixels do not idle lanes through that work.  The
// list holds one job's pixels: it is drained when the job changes (and at
// the end), before the job's partial sums are flushed.
template <int KIND>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjointArgs a, WorkspaceHeader* __restrict__ hdr) {
    const unsigned long long r0 = hdr->range[KIND][0];
    const unsigned long long tiles = (hdr->range[KIND][1] - r0) >> 6;
    const int n_jobs = a.n_jobs;
    const int lane = threadIdx.x & 63;
    float acc[kGradSlots];
#pragma unroll
    for (int s = 0; s < kGradSlots; ++s) acc[s] = 0.0f;
    int cur = -1;   // caller's index of the job the partial sums belong to (uniform across the wave)
    int qj = -1;    // table index of the queued pixels' job (uniform)
    int qn = 0;     // queued surface hits (uniform, < 64 between tiles)
    __shared__ int queue_lds[4][128];
    int* q = queue_lds[threadIdx.x >> 6];
    // evaluate the first n (<= 64) queued pixels, then move the rest down
    auto drain = [&](int n) {
        const JobDev& J = a.jobs[qj];
        const AdjointJob& A = a.ajobs[qj];
        if (!FRT_CHECK(hdr, n >= 1 && n <= 64 && n <= qn && qn < 128, kCheckList)) {
            qn = 0;   // a list out of its bounds: dropped
            return;
        }
        const int item = lane < n ? q[lane] : 0;
        const int rest = qn - n;   // < 64
        const int moved = lane < rest ? q[n + lane] : 0;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) q[lane] = moved;
        __builtin_amdgcn_wave_barrier();
        qn = rest;
        if (lane < n && FRT_CHECK(hdr, item >= 0 && item < J.npix, kCheckPixel)) surface_item<KIND>(J, A, item, acc);
    };
    JobCursor jc;
    const unsigned long long n_waves = static_cast<unsigned long long>(gridDim.x) * (blockDim.x >> 6);
    unsigned long long grp =
        static_cast<unsigned long long>(blockIdx.x) * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (bool first = true;; first = false) {
        if (!first) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(&hdr->adj_queue[KIND], 1ull);
            grp = n_waves + bcast_first(c);
        }
        const unsigned long long t0 = grp * kAdjTiles;
        if (t0 >= tiles) break;
        const unsigned long long t1 = min(t0 + kAdjTiles, tiles);
        for (unsigned long long t = t0; t < t1; ++t) {
            const unsigned long long g0 = r0 + (t << 6);
            job_seek<true>(a.jobs, a.jobs[0], n_jobs, g0, jc);
            if (!FRT_CHECK(hdr, jc.j >= 0 && jc.j < n_jobs, kCheckJob) ||
                !FRT_CHECK(hdr, g0 >= jc.begin && g0 + 64ull <= jc.end, kCheckRay)) continue;
            const int j = jc.j;
            if (j != qj) {
                while (qn > 0) drain(min(qn, 64));
                qj = j;
            }
            const JobDev& J = a.jobs[j];
            const AdjointJob& A = a.ajobs[j];
            if (A.out_index != cur) {
                if (cur >= 0) flush(a, cur, acc);
                cur = A.out_index;
            }
            int px, py;
            const bool in = tile_pixel(J, static_cast<long long>(g0 - jc.begin) + lane, px, py);
            const long long NP = J.npix;
            const long long p = static_cast<long long>(py) * J.width + px;
            bool surf = false;
            if (in && FRT_CHECK(hdr, p >= 0 && p < NP, kCheckPixel)) {
                const int st = J.status[p];
                const int cls = st & 7;
                const bool smooth = cls == kHitCut || (cls == kHit && !(st & kFlagUnrefined));
                bool any = false;
                if (smooth) {
                    any = A.g_depth && A.g_depth[p] != 0.0f;
                    if (A.g_colour) any = any || A.g_colour[p] != 0.0f || A.g_colour[NP + p] != 0.0f || A.g_colour[2 * NP + p] != 0.0f;
                    if (A.g_normal) any = any || A.g_normal[p] != 0.0f || A.g_normal[NP + p] != 0.0f || A.g_normal[2 * NP + p] != 0.0f;
                }
                surf = smooth && any && cls == kHit;
                if (A.g_pixel) {
                    // a queued pixel writes its own kind's slots later
                    for (int s = 0; s < kGradSlots; ++s) {
                        const bool own = KIND == kJulia ? s < 4 : s == 4;
                        if (!(surf && own)) A.g_pixel[s * NP + p] = 0.0f;
                    }
                }
                if (smooth && any && cls == kHitCut) {
                    // entry plane as the forward pass found it (float32 ray)
                    const bool lit = !(st & kFlagShadowed);
                    const float gd = A.g_depth ? A.g_depth[p] : 0.0f;
                    float dx, dy, dz;
                    primary_dir(J, px, py, dx, dy, dz);
                    float lo, hi;
                    int e;
                    const bool ok = ray_interval(J, J.eye[0], J.eye[1], J.eye[2], dx, dy, dz, J.eps_abs, lo, hi, e);
                    if (ok && e >= 0) {
                        float pa[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                        cut_face_grad(J, A, p, NP, lit, e, px, py, gd, pa);
                        drop_nonfinite(pa);
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            if (e == 0) acc[5 + s] += pa[s]; else acc[9 + s] += pa[s];
                        }
                        if (A.g_pixel) {
                            for (int s = 0; s < 4; ++s) A.g_pixel[(5 + 4 * e + s) * NP + p] = pa[s];
                        }
                    }
                }
            }
            // append this tile's surface hits to the queue
            const unsigned long long m = __ballot(surf);
            if (surf && FRT_CHECK(hdr, qn + static_cast<int>(lane_rank(m)) < 128, kCheckList))
                q[qn + static_cast<int>(lane_rank(m))] = static_cast<int>(p);
            __builtin_amdgcn_wave_barrier();
            qn += __popcll(m);
            if (qn >= 64) drain(64);
        }
    }
    while (qn > 0) drain(min(qn, 64));
    if (cur >= 0) flush(a, cur, acc);
}

__global__ void adjoint_reset_kernel(AdjointArgs a, WorkspaceHeader* __restrict__ hdr) {
    const long long n = a.n_jobs;
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < 8 * n;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        a.grad_plane[i] = 0.0f;
        if (i < 4 * n) a.grad_c[i] = 0.0f;
        if (i < n) a.grad_power[i] = 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) hdr->adj_queue[threadIdx.x] = 0ull;
}

hipError_t launch_adjoint(const AdjointArgs& a, WorkspaceHeader* hdr, hipStream_t stream) {
    const long long n8 = 8ll * a.n_jobs;
    const int rgrid = static_cast<int>(std::min<long long>((n8 + 255) / 256, 1024));
    hipLaunchKernelGGL(adjoint_reset_kernel, dim3(rgrid), dim3(256), 0, stream, a, hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.grid[kJulia] > 0) {
        hipLaunchKernelGGL(adjoint_kernel<kJulia>, dim3(a.grid[kJulia]), dim3(256), 0, stream, a, hdr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.grid[kBulb] > 0) {
        hipLaunchKernelGGL(adjoint_kernel<kBulb>, dim3(a.grid[kBulb]), dim3(256), 0, stream, a, hdr);
        e = hipGetLastError();
    }
    return e;
}

const void* adjoint_kernel_symbol(int kind) {
    return kind == kJulia ? reinterpret_cast<const void*>(&adjoint_kernel<kJulia>)
                          : reinterpret_cast<const void*>(&adjoint_kernel<kBulb>);
}

}  // namespace frt
