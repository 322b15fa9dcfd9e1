// frt_scene.hip -- scenes of several fractal objects in one launch (Sec. 3:
// each procedural object sits in its own box with a world-to-local
// transform; the intersection shader marches the ray in local space and the
// closest hit is kept, its normal mapped back to world space).
//
// Object k maps world points by the similarity x_obj = R_k^T (x - T_k) / s_k.
// A world ray o + t dir becomes o_k + (t / s_k) dir_k with dir_k = R_k^T dir,
// and s_k d_k(x_obj) bounds the world distance, so the march runs in object
// units with eps_abs / s_k, eps_rel, step_clamp / s_k and t_max / s_k (the
// host scales them) and reports world depth s_k t_obj.  Normals map back as
// R_k n_obj.
//
// One lane per pixel (8x8 tiles, one wave a tile).  Each lane marches every
// object in index order with the same rules as the persistent march kernel
// (interval, cut face, Listing 3, bisection to eps/32 and a secant step),
// capping an object's range at the best world depth so far plus one full
// step, so a later object can only replace the hit with a closer one (ties
// keep the lower index).  The hit is shaded in world space; its shadow ray
// is blocked by a hit on any object.  With the closest-hit shading model a
// white Phong highlight is added, and one reflection ray, traced against
// every object with the threshold carried on from eps(t*), adds its hit's
// Lambert and highlight terms weighted by Schlick's Fresnel term
// (f0 = albedo); there a trap palette colours each hit's albedo by the
// orbit trap of its point.  The orbit trap at the hit point is written on
// request.
#include <hip/hip_runtime.h>

#include "frt_internal.hpp"
#include "frt_job.hpp"
#include "frt_normal.hpp"
#include "frt_ray.hpp"

namespace frt {

namespace {

constexpr float kSceneRefineTol = 1.0f / 32.0f;   // same bracket width as the march kernel

struct MarchOut {
    int status;      // class and flags
    float t;         // object-space depth
    int steps;
    int hit_it;
    int entry;       // cut-face plane
    unsigned evals;
    unsigned bodies;
    bool entered;    // the search interval was not empty
};

// One ray through one object in its own frame.  ea, er: the stop threshold
// eps(t) = ea + er t; tmin: interval start; cap: upper bound on t besides
// the object's own t_max; shadow: stop at the first sample under eps.
template <int VAR>
__device__ MarchOut march_object(const JobDev& J, const OrbitParams& P, float ox, float oy, float oz, float dx,
                                 float dy, float dz, float tmin, float cap, float ea, float er, bool shadow) {
    using Orbit = typename OrbitOf<VAR>::T;
    MarchOut r{kMissBounds, -1.0f, 0, 0, -1, 0u, 0u, false};
    float lo, hi;
    int entry;
    if (!ray_interval(J, ox, oy, oz, dx, dy, dz, tmin, lo, hi, entry)) return r;
    r.entered = true;
    hi = fminf(hi, cap);
    if (lo > hi) {
        r.status = kMissTmax;
        return r;
    }
    Orbit orb;
    float t = lo;
    DEResult de = de_once(orb, P, fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz));
    r.evals = 1u;
    r.bodies = static_cast<unsigned>(de.bodies);
    if (entry >= 0 && (de.it == P.max_iter || de.d < fmaf(er, t, ea))) {
        r.status = kHitCut;
        r.t = t;
        r.hit_it = de.it;
        r.entry = entry;
        return r;
    }
    float lt = t, lh = 0.0f;
    for (;;) {
        ++r.steps;
        r.hit_it = de.it;
        if (de.d < fmaf(er, t, ea)) {
            if (shadow || r.steps == 1) {
                r.status = shadow ? kHit : (kHit | kFlagUnrefined);
                r.t = t;
                return r;
            }
            // refine the root of g = d - eps on [lt, t], g(lt) >= 0 > g(t)
            float t1 = t, gb = de.d - fmaf(er, t, ea);
            lh -= fmaf(er, lt, ea);
            int rk = 0;
            while (rk < J.refine_iters && t1 - lt > kSceneRefineTol * fmaf(er, t1, ea)) {
                const float tm = 0.5f * (lt + t1);
                de = de_once(orb, P, fmaf(tm, dx, ox), fmaf(tm, dy, oy), fmaf(tm, dz, oz));
                r.evals += 1u;
                r.bodies += static_cast<unsigned>(de.bodies);
                const float fx = de.d - fmaf(er, tm, ea);
                if (fx < 0.0f) {
                    t1 = tm;
                    gb = fx;
                } else {
                    lt = tm;
                    lh = fx;
                }
                ++rk;
            }
            r.status = kHit;
            r.t = fmaf(-gb, __fdividef(t1 - lt, gb - lh), t1);
            return r;
        }
        lt = t;
        lh = de.d;
        t += fminf(de.d, J.clamp);
        if (t > hi) {
            r.status = kMissTmax;
            return r;
        }
        if (r.steps >= J.max_steps) {
            r.status = kHitExhausted | kFlagUnrefined;
            r.t = t;
            return r;
        }
        de = de_once(orb, P, fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz));
        r.evals += 1u;
        r.bodies += static_cast<unsigned>(de.bodies);
    }
}

__device__ MarchOut march_any(int variant, const JobDev& J, const OrbitParams& P, float ox, float oy, float oz,
                              float dx, float dy, float dz, float tmin, float cap, float ea, float er, bool shadow) {
    switch (variant) {
        case kVarJulia: return march_object<kVarJulia>(J, P, ox, oy, oz, dx, dy, dz, tmin, cap, ea, er, shadow);
        case kVarBulbReal: return march_object<kVarBulbReal>(J, P, ox, oy, oz, dx, dy, dz, tmin, cap, ea, er, shadow);
        case kVarBulbInt: return march_object<kVarBulbInt>(J, P, ox, oy, oz, dx, dy, dz, tmin, cap, ea, er, shadow);
        case kVarBulb8: return march_object<kVarBulb8>(J, P, ox, oy, oz, dx, dy, dz, tmin, cap, ea, er, shadow);
        default: return march_object<kVarJuliaDeg>(J, P, ox, oy, oz, dx, dy, dz, tmin, cap, ea, er, shadow);
    }
}

__device__ void normal_any(int variant, const OrbitParams& P, int mode, float x, float y, float z, float eps,
                           float& gx, float& gy, float& gz, unsigned& evals, unsigned& bodies) {
    switch (variant) {
        case kVarJulia: estimate_normal<kVarJulia>(P, mode, x, y, z, eps, gx, gy, gz, evals, bodies); break;
        case kVarBulbReal: estimate_normal<kVarBulbReal>(P, mode, x, y, z, eps, gx, gy, gz, evals, bodies); break;
        case kVarBulbInt: estimate_normal<kVarBulbInt>(P, mode, x, y, z, eps, gx, gy, gz, evals, bodies); break;
        case kVarBulb8: estimate_normal<kVarBulb8>(P, mode, x, y, z, eps, gx, gy, gz, evals, bodies); break;
        default: estimate_normal<kVarJuliaDeg>(P, mode, x, y, z, eps, gx, gy, gz, evals, bodies); break;
    }
}

__device__ void trap_any(int variant, const OrbitParams& P, float x, float y, float z, float (&tr)[4]) {
    switch (variant) {
        case kVarJulia: orbit_trap<kVarJulia>(P, x, y, z, tr); break;
        case kVarBulbReal: orbit_trap<kVarBulbReal>(P, x, y, z, tr); break;
        case kVarBulbInt: orbit_trap<kVarBulbInt>(P, x, y, z, tr); break;
        case kVarBulb8: orbit_trap<kVarBulb8>(P, x, y, z, tr); break;
        default: orbit_trap<kVarJuliaDeg>(P, x, y, z, tr); break;
    }
}

// Phong highlight max(0, R.V)^shininess, R = 2 (N.L) N - L; 0 when N.L <= 0
__device__ __forceinline__ float phong_spec(float nx, float ny, float nz, const float* L, float vx, float vy, float vz,
                                            float ndl, float shininess) {
    if (!(ndl > 0.0f)) return 0.0f;
    const float rx = fmaf(2.0f * ndl, nx, -L[0]);
    const float ry = fmaf(2.0f * ndl, ny, -L[1]);
    const float rz = fmaf(2.0f * ndl, nz, -L[2]);
    const float rv = fmaf(rx, vx, fmaf(ry, vy, rz * vz));
    return rv > 0.0f ? hw_exp2(shininess * hw_log2(rv)) : 0.0f;
}

// Trap colouring of the closest-hit model: albedo_c + sum_k pal[k][c] T_k,
// clamped to [0, 1].
__device__ __forceinline__ void trap_albedo(const JobDev& cam, const float (&tr)[4], float (&alb)[3]) {
    for (int c = 0; c < 3; ++c) {
        float a = cam.albedo[c];
        for (int k = 0; k < 4; ++k) a = fmaf(cam.trap_pal[k][c], tr[k], a);
        alb[c] = fminf(fmaxf(a, 0.0f), 1.0f);
    }
}

// world point / direction -> object frame (x_obj = R^T (x - T) / s; directions R^T d)
__device__ __forceinline__ void to_object(const SceneObject& S, float x, float y, float z, bool point, float& ox,
                                          float& oy, float& oz) {
    if (point) {
        x -= S.trans[0];
        y -= S.trans[1];
        z -= S.trans[2];
    }
    const float* R = S.rot;
    float a = fmaf(R[0], x, fmaf(R[3], y, R[6] * z));
    float b = fmaf(R[1], x, fmaf(R[4], y, R[7] * z));
    float c = fmaf(R[2], x, fmaf(R[5], y, R[8] * z));
    if (point) {
        a *= S.inv_scale;
        b *= S.inv_scale;
        c *= S.inv_scale;
    }
    ox = a;
    oy = b;
    oz = c;
}

}  // namespace

__global__ void __launch_bounds__(256) scene_kernel(const SceneObject* __restrict__ objs, int n_obj,
                                                    const JobDev cam, int* __restrict__ object_id,
                                                    float* __restrict__ trap) {
    const long long g = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    int j, px, py;
    if (!ray_pixel<false>(nullptr, cam, 1, g, j, px, py)) return;
    const int p = py * cam.width + px;
    const long long NP = cam.npix;
    float dx, dy, dz;
    primary_dir(cam, px, py, dx, dy, dz);
    const float ex = cam.eye[0], ey = cam.eye[1], ez = cam.eye[2];

    // closest hit over the objects
    int best = -1;
    MarchOut hit{kMissBounds, -1.0f, 0, 0, -1, 0u, 0u, false};
    float best_tw = 0.0f;
    bool entered = false;
    float bdx = 0.f, bdy = 0.f, bdz = 0.f, box = 0.f, boy = 0.f, boz = 0.f;
    for (int k = 0; k < n_obj; ++k) {
        const SceneObject& S = objs[k];
        const JobDev& J = S.job;
        const OrbitParams P = orbit_params(J);
        float oox, ooy, ooz, odx, ody, odz;
        to_object(S, ex, ey, ez, true, oox, ooy, ooz);
        to_object(S, dx, dy, dz, false, odx, ody, odz);
        const float cap = best >= 0 ? fmaf(best_tw, S.inv_scale, J.clamp) : J.t_max;
        const MarchOut r = march_any(S.variant, J, P, oox, ooy, ooz, odx, ody, odz, J.eps_abs, cap, J.eps_abs,
                                     J.eps_rel, false);
        entered = entered || r.entered;
        if ((r.status & 7) >= kHit) {
            const float tw = r.t * S.scale;
            if (best < 0 || tw < best_tw) {
                best = k;
                best_tw = tw;
                hit = r;
                box = oox; boy = ooy; boz = ooz;
                bdx = odx; bdy = ody; bdz = odz;
            }
        }
    }
    if (object_id) object_id[p] = best;
    if (best < 0) {
        cam.depth[p] = -1.0f;
        for (int c = 0; c < 3; ++c) {
            cam.normal[c * NP + p] = 0.0f;
            cam.colour[c * NP + p] = 0.0f;
        }
        cam.status[p] = static_cast<uint8_t>(entered ? kMissTmax : kMissBounds);
        if (cam.counters)
            for (int c = 0; c < kCounterPlanes; ++c) cam.counters[c * NP + p] = 0u;
        if (trap)
            for (int c = 0; c < 4; ++c) trap[c * NP + p] = 0.0f;
        return;
    }

    // normal in the object's frame, mapped back by R
    const SceneObject& S = objs[best];
    const JobDev& J = S.job;
    float nox, noy, noz;
    unsigned nev = 0, nbo = 0;
    if ((hit.status & 7) == kHitCut) {
        nox = J.pn[hit.entry][0];
        noy = J.pn[hit.entry][1];
        noz = J.pn[hit.entry][2];
    } else {
        const OrbitParams P = orbit_params(J);
        const float ts = hit.t;
        const float eps = fmaf(J.eps_rel, ts, J.eps_abs);
        float gx, gy, gz;
        normal_any(S.variant, P, J.normal_mode, fmaf(ts, bdx, box), fmaf(ts, bdy, boy), fmaf(ts, bdz, boz), eps, gx,
                   gy, gz, nev, nbo);
        if (!unit_normal(gx, gy, gz, nox, noy, noz)) {
            nox = -bdx;
            noy = -bdy;
            noz = -bdz;
        }
    }
    const float* R = S.rot;
    float nx = fmaf(R[0], nox, fmaf(R[1], noy, R[2] * noz));
    float ny = fmaf(R[3], nox, fmaf(R[4], noy, R[5] * noz));
    float nz = fmaf(R[6], nox, fmaf(R[7], noy, R[8] * noz));
    {
        float tx, ty, tz;
        if (unit_normal(nx, ny, nz, tx, ty, tz)) {
            nx = tx;
            ny = ty;
            nz = tz;
        }
    }

    // Lambert term and the shadow ray, in world space
    const float tw = best_tw;
    const float ndl = fmaf(nx, cam.light[0], fmaf(ny, cam.light[1], nz * cam.light[2]));
    int status = hit.status;
    unsigned sev = 0, sbo = 0;
    float vis = 1.0f;
    if (cam.shadow && ndl > 0.0f) {
        const float eps_s = fmaf(cam.eps_rel, tw, cam.eps_abs);
        const float off = 4.0f * eps_s;
        const float qx = fmaf(off, nx, fmaf(tw, dx, ex));
        const float qy = fmaf(off, ny, fmaf(tw, dy, ey));
        const float qz = fmaf(off, nz, fmaf(tw, dz, ez));
        for (int k = 0; k < n_obj; ++k) {
            const SceneObject& O = objs[k];
            const JobDev& JO = O.job;
            const OrbitParams P = orbit_params(JO);
            float sox, soy, soz, sdx, sdy, sdz;
            to_object(O, qx, qy, qz, true, sox, soy, soz);
            to_object(O, cam.light[0], cam.light[1], cam.light[2], false, sdx, sdy, sdz);
            const float eo = eps_s * O.inv_scale;
            const MarchOut r = march_any(O.variant, JO, P, sox, soy, soz, sdx, sdy, sdz, eo, JO.t_max, eo, 0.0f, true);
            sev += r.evals;
            sbo += r.bodies;
            if ((r.status & 7) >= kHit) {
                vis = 0.0f;
                status |= kFlagShadowed;
                break;
            }
        }
    }
    // albedo of the hit: the given one, or with the closest-hit model and a
    // trap palette, coloured by the orbit trap of the hit point
    float alb[3] = {cam.albedo[0], cam.albedo[1], cam.albedo[2]};
    float tr[4] = {0.f, 0.f, 0.f, 0.f};
    const bool need_trap = trap != nullptr || (cam.shading == 1 && cam.trap_colour);
    if (need_trap) {
        const OrbitParams P = orbit_params(J);
        trap_any(S.variant, P, fmaf(hit.t, bdx, box), fmaf(hit.t, bdy, boy), fmaf(hit.t, bdz, boz), tr);
        if (cam.shading == 1 && cam.trap_colour) trap_albedo(cam, tr, alb);
    }
    const float lam = fmaf(cam.k_d * vis, fmaxf(ndl, 0.0f), cam.k_a);
    float col[3] = {alb[0] * lam, alb[1] * lam, alb[2] * lam};
    if (cam.shading == 1) {
        // closest-hit shading: highlight, then one reflection bounce
        const float spec = cam.k_s * vis * phong_spec(nx, ny, nz, cam.light, -dx, -dy, -dz, ndl, cam.shininess);
        for (int c = 0; c < 3; ++c) col[c] += spec;
        const float dn = fmaf(dx, nx, fmaf(dy, ny, dz * nz));
        const float rdx = fmaf(-2.0f * dn, nx, dx), rdy = fmaf(-2.0f * dn, ny, dy), rdz = fmaf(-2.0f * dn, nz, dz);
        const float eps_s = fmaf(cam.eps_rel, tw, cam.eps_abs);
        const float off = 4.0f * eps_s;
        const float qx = fmaf(off, nx, fmaf(tw, dx, ex));
        const float qy = fmaf(off, ny, fmaf(tw, dy, ey));
        const float qz = fmaf(off, nz, fmaf(tw, dz, ez));
        int rbest = -1;
        float rtw = 0.0f, rox = 0.f, roy = 0.f, roz = 0.f, rvx = 0.f, rvy = 0.f, rvz = 0.f, reo = 0.f;
        MarchOut rh{kMissBounds, -1.0f, 0, 0, -1, 0u, 0u, false};
        for (int k = 0; k < n_obj; ++k) {
            const SceneObject& O = objs[k];
            const JobDev& JO = O.job;
            const OrbitParams P = orbit_params(JO);
            float sox, soy, soz, sdx, sdy, sdz;
            to_object(O, qx, qy, qz, true, sox, soy, soz);
            to_object(O, rdx, rdy, rdz, false, sdx, sdy, sdz);
            const float eo = eps_s * O.inv_scale;
            const float cap = rbest >= 0 ? fmaf(rtw, O.inv_scale, JO.clamp) : JO.t_max;
            const MarchOut r = march_any(O.variant, JO, P, sox, soy, soz, sdx, sdy, sdz, eo, cap, eo, JO.eps_rel, false);
            sev += r.evals;
            sbo += r.bodies;
            if ((r.status & 7) >= kHit) {
                const float t_w = r.t * O.scale;
                if (rbest < 0 || t_w < rtw) {
                    rbest = k;
                    rtw = t_w;
                    rh = r;
                    rox = sox; roy = soy; roz = soz;
                    rvx = sdx; rvy = sdy; rvz = sdz;
                    reo = eo;
                }
            }
        }
        if (rbest >= 0) {
            status |= kFlagReflectHit;
            const SceneObject& O = objs[rbest];
            const JobDev& JO = O.job;
            float mx, my, mz;
            if ((rh.status & 7) == kHitCut) {
                mx = JO.pn[rh.entry][0];
                my = JO.pn[rh.entry][1];
                mz = JO.pn[rh.entry][2];
            } else {
                const OrbitParams P = orbit_params(JO);
                float gx, gy, gz;
                unsigned ev = 0, bo = 0;
                normal_any(O.variant, P, JO.normal_mode, fmaf(rh.t, rvx, rox), fmaf(rh.t, rvy, roy),
                           fmaf(rh.t, rvz, roz), fmaf(JO.eps_rel, rh.t, reo), gx, gy, gz, ev, bo);
                sev += ev;
                sbo += bo;
                if (!unit_normal(gx, gy, gz, mx, my, mz)) {
                    mx = -rvx;
                    my = -rvy;
                    mz = -rvz;
                }
            }
            const float* RO = O.rot;
            float wx = fmaf(RO[0], mx, fmaf(RO[1], my, RO[2] * mz));
            float wy = fmaf(RO[3], mx, fmaf(RO[4], my, RO[5] * mz));
            float wz = fmaf(RO[6], mx, fmaf(RO[7], my, RO[8] * mz));
            float ux, uy, uz;
            if (unit_normal(wx, wy, wz, ux, uy, uz)) {
                wx = ux;
                wy = uy;
                wz = uz;
            }
            float ralb[3] = {cam.albedo[0], cam.albedo[1], cam.albedo[2]};
            if (cam.trap_colour) {
                const OrbitParams P = orbit_params(JO);
                float rtr[4];
                trap_any(O.variant, P, fmaf(rh.t, rvx, rox), fmaf(rh.t, rvy, roy), fmaf(rh.t, rvz, roz), rtr);
                trap_albedo(cam, rtr, ralb);
            }
            const float rndl = fmaf(wx, cam.light[0], fmaf(wy, cam.light[1], wz * cam.light[2]));
            const float rlam = fmaf(cam.k_d, fmaxf(rndl, 0.0f), cam.k_a);
            const float rspec = cam.k_s * phong_spec(wx, wy, wz, cam.light, -rdx, -rdy, -rdz, rndl, cam.shininess);
            const float ci = 1.0f - fmaxf(0.0f, -dn);
            const float ci2 = ci * ci;
            const float f5 = ci2 * ci2 * ci;
            for (int c = 0; c < 3; ++c) {
                const float F = fmaf(1.0f - alb[c], f5, alb[c]);
                col[c] = fmaf(cam.k_r * F, fmaf(ralb[c], rlam, rspec), col[c]);
            }
        }
    }
    if (trap)
        for (int c = 0; c < 4; ++c) trap[c * NP + p] = tr[c];
    cam.depth[p] = tw;
    cam.normal[p] = nx;
    cam.normal[NP + p] = ny;
    cam.normal[2 * NP + p] = nz;
    cam.colour[p] = col[0];
    cam.colour[NP + p] = col[1];
    cam.colour[2 * NP + p] = col[2];
    cam.status[p] = static_cast<uint8_t>(status);
    if (cam.counters) {
        cam.counters[p] = static_cast<unsigned>(hit.steps);
        cam.counters[NP + p] = hit.evals;
        cam.counters[2 * NP + p] = hit.bodies;
        cam.counters[3 * NP + p] = static_cast<unsigned>(hit.hit_it);
        cam.counters[4 * NP + p] = nev;
        cam.counters[5 * NP + p] = nbo;
        cam.counters[6 * NP + p] = sev;
        cam.counters[7 * NP + p] = sbo;
    }
}

hipError_t launch_scene(const SceneObject* objs, int n_obj, const JobDev& cam, int* object_id, float* trap,
                        hipStream_t stream) {
    const long long rays = cam.ray_count;
    const int block = 256;
    const long long grid = (rays + block - 1) / block;
    hipLaunchKernelGGL(scene_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, stream, objs, n_obj, cam,
                       object_id, trap);
    return hipGetLastError();
}

}  // namespace frt
