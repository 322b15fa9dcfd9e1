/*
 * frt_oracle.c -- FP64 CPU oracle for per-pixel sphere tracing of escape-time
 * fractals: the quaternion Julia set z^p+c sliced to 3-D (optionally cut by
 * planes) and the White-Nylander power-n Mandelbulb, as described in
 * da Silva, Novello, Lopes, Velho, "Real-time rendering of complex fractals"
 * (arXiv 2102.01747).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does.  It shares no code, header, table or constant
 * generator with the GPU library: every structure below is declared here.
 *
 * Arithmetic is IEEE double with the C library's libm (build with
 * -O2 -fno-fast-math).  Parameters arrive as the caller's float32 values
 * widened to double, so parameter rounding does not pollute parity.
 *
 * Readings of the paper that this file fixes (each one repeated at its use):
 *   R1  Julia degree p, an integer >= 2 (2 is the text's z^2+c, 3 the cubic
 *       of Listing 4).  z^p is p - 1 quaternion products of z by itself.
 *       Running squared derivative dz2 <- p^2 |z^(p-1)|^2 dz2 (Eq. 4 taken
 *       in norm, as Listing 4 does with 9 |z^2|^2 at p = 3), updated before
 *       z.
 *   R2  Quaternion component 0 is the real part; the 3-D slice is z0=(x,y,z,0).
 *   R3  DE d = 0.25 ln(m2) sqrt(m2/dz2) = 0.5|z|ln|z|/|z'| (Listings 4, 7).
 *   R4  Mandelbulb power map as in Listing 7 (y is the polar axis,
 *       theta = acos(y/r), phi = atan2(x, z)), generalised to real n.
 *   R5  Escape count = number of orbit bodies whose result did not exceed the
 *       bailout; "no escape" means the count equals max_iter.
 *   R6  March per Listing 3: stop when d < eps(t) = eps_abs + eps_rel*t,
 *       step min(d, clamp), miss when t > t1, running out of steps is a hit.
 *   R7  Interval per the text around Listing 3: [eps_abs, t_max] cut by a
 *       bounding sphere (provable escape radius) and up to two half-spaces.
 *   R8  A ray that enters through a plane hits the cut face when the entry
 *       point is inside (no escape in max_iter, or d < eps) -- the 2-D
 *       escape-time test of Sec. 1.1 applied on the face.
 *   R9  Hit depth is the root of d(o+t*dir) - eps(t) between the last two
 *       samples (the listing's lt/lh); here by bisection to the resolution
 *       of double precision.
 *   R10 Normals: tetrahedral taps of Eq. 5 with h = 0.5773 eps (Listing 5),
 *       central differences with h = eps, or (mode 2) the analytic normal of
 *       Sec. 2's quotient-rule remark: the exact gradient of the estimate d
 *       at the hit point itself, by forward-mode differentiation.
 *   R11 Lambert shading with one optional shadow ray replaces the paper's
 *       Phong/Fresnel closest-hit shader.
 *
 * Pins: the test suite ties every function here to closed forms, symmetries,
 * special cases or brute force.  The Mandelbulb running derivative is pinned
 * on the positive polar axis, where the orbit is the real map y <- y^n + c
 * and dr must be its exact c-derivative.  The two rounding probes
 * (oracle_normal_perturbed, oracle_trap_perturbed) perturb each orbit body on
 * purpose; they are pinned only as far as a probe can be: with a zero
 * perturbation they reproduce the plain normal and trap bit for bit, they
 * converge to them as the perturbation shrinks, and their factor is uniform
 * on the stated interval.  How well a probe models float32 rounding is an
 * assumption of the comparison masks, not a pinned fact.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameter blocks (oracle-private layout, filled from Python via ctypes).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;
    int32_t width, height;
} or_camera;

typedef struct {
    int32_t kind;      /* 0 = quaternion Julia z^p+c, 1 = Mandelbulb p^n+c */
    double c[4];       /* Julia constant (component 0 real)                 */
    double power;      /* Mandelbulb exponent n (real, >= 2); Julia degree  */
                       /* p (an integer >= 2)                               */
    int32_t max_iter;  /* orbit bodies per distance evaluation (>= 1)       */
    double bailout2;   /* escape when |z|^2 exceeds this                    */
    double bound_radius; /* caller's bounding radius; the larger of it and   */
                         /* the provable escape radius is used               */
} or_fractal;

typedef struct {
    double n[3];       /* raw normal; kept side is  n_hat . x <= d          */
    double d;
} or_plane;

typedef struct {
    int32_t max_steps;
    double eps_abs, eps_rel, step_clamp, t_max;
    int32_t normal_mode;   /* 0 tetrahedral (Eq. 5), 1 central differences, 2 analytic gradient */
    int32_t shadow;        /* 1: one shadow ray per lit hit                */
    double light[3], albedo[3], k_ambient, k_diffuse;
    int32_t shading;       /* 0 Lambert; 1 Phong + Fresnel reflection (scenes, R23) */
    double k_specular, shininess, k_reflect;
} or_march;

/* status classes (low 3 bits) and flags */
enum { ST_MISS_BOUNDS = 0, ST_MISS_TMAX = 1, ST_HIT = 2, ST_HIT_CUT = 3, ST_HIT_EXHAUSTED = 4 };
enum { ST_FLAG_SHADOWED = 8, ST_FLAG_UNREFINED = 16, ST_FLAG_JUMP = 32 };

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void normalize3(double v[3]) {
    double l = sqrt(dot3(v, v));
    v[0] /= l; v[1] /= l; v[2] /= l;
}
static void cross3(const double a[3], const double b[3], double out[3]) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    out[0] = x; out[1] = y; out[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Quaternion algebra (R2): q = a + b i + c j + d k stored as {a, b, c, d}.  */
/* Square of a quaternion with real part a and vector part v:                */
/*   (a + v)^2 = a^2 - |v|^2 + 2 a v     (v v = -|v|^2 for pure imaginary v) */
/* ------------------------------------------------------------------------ */
void oracle_quat_square(const double z[4], double out[4]) {
    double a = z[0];
    double vv = z[1] * z[1] + z[2] * z[2] + z[3] * z[3];
    out[0] = a * a - vv;
    out[1] = 2.0 * a * z[1];
    out[2] = 2.0 * a * z[2];
    out[3] = 2.0 * a * z[3];
}

/* Hamilton product x y with i^2 = j^2 = k^2 = ijk = -1:                     */
/*   (a1 + v1)(a2 + v2) = a1 a2 - v1.v2 + a1 v2 + a2 v1 + v1 x v2.           */
void oracle_quat_mul(const double x[4], const double y[4], double out[4]) {
    double r0 = x[0] * y[0] - (x[1] * y[1] + x[2] * y[2] + x[3] * y[3]);
    double r1 = x[0] * y[1] + y[0] * x[1] + (x[2] * y[3] - x[3] * y[2]);
    double r2 = x[0] * y[2] + y[0] * x[2] + (x[3] * y[1] - x[1] * y[3]);
    double r3 = x[0] * y[3] + y[0] * x[3] + (x[1] * y[2] - x[2] * y[1]);
    out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3;
}

/* z^p for an integer p >= 1 (R1): z^1 = z, z^2 by the square above, and    */
/* each further power one more product by z.                                 */
void oracle_quat_pow(const double z[4], int32_t p, double out[4]) {
    double w[4] = { z[0], z[1], z[2], z[3] };
    if (p >= 2) oracle_quat_square(z, w);
    for (int32_t k = 3; k <= p; ++k) {
        double t[4];
        oracle_quat_mul(w, z, t);
        for (int i = 0; i < 4; ++i) w[i] = t[i];
    }
    for (int i = 0; i < 4; ++i) out[i] = w[i];
}

static double qlen2(const double z[4]) {
    return z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3];
}

/* Julia degree (R1). */
static int32_t julia_degree(const or_fractal* f) {
    return (int32_t)f->power;
}

/* Factor the squared running derivative gains in one body at z (R1):       */
/* p^2 |z^(p-1)|^2, which is 4 |z|^2 at p = 2.                               */
static double julia_deriv_factor(const double z[4], int32_t p) {
    double zp[4];
    oracle_quat_pow(z, p - 1, zp);
    return (double)p * (double)p * qlen2(zp);
}

/* ------------------------------------------------------------------------ */
/* White-Nylander n-th power, Eq. 1 in the axis convention of Listing 7      */
/* (R4): y is the polar axis, theta = acos(y/r), phi = atan2(x, z),          */
/*   p^n = r^n ( sin(n theta) sin(n phi), cos(n theta), sin(n theta) cos(n phi) ). */
/* r = 0 maps to 0; the acos argument is clamped to [-1, 1]; atan2(0,0) = 0. */
/* ------------------------------------------------------------------------ */
void oracle_bulb_power(const double w[3], double n, double out[3]) {
    double r = sqrt(dot3(w, w));
    if (r == 0.0) { out[0] = out[1] = out[2] = 0.0; return; }
    double u = w[1] / r;
    if (u > 1.0) u = 1.0;
    if (u < -1.0) u = -1.0;
    double b = n * acos(u);
    double a = n * atan2(w[0], w[2]);
    double rn = pow(r, n);
    out[0] = rn * sin(b) * sin(a);
    out[1] = rn * cos(b);
    out[2] = rn * sin(b) * cos(a);
}

/* ------------------------------------------------------------------------ */
/* Distance estimators.                                                      */
/* Julia (Sec. 2, Eq. 2-4; Listing 4, R1-R3, R5), degree p:                  */
/*   z = (x, 0); dz2 = 1; repeat max_iter: dz2 *= p^2 |z^(p-1)|^2;           */
/*   z = z^p + c; m2 = |z|^2; stop if m2 > bailout2.                         */
/*   d = 0.25 ln(m2) sqrt(m2 / dz2).                                          */
/* Mandelbulb (Listing 7 with general n, R4-R5): w = p; m = |w|^2; dr = 1;   */
/*   repeat: dr = n r^(n-1) dr + 1 (r = |w| before the update);              */
/*   w = w^n + p; m = |w|^2; stop if m > bailout2.  d = 0.25 ln(m) sqrt(m)/dr.*/
/* m = 0 (orbit pinned at the origin) is defined as d = 0.                   */
/* ------------------------------------------------------------------------ */
typedef struct { double d; int32_t iters; double m2; double deriv; int32_t bodies; } de_result;

static de_result julia_de(const or_fractal* f, const double p[3]) {
    de_result res;
    double z[4] = { p[0], p[1], p[2], 0.0 };
    double dz2 = 1.0, m2 = 0.0;
    int32_t n = 0, bodies = 0;
    int32_t deg = julia_degree(f);
    for (int32_t i = 0; i < f->max_iter; ++i) {
        ++bodies;
        dz2 *= julia_deriv_factor(z, deg);
        double zp[4];
        oracle_quat_pow(z, deg, zp);
        for (int k = 0; k < 4; ++k) z[k] = zp[k] + f->c[k];
        m2 = qlen2(z);
        if (m2 > f->bailout2) break;
        ++n;
    }
    res.d = (m2 == 0.0) ? 0.0 : 0.25 * log(m2) * sqrt(m2 / dz2);
    res.iters = n; res.m2 = m2; res.deriv = dz2; res.bodies = bodies;
    return res;
}

static de_result bulb_de(const or_fractal* f, const double p[3]) {
    de_result res;
    double w[3] = { p[0], p[1], p[2] };
    double m = dot3(w, w);
    double dr = 1.0;
    int32_t n = 0, bodies = 0;
    for (int32_t i = 0; i < f->max_iter; ++i) {
        ++bodies;
        double r = sqrt(m);
        dr = f->power * pow(r, f->power - 1.0) * dr + 1.0;
        double wn[3];
        oracle_bulb_power(w, f->power, wn);
        w[0] = wn[0] + p[0]; w[1] = wn[1] + p[1]; w[2] = wn[2] + p[2];
        m = dot3(w, w);
        if (m > f->bailout2) break;
        ++n;
    }
    res.d = (m == 0.0) ? 0.0 : 0.25 * log(m) * sqrt(m) / dr;
    res.iters = n; res.m2 = m; res.deriv = dr; res.bodies = bodies;
    return res;
}

static de_result fractal_de(const or_fractal* f, const double p[3]) {
    return f->kind == 0 ? julia_de(f, p) : bulb_de(f, p);
}

/* Gradient of the estimate at p (the analytic normal of R10), defined with
 * the dual numbers further down.                                            */
static int32_t analytic_gradient(const or_fractal* f, const double p[3], double rel, uint64_t seed, uint64_t key,
                                 double g[3]);

/* Escape count of the orbit at p with an explicit iteration budget (R5). */
int32_t oracle_escape_iters(const or_fractal* f, const double p[3], int32_t max_iter) {
    or_fractal g = *f;
    g.max_iter = max_iter;
    return fractal_de(&g, p).iters;
}

/* Batched DE for tests: d, escape count, final |z|^2, running derivative.  */
void oracle_de(const or_fractal* f, const double* pts, int64_t n_pts,
               double* d, int32_t* iters, double* m2, double* deriv) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n_pts; ++i) {
        de_result r = fractal_de(f, pts + 3 * i);
        if (d) d[i] = r.d;
        if (iters) iters[i] = r.iters;
        if (m2) m2[i] = r.m2;
        if (deriv) deriv[i] = r.deriv;
    }
}

/* Tetrahedron vertices of Eq. 5. */
static const double TETRA[4][3] = { { 1, -1, -1 }, { -1, -1, 1 }, { -1, 1, -1 }, { 1, 1, 1 } };

/* ------------------------------------------------------------------------ */
/* Conditioning probe: the estimate with a relative perturbation of size     */
/* `rel` (uniform in [-rel, rel], one draw per component per body) applied   */
/* to the power z^p of every body before c is added -- a Monte-Carlo model   */
/* of rounding in a lower precision, placed where it matters: near the set   */
/* z^p + c cancels, so the absolute error of z^p becomes a large relative    */
/* error of the sum that the next body multiplies again.  Draws come from    */
/* SplitMix64 (Steele, Lea and Flood, 2014) keyed by (seed, point, body,     */
/* component).                                                               */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
static double noise(uint64_t seed, uint64_t point, int body, int comp, double rel) {
    uint64_t h = splitmix64(seed ^ splitmix64(point * 0x100000001B3ull + (uint64_t)body * 8u + (uint64_t)comp));
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);   /* [0, 1) */
    return 1.0 + rel * (2.0 * u - 1.0);
}

/* The probe's factor for one (seed, point, body, component), exported so
 * that the tests can check its distribution.                               */
double oracle_probe_noise(uint64_t seed, uint64_t point, int32_t body, int32_t comp, double rel) {
    return noise(seed, point, body, comp, rel);
}

static double perturbed_de(const or_fractal* f, const double p[3], double rel, uint64_t seed, uint64_t key) {
    if (f->kind == 0) {
        double z[4] = { p[0], p[1], p[2], 0.0 };
        double dz2 = 1.0, m2 = 0.0;
        int32_t deg = julia_degree(f);
        for (int32_t i = 0; i < f->max_iter; ++i) {
            dz2 *= julia_deriv_factor(z, deg);
            double zp[4];
            oracle_quat_pow(z, deg, zp);
            for (int k = 0; k < 4; ++k) z[k] = zp[k] * noise(seed, key, i, k, rel) + f->c[k];
            m2 = qlen2(z);
            if (m2 > f->bailout2) break;
        }
        return (m2 == 0.0) ? 0.0 : 0.25 * log(m2) * sqrt(m2 / dz2);
    }
    double w[3] = { p[0], p[1], p[2] };
    double m = dot3(w, w), dr = 1.0;
    for (int32_t i = 0; i < f->max_iter; ++i) {
        double r = sqrt(m);
        dr = f->power * pow(r, f->power - 1.0) * dr + 1.0;
        double wn[3];
        oracle_bulb_power(w, f->power, wn);
        for (int k = 0; k < 3; ++k) w[k] = wn[k] * noise(seed, key, i, k, rel) + p[k];
        m = dot3(w, w);
        if (m > f->bailout2) break;
    }
    return (m == 0.0) ? 0.0 : 0.25 * log(m) * sqrt(m) / dr;
}

/* Normal (R10) at points with the perturbed estimate at every tap. */
void oracle_normal_perturbed(const or_fractal* f, const double* pts, const double* dirs, const double* eps,
                             int64_t n, int32_t mode, double rel, uint64_t seed, double* out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const double* p = pts + 3 * i;
        double g[3] = { 0, 0, 0 };
        if (mode == 0) {
            double h = 0.5773 * eps[i];
            for (int a = 0; a < 4; ++a) {
                double q[3] = { p[0] + h * TETRA[a][0], p[1] + h * TETRA[a][1], p[2] + h * TETRA[a][2] };
                double d = perturbed_de(f, q, rel, seed, (uint64_t)i * 8u + (uint64_t)a);
                for (int k = 0; k < 3; ++k) g[k] += TETRA[a][k] * d;
            }
        } else if (mode == 2) {
            analytic_gradient(f, p, rel, seed, (uint64_t)i * 8u, g);
        } else {
            for (int k = 0; k < 3; ++k) {
                double qp[3] = { p[0], p[1], p[2] }, qm[3] = { p[0], p[1], p[2] };
                qp[k] += eps[i];
                qm[k] -= eps[i];
                g[k] = perturbed_de(f, qp, rel, seed, (uint64_t)i * 8u + (uint64_t)(2 * k)) -
                       perturbed_de(f, qm, rel, seed, (uint64_t)i * 8u + (uint64_t)(2 * k + 1));
            }
        }
        double l = sqrt(dot3(g, g));
        for (int k = 0; k < 3; ++k) out[3 * i + k] = l > 0.0 ? g[k] / l : -dirs[3 * i + k];
    }
}

/* Escape-decision margin of the orbit at p: the smallest relative distance
 * | |z_k|^2 - bailout2 | / bailout2 over the executed bodies, and whether the
 * orbit escaped.  A small margin means the escape count (and so the estimate,
 * which jumps where the count changes) is decided by rounding.             */
static double escape_margin(const or_fractal* f, const double p[3], int* escaped) {
    double best = INFINITY;
    *escaped = 0;
    if (f->kind == 0) {
        double z[4] = { p[0], p[1], p[2], 0.0 };
        int32_t deg = julia_degree(f);
        for (int32_t i = 0; i < f->max_iter; ++i) {
            double zp[4];
            oracle_quat_pow(z, deg, zp);
            for (int k = 0; k < 4; ++k) z[k] = zp[k] + f->c[k];
            double m2 = qlen2(z);
            best = fmin(best, fabs(m2 - f->bailout2) / f->bailout2);
            if (m2 > f->bailout2) { *escaped = 1; break; }
        }
    } else {
        double w[3] = { p[0], p[1], p[2] };
        for (int32_t i = 0; i < f->max_iter; ++i) {
            double wn[3];
            oracle_bulb_power(w, f->power, wn);
            w[0] = wn[0] + p[0]; w[1] = wn[1] + p[1]; w[2] = wn[2] + p[2];
            double m = dot3(w, w);
            best = fmin(best, fabs(m - f->bailout2) / f->bailout2);
            if (m > f->bailout2) { *escaped = 1; break; }
        }
    }
    return best;
}

void oracle_escape_margin(const or_fractal* f, const double* pts, int64_t n, double* margin, int32_t* escaped) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int e;
        margin[i] = escape_margin(f, pts + 3 * i, &e);
        if (escaped) escaped[i] = e;
    }
}

/* Bounding-sphere radius (R7): any point farther out escapes.
 * Julia of degree p: |z^p + c| >= |z|^p - |c| > |z| whenever |z| exceeds the
 * root R >= 1 of R^p - R - |c| = 0; at p = 2 that root is
 * (1 + sqrt(1 + 4|c|))/2, for larger p it is found by bisection on
 * [1, 2 + |c|] (the polynomial is <= 0 at 1 and > 0 at 2 + |c|).
 * Mandelbulb: |p^n| = r^n, so the Multibrot bound 2^(1/(n-1)) applies.     */
double oracle_bound_radius(const or_fractal* f) {
    double R;
    if (f->kind == 0) {
        double cn = sqrt(qlen2(f->c));
        int32_t deg = julia_degree(f);
        if (deg == 2) {
            R = 0.5 * (1.0 + sqrt(1.0 + 4.0 * cn));
        } else {
            double lo = 1.0, hi = 2.0 + cn;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (pow(mid, (double)deg) - mid - cn > 0.0) hi = mid; else lo = mid;
            }
            R = hi;
        }
    } else {
        R = pow(2.0, 1.0 / (f->power - 1.0));
    }
    return fmax(R, f->bound_radius);
}

/* ------------------------------------------------------------------------ */
/* Camera: pinhole, vertical field of view, pixel centres, row 0 at the top. */
/* ------------------------------------------------------------------------ */
void oracle_camera_ray(const or_camera* cam, int32_t i, int32_t j, double o[3], double dir[3]) {
    double f[3] = { cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1], cam->target[2] - cam->eye[2] };
    normalize3(f);
    double r[3];
    cross3(f, cam->up, r);
    normalize3(r);
    double u[3];
    cross3(r, f, u);
    double s = tan(0.5 * cam->fov_y_deg * M_PI / 180.0);
    double x = (2.0 * (i + 0.5) / cam->width - 1.0) * s * (double)cam->width / (double)cam->height;
    double y = (1.0 - 2.0 * (j + 0.5) / cam->height) * s;
    for (int k = 0; k < 3; ++k) {
        o[k] = cam->eye[k];
        dir[k] = f[k] + x * r[k] + y * u[k];
    }
    normalize3(dir);
}

/* ------------------------------------------------------------------------ */
/* Search interval (R7): [tmin, t_max] intersected with |x| <= R and with    */
/* each kept half-space n_hat . x <= d.  Reports which plane (if any) set    */
/* the entry strictly after every other lower bound.                          */
/* ------------------------------------------------------------------------ */
static int ray_interval(const or_fractal* f, const or_plane* planes, int32_t n_planes,
                        const double o[3], const double dir[3], double tmin, double tmax,
                        double* lo_out, double* hi_out, int* entry_plane) {
    double R = oracle_bound_radius(f);
    double b = dot3(o, dir);
    double cc = dot3(o, o) - R * R;
    double disc = b * b - cc;
    if (disc < 0.0) return 0;
    double sq = sqrt(disc);
    double lo = fmax(tmin, -b - sq);
    double hi = fmin(tmax, -b + sq);
    int entry = -1;
    for (int32_t k = 0; k < n_planes; ++k) {
        double nh[3] = { planes[k].n[0], planes[k].n[1], planes[k].n[2] };
        normalize3(nh);
        double denom = dot3(nh, dir);
        double num = planes[k].d - dot3(nh, o);
        if (denom == 0.0) {
            if (num < 0.0) return 0;
        } else if (denom > 0.0) {
            hi = fmin(hi, num / denom);
        } else {
            double tk = num / denom;
            if (tk > lo) { lo = tk; entry = k; }
        }
    }
    if (lo > hi) return 0;
    *lo_out = lo; *hi_out = hi; *entry_plane = entry;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* One traced ray: interval, cut-face test, sphere-tracing march (R6-R8).    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int status;
    double t, lt, lh;    /* final sample, previous sample and its distance   */
    int has_prev;
    double lo, hi;
    int entry_plane;
    int32_t steps;       /* march samples                                     */
    int32_t hit_iters;   /* escape count at the final march sample            */
    int64_t de_evals, orbit_bodies;
} trace_result;

static void trace_ray(const or_fractal* f, const or_plane* planes, int32_t n_planes,
                      const double o[3], const double dir[3], double eps_abs, double eps_rel,
                      double tmin, int32_t max_steps, double clamp, double tmax, trace_result* tr) {
    memset(tr, 0, sizeof(*tr));
    tr->entry_plane = -1;
    double lo, hi;
    int entry;
    if (!ray_interval(f, planes, n_planes, o, dir, tmin, tmax, &lo, &hi, &entry)) {
        tr->status = ST_MISS_BOUNDS;
        return;
    }
    tr->lo = lo; tr->hi = hi; tr->entry_plane = entry;
    if (entry >= 0) {
        /* R8: the entry point lies on the cut plane; it is on the cut face
         * when the orbit there does not escape, or the estimate is below eps. */
        double p[3] = { o[0] + lo * dir[0], o[1] + lo * dir[1], o[2] + lo * dir[2] };
        de_result r = fractal_de(f, p);
        tr->de_evals++; tr->orbit_bodies += r.bodies;
        if (r.iters == f->max_iter || r.d < eps_abs + eps_rel * lo) {
            tr->status = ST_HIT_CUT;
            tr->t = lo;
            tr->hit_iters = r.iters;
            return;
        }
    }
    /* Listing 3. */
    double t = lo;
    for (int32_t s = 0; s < max_steps; ++s) {
        double p[3] = { o[0] + t * dir[0], o[1] + t * dir[1], o[2] + t * dir[2] };
        de_result r = fractal_de(f, p);
        tr->de_evals++; tr->orbit_bodies += r.bodies;
        tr->steps++;
        tr->hit_iters = r.iters;
        if (r.d < eps_abs + eps_rel * t) {
            tr->status = ST_HIT;
            tr->t = t;
            return;
        }
        tr->lt = t; tr->lh = r.d; tr->has_prev = 1;
        t += fmin(r.d, clamp);
        if (t > hi) {
            tr->status = ST_MISS_TMAX;
            tr->t = t;
            return;
        }
    }
    tr->status = ST_HIT_EXHAUSTED;
    tr->t = t;
}

/* R9: bisection on g(t) = d(o + t dir) - eps(t), g(a) >= 0 > g(b), until
 * the bracket cannot be split any further in double precision.  The
 * estimate is only piecewise smooth (the escape count, and for non-integer
 * n the azimuth branch cut, make it jump), so a bracket may close on a jump
 * instead of a root; *jump reports that (|g| stays large on both sides). */
static double refine_root(const or_fractal* f, const double o[3], const double dir[3],
                          double eps_abs, double eps_rel, double a, double b, int64_t* evals, int64_t* bodies,
                          int* jump) {
    double ga = 1.0, gb = -1.0;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (a + b);
        if (m <= a || m >= b) break;
        double p[3] = { o[0] + m * dir[0], o[1] + m * dir[1], o[2] + m * dir[2] };
        de_result r = fractal_de(f, p);
        (*evals)++; (*bodies) += r.bodies;
        double g = r.d - (eps_abs + eps_rel * m);
        if (g < 0.0) { b = m; gb = g; } else { a = m; ga = g; }
    }
    *jump = fmin(fabs(ga), fabs(gb)) > 1e-10;
    return 0.5 * (a + b);
}

/* R10: normal at p from distance taps, or the analytic gradient (mode 2).
 * A zero gradient falls back to -dir.                                       */

static void estimate_normal(const or_fractal* f, const double p[3], double eps, int mode,
                            const double dir[3], double nrm[3], int64_t* evals, int64_t* bodies) {
    double g[3] = { 0, 0, 0 };
    if (mode == 0) {
        double h = 0.5773 * eps;
        for (int i = 0; i < 4; ++i) {
            double q[3] = { p[0] + h * TETRA[i][0], p[1] + h * TETRA[i][1], p[2] + h * TETRA[i][2] };
            de_result r = fractal_de(f, q);
            (*evals)++; (*bodies) += r.bodies;
            for (int k = 0; k < 3; ++k) g[k] += TETRA[i][k] * r.d;
        }
    } else if (mode == 1) {
        double h = eps;
        for (int k = 0; k < 3; ++k) {
            double qp[3] = { p[0], p[1], p[2] }, qm[3] = { p[0], p[1], p[2] };
            qp[k] += h; qm[k] -= h;
            de_result rp = fractal_de(f, qp), rm = fractal_de(f, qm);
            (*evals) += 2; (*bodies) += rp.bodies + rm.bodies;
            g[k] = rp.d - rm.d;
        }
    } else {
        int32_t it = analytic_gradient(f, p, 0.0, 0, 0, g);
        (*evals) += 1; (*bodies) += it < f->max_iter ? it + 1 : it;
    }
    double l = sqrt(dot3(g, g));
    if (!(l > 0.0 && isfinite(l))) { nrm[0] = -dir[0]; nrm[1] = -dir[1]; nrm[2] = -dir[2]; return; }
    nrm[0] = g[0] / l; nrm[1] = g[1] / l; nrm[2] = g[2] / l;
}

/* Normal (R10) at given points with a given eps, for parity checks that
 * separate depth error from normal error.  dirs gives the fallback for a
 * zero gradient.                                                            */
void oracle_normal_at(const or_fractal* f, const double* pts, const double* dirs, const double* eps, int64_t n,
                      int32_t mode, double* out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int64_t ev = 0, bo = 0;
        estimate_normal(f, pts + 3 * i, eps[i], mode, dirs + 3 * i, out + 3 * i, &ev, &bo);
    }
}

/* ------------------------------------------------------------------------ */
/* Full pixel: ray, trace, refine, normal, Lambert + shadow (R6-R11).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double depth, normal[3], colour[3];
    int status;
    int32_t steps, hit_iters;
    int64_t de_evals, orbit_bodies;
    double raw_t;
    int entry_plane;
} pixel_result;

/* Primary part of one ray (R6-R10): interval, march, refinement and normal,
 * no shading.  px->depth is t* (-1 on a miss), px->normal the normal,
 * px->status the class with the JUMP / UNREFINED flags; *lt receives the
 * last-but-one march sample (-1 without one).                              */
static void trace_primary(const or_fractal* f, const or_plane* planes, int32_t n_planes, const or_march* mc,
                          const double o[3], const double dir[3], pixel_result* px, double* lt) {
    memset(px, 0, sizeof(*px));
    trace_result tr;
    trace_ray(f, planes, n_planes, o, dir, mc->eps_abs, mc->eps_rel, mc->eps_abs,
              mc->max_steps, mc->step_clamp, mc->t_max, &tr);
    px->steps = tr.steps; px->hit_iters = tr.hit_iters;
    px->de_evals = tr.de_evals; px->orbit_bodies = tr.orbit_bodies;
    px->raw_t = tr.t; px->entry_plane = tr.entry_plane;
    *lt = tr.has_prev ? tr.lt : -1.0;
    if (tr.status == ST_MISS_BOUNDS || tr.status == ST_MISS_TMAX) {
        px->status = tr.status;
        px->depth = -1.0;
        return;
    }
    int flags = 0;
    double ts, nrm[3];
    if (tr.status == ST_HIT_CUT) {
        ts = tr.t;
        double nh[3] = { planes[tr.entry_plane].n[0], planes[tr.entry_plane].n[1], planes[tr.entry_plane].n[2] };
        normalize3(nh);
        nrm[0] = nh[0]; nrm[1] = nh[1]; nrm[2] = nh[2];
    } else {
        if (tr.status == ST_HIT && tr.has_prev) {
            int jump = 0;
            ts = refine_root(f, o, dir, mc->eps_abs, mc->eps_rel, tr.lt, tr.t, &px->de_evals, &px->orbit_bodies,
                             &jump);
            if (jump) flags |= ST_FLAG_JUMP;
        } else {
            ts = tr.t;
            flags |= ST_FLAG_UNREFINED;
        }
        double p[3] = { o[0] + ts * dir[0], o[1] + ts * dir[1], o[2] + ts * dir[2] };
        estimate_normal(f, p, mc->eps_abs + mc->eps_rel * ts, mc->normal_mode, dir, nrm,
                        &px->de_evals, &px->orbit_bodies);
    }
    px->depth = ts;
    for (int k = 0; k < 3; ++k) px->normal[k] = nrm[k];
    px->status = tr.status | flags;
}

static void render_pixel(const or_camera* cam, const or_fractal* f, const or_plane* planes, int32_t n_planes,
                         const or_march* mc, int32_t i, int32_t j, pixel_result* px) {
    double o[3], dir[3], lt;
    oracle_camera_ray(cam, i, j, o, dir);
    trace_primary(f, planes, n_planes, mc, o, dir, px, &lt);
    if ((px->status & 7) < ST_HIT) return;            /* miss: normal and colour stay 0 */
    double ts = px->depth;
    const double* nrm = px->normal;
    double eps_s = mc->eps_abs + mc->eps_rel * ts;
    double L[3] = { mc->light[0], mc->light[1], mc->light[2] };
    normalize3(L);
    double ndl = dot3(nrm, L);
    double vis = 1.0;
    if (mc->shadow && ndl > 0.0) {
        double q[3];
        for (int k = 0; k < 3; ++k) q[k] = o[k] + ts * dir[k] + 4.0 * eps_s * nrm[k];
        trace_result sh;
        trace_ray(f, planes, n_planes, q, L, eps_s, 0.0, eps_s, mc->max_steps, mc->step_clamp, mc->t_max, &sh);
        px->de_evals += sh.de_evals; px->orbit_bodies += sh.orbit_bodies;
        if (sh.status >= ST_HIT) { vis = 0.0; px->status |= ST_FLAG_SHADOWED; }
    }
    double lam = mc->k_ambient + mc->k_diffuse * fmax(0.0, ndl) * vis;
    for (int k = 0; k < 3; ++k) px->colour[k] = mc->albedo[k] * lam;
}

/* Sign changes of g(s) = d(o + s dir) - eps(s) over `samples` + 1 uniform
 * points of [lo, hi].                                                       */
static int32_t count_crossings(const or_fractal* f, const or_march* mc, const double o[3], const double dir[3],
                               double lo, double hi, int32_t samples) {
    int count = 0, prev_sign = 0;
    for (int32_t k = 0; k <= samples; ++k) {
        double s = lo + (hi - lo) * (double)k / (double)samples;
        double pt[3] = { o[0] + s * dir[0], o[1] + s * dir[1], o[2] + s * dir[2] };
        double g = fractal_de(f, pt).d - (mc->eps_abs + mc->eps_rel * s);
        int sg = g < 0.0 ? -1 : 1;
        if (k > 0 && sg != prev_sign) ++count;
        prev_sign = sg;
    }
    return count;
}

/* Primary part (trace_primary) of n explicit rays, origins and unit
 * directions [n][3], in the fractal's own frame and units: the building
 * block of scenes, whose objects the caller places by similarity maps.
 * eps0 (may be NULL) gives each ray its own eps_abs, which is also where it
 * starts (reflection rays).  normal is [n][3]; lt the last-but-one sample;
 * crossings (when samples > 0) the sign changes of d - eps over the final
 * bracket of refinable hits.                                                */
int oracle_trace_rays(const or_fractal* f, const or_plane* planes, int32_t n_planes, const or_march* mc,
                      const double* orig, const double* dirs, const double* eps0, int64_t n, int32_t samples,
                      uint8_t* status,
                      double* depth, double* normal, int32_t* steps, int32_t* hit_iters, double* raw_t, double* lt,
                      int32_t* crossings, int64_t* de_evals, int64_t* orbit_bodies) {
    if (!f || !mc || !orig || !dirs) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < n; ++q) {
        pixel_result px;
        double l;
        or_march m = *mc;
        if (eps0) m.eps_abs = eps0[q];
        trace_primary(f, planes, n_planes, &m, orig + 3 * q, dirs + 3 * q, &px, &l);
        if (status) status[q] = (uint8_t)px.status;
        if (depth) depth[q] = px.depth;
        if (normal) for (int k = 0; k < 3; ++k) normal[3 * q + k] = px.normal[k];
        if (steps) steps[q] = px.steps;
        if (hit_iters) hit_iters[q] = px.hit_iters;
        if (raw_t) raw_t[q] = px.raw_t;
        if (lt) lt[q] = l;
        if (crossings) {
            crossings[q] = ((px.status & 7) == ST_HIT && l >= 0.0 && samples > 0)
                               ? count_crossings(f, &m, orig + 3 * q, dirs + 3 * q, l, px.raw_t, samples)
                               : 0;
        }
        if (de_evals) de_evals[q] = px.de_evals;
        if (orbit_bodies) orbit_bodies[q] = px.orbit_bodies;
    }
    return 0;
}

/* Shadow test of n explicit rays (R11): does the ray from q [n][3] along the
 * unit direction light [n][3] hit the object (threshold eps[n], started at
 * eps, the march's step cap and range)?  hit[n] is 1 or 0.                  */
int oracle_occluded(const or_fractal* f, const or_plane* planes, int32_t n_planes, const or_march* mc,
                    const double* q, const double* light, const double* eps, int64_t n, uint8_t* hit) {
    if (!f || !mc || !q || !light || !eps || !hit) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t k = 0; k < n; ++k) {
        trace_result sh;
        trace_ray(f, planes, n_planes, q + 3 * k, light + 3 * k, eps[k], 0.0, eps[k], mc->max_steps,
                  mc->step_clamp, mc->t_max, &sh);
        hit[k] = sh.status >= ST_HIT ? 1 : 0;
    }
    return 0;
}

/* Render the listed pixels (linear index j*W + i), or all when pix == NULL.
 * Outputs are planes of length n (SoA); any output pointer may be NULL.     */
int oracle_render(const or_camera* cam, const or_fractal* f, const or_plane* planes, int32_t n_planes,
                  const or_march* mc, const int64_t* pix, int64_t n, int32_t n_threads,
                  double* depth, double* normal, double* colour, uint8_t* status,
                  int32_t* steps, int32_t* hit_iters, int64_t* de_evals, int64_t* orbit_bodies,
                  double* raw_t) {
    if (!cam || !f || !mc) return -1;
    if (pix == NULL) n = (int64_t)cam->width * cam->height;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < n; ++q) {
        int64_t lin = pix ? pix[q] : q;
        int32_t i = (int32_t)(lin % cam->width), j = (int32_t)(lin / cam->width);
        pixel_result px;
        render_pixel(cam, f, planes, n_planes, mc, i, j, &px);
        if (depth) depth[q] = px.depth;
        for (int k = 0; k < 3; ++k) {
            if (normal) normal[k * n + q] = px.normal[k];
            if (colour) colour[k * n + q] = px.colour[k];
        }
        if (status) status[q] = (uint8_t)px.status;
        if (steps) steps[q] = px.steps;
        if (hit_iters) hit_iters[q] = px.hit_iters;
        if (de_evals) de_evals[q] = px.de_evals;
        if (orbit_bodies) orbit_bodies[q] = px.orbit_bodies;
        if (raw_t) raw_t[q] = px.raw_t;
    }
    return 0;
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Orbit trap at points (R24): over the orbit of the estimate at p (the
 * start point and the result of every body run, the escaping one included)
 * the minima of |x|, |y|, |z| (the first three quaternion components for
 * Julia) and of the squared norm.  out is [n][4].                          */
static void trap_at(const or_fractal* f, const double p[3], double rel, uint64_t seed, uint64_t key,
                    double tr[4]) {
    tr[0] = fabs(p[0]); tr[1] = fabs(p[1]); tr[2] = fabs(p[2]); tr[3] = dot3(p, p);
    if (f->kind == 0) {
        double z[4] = { p[0], p[1], p[2], 0.0 };
        int32_t deg = julia_degree(f);
        for (int32_t k = 0; k < f->max_iter; ++k) {
            double zp[4];
            oracle_quat_pow(z, deg, zp);
            for (int c = 0; c < 4; ++c)
                z[c] = (rel != 0.0 ? zp[c] * noise(seed, key, k, c, rel) : zp[c]) + f->c[c];
            double m2 = qlen2(z);
            tr[0] = fmin(tr[0], fabs(z[0])); tr[1] = fmin(tr[1], fabs(z[1])); tr[2] = fmin(tr[2], fabs(z[2]));
            tr[3] = fmin(tr[3], m2);
            if (m2 > f->bailout2) break;
        }
    } else {
        double w[3] = { p[0], p[1], p[2] };
        for (int32_t k = 0; k < f->max_iter; ++k) {
            double wn[3];
            oracle_bulb_power(w, f->power, wn);
            for (int c = 0; c < 3; ++c)
                w[c] = (rel != 0.0 ? wn[c] * noise(seed, key, k, c, rel) : wn[c]) + p[c];
            double m = dot3(w, w);
            tr[0] = fmin(tr[0], fabs(w[0])); tr[1] = fmin(tr[1], fabs(w[1])); tr[2] = fmin(tr[2], fabs(w[2]));
            tr[3] = fmin(tr[3], m);
            if (m > f->bailout2) break;
        }
    }
}

void oracle_trap(const or_fractal* f, const double* pts, int64_t n, double* out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) trap_at(f, pts + 3 * i, 0.0, 0, 0, out + 4 * i);
}

/* The trap with the rounding probe of perturbed_de on every power: a
 * conditioning check of the trap at float32 resolution.                    */
void oracle_trap_perturbed(const or_fractal* f, const double* pts, int64_t n, double rel, uint64_t seed,
                           double* out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) trap_at(f, pts + 3 * i, rel, seed, (uint64_t)i, out + 4 * i);
}

/* Final march bracket of listed pixels (R9): for a refinable surface hit the
 * last two samples [lt, t] and the number of sign changes of
 * g(s) = d(o + s dir) - eps(s) over `samples` + 1 uniform points of it.
 * More than one crossing means the bracket holds several correct depths
 * (a chaotic layer of the estimate); other pixels report lt = t = -1 and 0. */
int oracle_bracket_crossings(const or_camera* cam, const or_fractal* f, const or_plane* planes, int32_t n_planes,
                             const or_march* mc, const int64_t* pix, int64_t n, int32_t samples, double* lt,
                             double* t, int32_t* crossings) {
    if (!cam || !f || !mc || !pix || samples < 1) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t q = 0; q < n; ++q) {
        int32_t i = (int32_t)(pix[q] % cam->width), j = (int32_t)(pix[q] / cam->width);
        double o[3], dir[3];
        oracle_camera_ray(cam, i, j, o, dir);
        trace_result tr;
        trace_ray(f, planes, n_planes, o, dir, mc->eps_abs, mc->eps_rel, mc->eps_abs, mc->max_steps,
                  mc->step_clamp, mc->t_max, &tr);
        lt[q] = t[q] = -1.0;
        crossings[q] = 0;
        if (tr.status != ST_HIT || !tr.has_prev) continue;
        lt[q] = tr.lt;
        t[q] = tr.t;
        crossings[q] = count_crossings(f, mc, o, dir, tr.lt, tr.t, samples);
    }
    return 0;
}

/* ======================================================================== */
/* Gradients by forward-mode automatic differentiation (dual numbers).       */
/*                                                                           */
/* Parameter slots: 0-3 Julia c, 4 Mandelbulb power n, 5-8 plane 0 (raw      */
/* n xyz, d), 9-12 plane 1, 13 the ray parameter t (used only to get the     */
/* derivative of the distance along the ray).                                */
/*                                                                           */
/* For a refined hit the depth ts solves g(t*, theta) = d(o + t* dir; theta) */
/* - eps_abs - eps_rel t* = 0, so by the implicit function theorem           */
/*   dts/dtheta = -(dd/dtheta) / (dd/dt - eps_rel).                          */
/* The normal taps are then evaluated at points that carry that derivative,  */
/* and normal and colour follow by the chain rule through the same code as  */
/* the forward pass.  Cut-face pixels: t* = (d - n_hat.o)/(n_hat.dir) and    */
/* normal n_hat.  Exhausted, unrefined and jump hits get a zero Jacobian     */
/* (their depth is not a smooth root).  The shadow visibility is piecewise constant and    */
/* contributes no derivative.                                                */
/* ======================================================================== */
#define ND 14
typedef struct { double v; double g[ND]; } dual;

static dual dc(double v) { dual r; r.v = v; memset(r.g, 0, sizeof(r.g)); return r; }
static dual dseed(double v, int k) { dual r = dc(v); r.g[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.g[k] = a.g[k] + b.g[k]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.g[k] = a.g[k] - b.g[k]; return r; }
static dual dmul(dual a, dual b) {
    dual r; r.v = a.v * b.v;
    for (int k = 0; k < ND; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
    return r;
}
static dual ddiv(dual a, dual b) {
    dual r; r.v = a.v / b.v;
    for (int k = 0; k < ND; ++k) r.g[k] = (a.g[k] * b.v - a.v * b.g[k]) / (b.v * b.v);
    return r;
}
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < ND; ++k) r.g[k] = a.g[k] * s; return r; }
static dual daddc(dual a, double s) { a.v += s; return a; }
/* chain rule for a scalar function with value fv and derivative fd at a.v */
static dual dchain(dual a, double fv, double fd) {
    dual r; r.v = fv;
    for (int k = 0; k < ND; ++k) r.g[k] = fd * a.g[k];
    return r;
}
static dual dsqrt(dual a) { double s = sqrt(a.v); return dchain(a, s, 0.5 / s); }
static dual dlog(dual a) { return dchain(a, log(a.v), 1.0 / a.v); }
static dual dexp(dual a) { double e = exp(a.v); return dchain(a, e, e); }
static dual dsin(dual a) { return dchain(a, sin(a.v), cos(a.v)); }
static dual dcos(dual a) { return dchain(a, cos(a.v), -sin(a.v)); }
static dual dacos(dual a) { return dchain(a, acos(a.v), -1.0 / sqrt(1.0 - a.v * a.v)); }
static dual datan2(dual y, dual x) {
    dual r; r.v = atan2(y.v, x.v);
    double den = x.v * x.v + y.v * y.v;
    for (int k = 0; k < ND; ++k) r.g[k] = (x.v * y.g[k] - y.v * x.g[k]) / den;
    return r;
}

/* Quaternion square, product and integer power (R1) in dual arithmetic.   */
static void dquat_square(const dual z[4], dual out[4]) {
    dual vv = dadd(dadd(dmul(z[1], z[1]), dmul(z[2], z[2])), dmul(z[3], z[3]));
    dual a2 = dscale(z[0], 2.0);
    out[0] = dsub(dmul(z[0], z[0]), vv);
    out[1] = dmul(a2, z[1]);
    out[2] = dmul(a2, z[2]);
    out[3] = dmul(a2, z[3]);
}
static void dquat_mul(const dual x[4], const dual y[4], dual out[4]) {
    dual r0 = dsub(dmul(x[0], y[0]), dadd(dadd(dmul(x[1], y[1]), dmul(x[2], y[2])), dmul(x[3], y[3])));
    dual r1 = dadd(dadd(dmul(x[0], y[1]), dmul(y[0], x[1])), dsub(dmul(x[2], y[3]), dmul(x[3], y[2])));
    dual r2 = dadd(dadd(dmul(x[0], y[2]), dmul(y[0], x[2])), dsub(dmul(x[3], y[1]), dmul(x[1], y[3])));
    dual r3 = dadd(dadd(dmul(x[0], y[3]), dmul(y[0], x[3])), dsub(dmul(x[1], y[2]), dmul(x[2], y[1])));
    out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3;
}
static void dquat_pow(const dual z[4], int32_t p, dual out[4]) {
    dual w[4] = { z[0], z[1], z[2], z[3] };
    if (p >= 2) dquat_square(z, w);
    for (int32_t k = 3; k <= p; ++k) {
        dual t[4];
        dquat_mul(w, z, t);
        for (int i = 0; i < 4; ++i) w[i] = t[i];
    }
    for (int i = 0; i < 4; ++i) out[i] = w[i];
}
static dual dqlen2(const dual z[4]) {
    return dadd(dadd(dmul(z[0], z[0]), dmul(z[1], z[1])), dadd(dmul(z[2], z[2]), dmul(z[3], z[3])));
}

/* Julia distance in dual arithmetic, same steps as julia_de.  rel > 0
 * applies the rounding probe of perturbed_de to every power z^p.            */
static dual julia_de_dual(const or_fractal* f, const dual c[4], const dual p[3], int32_t* iters, double rel,
                          uint64_t seed, uint64_t key) {
    dual z[4] = { p[0], p[1], p[2], dc(0.0) };
    dual dz2 = dc(1.0), m2 = dc(0.0);
    int32_t n = 0;
    int32_t deg = julia_degree(f);
    for (int32_t i = 0; i < f->max_iter; ++i) {
        dual zq[4], zp[4];
        dquat_pow(z, deg - 1, zq);
        dz2 = dmul(dz2, dscale(dqlen2(zq), (double)deg * (double)deg));
        dquat_pow(z, deg, zp);
        if (rel != 0.0)
            for (int k = 0; k < 4; ++k) zp[k] = dscale(zp[k], noise(seed, key, i, k, rel));
        for (int k = 0; k < 4; ++k) z[k] = dadd(zp[k], c[k]);
        m2 = dqlen2(z);
        if (m2.v > f->bailout2) break;
        ++n;
    }
    if (iters) *iters = n;
    if (m2.v == 0.0) return dc(0.0);
    return dmul(dscale(dlog(m2), 0.25), dsqrt(ddiv(m2, dz2)));
}

/* Mandelbulb distance in dual arithmetic, same steps as bulb_de (rel as
 * for julia_de_dual, applied to every power w^n).                            */
static dual bulb_de_dual(const or_fractal* f, dual n, const dual p[3], int32_t* iters, double rel, uint64_t seed,
                         uint64_t key) {
    dual w[3] = { p[0], p[1], p[2] };
    dual m = dadd(dadd(dmul(w[0], w[0]), dmul(w[1], w[1])), dmul(w[2], w[2]));
    dual dr = dc(1.0);
    int32_t cnt = 0;
    for (int32_t i = 0; i < f->max_iter; ++i) {
        if (m.v == 0.0) {
            dr = dc(1.0);
            w[0] = p[0]; w[1] = p[1]; w[2] = p[2];
        } else {
            dual r = dsqrt(m);
            dual lr = dlog(r);
            dual rn1 = dexp(dmul(daddc(n, -1.0), lr));       /* r^(n-1) */
            dr = daddc(dmul(dmul(n, rn1), dr), 1.0);
            dual u = ddiv(w[1], r);
            if (u.v > 1.0) u = dc(1.0);
            if (u.v < -1.0) u = dc(-1.0);
            dual b = dmul(n, dacos(u));
            dual a = dmul(n, datan2(w[0], w[2]));
            dual rn = dexp(dmul(n, lr));                       /* r^n */
            dual sb = dsin(b);
            dual wn[3] = { dmul(rn, dmul(sb, dsin(a))), dmul(rn, dcos(b)), dmul(rn, dmul(sb, dcos(a))) };
            for (int k = 0; k < 3; ++k)
                w[k] = dadd(rel != 0.0 ? dscale(wn[k], noise(seed, key, i, k, rel)) : wn[k], p[k]);
        }
        m = dadd(dadd(dmul(w[0], w[0]), dmul(w[1], w[1])), dmul(w[2], w[2]));
        if (m.v > f->bailout2) break;
        ++cnt;
    }
    if (iters) *iters = cnt;
    if (m.v == 0.0) return dc(0.0);
    return ddiv(dmul(dscale(dlog(m), 0.25), dsqrt(m)), dr);
}

static dual fractal_de_dual(const or_fractal* f, const dual p[3], int32_t* iters) {
    if (f->kind == 0) {
        dual c[4];
        for (int k = 0; k < 4; ++k) c[k] = dseed(f->c[k], k);
        return julia_de_dual(f, c, p, iters, 0.0, 0, 0);
    }
    return bulb_de_dual(f, dseed(f->power, 4), p, iters, 0.0, 0, 0);
}

/* Gradient of the estimate with respect to the point (R10, mode 2): dual
 * numbers seeded on the three coordinates, the fractal parameters constant.
 * Returns the escape count.                                                 */
static int32_t analytic_gradient(const or_fractal* f, const double p[3], double rel, uint64_t seed, uint64_t key,
                                 double g[3]) {
    dual P[3] = { dseed(p[0], 0), dseed(p[1], 1), dseed(p[2], 2) };
    int32_t it = 0;
    dual d;
    if (f->kind == 0) {
        dual c[4];
        for (int k = 0; k < 4; ++k) c[k] = dc(f->c[k]);
        d = julia_de_dual(f, c, P, &it, rel, seed, key);
    } else {
        d = bulb_de_dual(f, dc(f->power), P, &it, rel, seed, key);
    }
    for (int k = 0; k < 3; ++k) g[k] = d.g[k];
    return it;
}

/* Jacobian rows per pixel: 0 depth, 1-3 normal, 4-6 colour; 13 columns
 * (slots 0-12).  Also returns the escape counts at p* and at every tap so
 * that the caller can build a mask of pixels whose branch structure is
 * unchanged under perturbation.  taps_iters has 7 entries per pixel
 * (p* first, then up to 6 taps; unused entries -1).                        */
int oracle_pixel_jacobian(const or_camera* cam, const or_fractal* f, const or_plane* planes, int32_t n_planes,
                          const or_march* mc, const int64_t* pix, int64_t n, int32_t n_threads,
                          double* jac, int32_t* tap_iters) {
    if (!cam || !f || !mc || !pix) return -1;
    /* the analytic normal's parameter derivative needs second derivatives of
     * the estimate, which first-order dual numbers do not carry */
    if (mc->normal_mode == 2) return -2;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t q = 0; q < n; ++q) {
        double* J = jac + q * 7 * 13;
        int32_t* TI = tap_iters ? tap_iters + q * 7 : NULL;
        memset(J, 0, sizeof(double) * 7 * 13);
        if (TI) for (int k = 0; k < 7; ++k) TI[k] = -1;
        int32_t i = (int32_t)(pix[q] % cam->width), j = (int32_t)(pix[q] / cam->width);
        pixel_result px;
        render_pixel(cam, f, planes, n_planes, mc, i, j, &px);
        int cls = px.status & 7;
        if (cls == ST_MISS_BOUNDS || cls == ST_MISS_TMAX || cls == ST_HIT_EXHAUSTED) continue;
        if (px.status & (ST_FLAG_UNREFINED | ST_FLAG_JUMP)) continue;
        double o[3], dir[3];
        oracle_camera_ray(cam, i, j, o, dir);
        double L[3] = { mc->light[0], mc->light[1], mc->light[2] };
        normalize3(L);
        double vis = (px.status & ST_FLAG_SHADOWED) ? 0.0 : 1.0;
        dual T, N[3];
        if (cls == ST_HIT_CUT) {
            int e = px.entry_plane;
            int base = 5 + 4 * e;
            dual nr[3] = { dseed(planes[e].n[0], base), dseed(planes[e].n[1], base + 1), dseed(planes[e].n[2], base + 2) };
            dual len = dsqrt(dadd(dadd(dmul(nr[0], nr[0]), dmul(nr[1], nr[1])), dmul(nr[2], nr[2])));
            for (int k = 0; k < 3; ++k) N[k] = ddiv(nr[k], len);
            dual dd = dseed(planes[e].d, base + 3);
            dual no = dadd(dadd(dscale(N[0], o[0]), dscale(N[1], o[1])), dscale(N[2], o[2]));
            dual nd = dadd(dadd(dscale(N[0], dir[0]), dscale(N[1], dir[1])), dscale(N[2], dir[2]));
            T = ddiv(dsub(dd, no), nd);
            if (TI) TI[0] = px.hit_iters;
        } else {
            /* implicit step at the refined root */
            double ts = px.depth;
            dual tt = dseed(ts, 13);
            dual p[3];
            for (int k = 0; k < 3; ++k) p[k] = daddc(dscale(tt, dir[k]), o[k]);
            int32_t it0;
            dual g = fractal_de_dual(f, p, &it0);
            if (TI) TI[0] = it0;
            double gt = g.g[13] - mc->eps_rel;
            T = dc(ts);
            for (int k = 0; k < 13; ++k) T.g[k] = -g.g[k] / gt;
            /* taps at points carrying dts/dtheta */
            dual eps = daddc(dscale(T, mc->eps_rel), mc->eps_abs);
            dual P[3];
            for (int k = 0; k < 3; ++k) P[k] = daddc(dscale(T, dir[k]), o[k]);
            dual G[3] = { dc(0), dc(0), dc(0) };
            if (mc->normal_mode == 0) {
                dual h = dscale(eps, 0.5773);
                for (int a = 0; a < 4; ++a) {
                    dual qv[3];
                    for (int k = 0; k < 3; ++k) qv[k] = dadd(P[k], dscale(h, TETRA[a][k]));
                    int32_t ita;
                    dual da = fractal_de_dual(f, qv, &ita);
                    if (TI) TI[1 + a] = ita;
                    for (int k = 0; k < 3; ++k) G[k] = dadd(G[k], dscale(da, TETRA[a][k]));
                }
            } else {
                dual h = eps;
                for (int k = 0; k < 3; ++k) {
                    dual qp[3] = { P[0], P[1], P[2] }, qm[3] = { P[0], P[1], P[2] };
                    qp[k] = dadd(qp[k], h);
                    qm[k] = dsub(qm[k], h);
                    int32_t itp, itm;
                    dual dp = fractal_de_dual(f, qp, &itp), dm = fractal_de_dual(f, qm, &itm);
                    if (TI) { TI[1 + 2 * k] = itp; TI[2 + 2 * k] = itm; }
                    G[k] = dsub(dp, dm);
                }
            }
            dual len = dsqrt(dadd(dadd(dmul(G[0], G[0]), dmul(G[1], G[1])), dmul(G[2], G[2])));
            if (len.v == 0.0) continue;
            for (int k = 0; k < 3; ++k) N[k] = ddiv(G[k], len);
        }
        dual ndl = dadd(dadd(dscale(N[0], L[0]), dscale(N[1], L[1])), dscale(N[2], L[2]));
        dual lam = dc(mc->k_ambient);
        if (ndl.v > 0.0) lam = dadd(lam, dscale(ndl, mc->k_diffuse * vis));
        for (int k = 0; k < 13; ++k) {
            J[0 * 13 + k] = T.g[k];
            for (int a = 0; a < 3; ++a) {
                J[(1 + a) * 13 + k] = N[a].g[k];
                J[(4 + a) * 13 + k] = mc->albedo[a] * lam.g[k];
            }
        }
    }
    return 0;
}
