"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, textbook maps, invariants, brute force and finite differences.  None
of them needs a GPU.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ---------------------------------------------------------------- quaternions
def _qmat(q):
    """Quaternion a+bi+cj+dk as the 2x2 complex matrix [[a+bi, c+di], [-c+di, a-bi]]."""
    a, b, c, d = q
    return np.array([[a + 1j * b, c + 1j * d], [-c + 1j * d, a - 1j * b]])


def test_quat_square_matches_matrix_representation(orc):
    rng = np.random.default_rng(10)
    for _ in range(200):
        q = rng.normal(size=4)
        m = _qmat(q) @ _qmat(q)
        ref = np.array([m[0, 0].real, m[0, 0].imag, m[0, 1].real, m[0, 1].imag])
        got = orc.quat_square(q)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
        assert abs(np.dot(got, got) - np.dot(q, q) ** 2) <= 1e-12 * np.dot(q, q) ** 2


def test_quat_product_matches_matrix_representation(orc):
    """General (non-commuting) products: the cross term of the Hamilton
    product is what a transposed operand or a sign slip would break."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        x, y = rng.normal(size=4), rng.normal(size=4)
        m = _qmat(x) @ _qmat(y)
        ref = np.array([m[0, 0].real, m[0, 0].imag, m[0, 1].real, m[0, 1].imag])
        np.testing.assert_allclose(orc.quat_mul(x, y), ref, rtol=1e-13, atol=1e-13)
    x, y = np.array([0.0, 1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0, 0.0])
    np.testing.assert_array_equal(orc.quat_mul(x, y), [0.0, 0.0, 0.0, 1.0])       # i j = k
    np.testing.assert_array_equal(orc.quat_mul(y, x), [0.0, 0.0, 0.0, -1.0])      # j i = -k


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8, 13])
def test_quat_power_matches_matrix_power(orc, p):
    rng = np.random.default_rng(13 + p)
    for _ in range(100):
        q = rng.normal(size=4) * 0.6
        m = np.linalg.matrix_power(_qmat(q), p)
        ref = np.array([m[0, 0].real, m[0, 0].imag, m[0, 1].real, m[0, 1].imag])
        got = orc.quat_pow(q, p)
        tol = 1e-13 * max(1.0, np.dot(q, q) ** (p / 2))
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=tol)


# ------------------------------------------------------------- Julia estimate
@pytest.mark.parametrize("max_iter,rmin", [(1, 0.3), (3, 0.3), (11, 0.95)])
def test_julia_c0_estimate_is_half_r_log_r(orc, max_iter, rmin):
    rng = np.random.default_rng(11 + max_iter)
    dirs = rng.normal(size=(500, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = rng.uniform(rmin, 3.0, size=500)
    pts = dirs * r[:, None]
    d, _, _, _ = orc.de(W.julia([0, 0, 0, 0], max_iter), pts)
    ref = GOLDEN["julia_c0"]["de_factor"] * r * np.log(r)
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("degree,max_iter,rmin", [(3, 3, 0.3), (3, 6, 0.9), (5, 3, 0.5), (7, 2, 0.3),
                                                  (16, 2, 0.7)])
def test_julia_degree_c0_estimate_is_half_r_log_r(orc, degree, max_iter, rmin):
    """c = 0, degree p: |z_k| = r^(p^k) and |z_k'| = p^k r^(p^k - 1), so
    0.5 |z| ln|z| / |z'| = 0.5 r ln r whatever p and k; the orbit escapes
    at the first k with r^(2 p^k) > bailout2."""
    rng = np.random.default_rng(40 + degree + max_iter)
    dirs = rng.normal(size=(500, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = rng.uniform(rmin, 3.0, size=500)
    pts = dirs * r[:, None]
    d, it, _, _ = orc.de(W.julia([0, 0, 0, 0], max_iter, degree=degree), pts)
    ref = GOLDEN["julia_c0"]["de_factor"] * r * np.log(r)
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-15)
    ref_it = np.full(r.size, max_iter)
    for i, ri in enumerate(r):
        for k in range(1, max_iter + 1):
            if 2.0 * degree ** k * math.log(ri) > math.log(256.0):
                ref_it[i] = k - 1
                break
    np.testing.assert_array_equal(it, ref_it)


def _complex_orbit(z0, c, max_iter, bailout2, degree=2):
    """Orbit of z -> z^p + c from z0, stopping as the estimator does."""
    z, n, bodies = z0, 0, 0
    for _ in range(max_iter):
        bodies += 1
        z = z ** degree + c
        if abs(z) ** 2 > bailout2:
            break
        n += 1
    return z, n, bodies


def _complex_iter_fixed(z0, c, bodies, degree=2):
    z = z0
    for _ in range(bodies):
        z = z ** degree + c
    return z


def _holomorphic_derivative(fn, z0, rho=1e-5, n=16):
    """f'(z0) by Cauchy's integral formula on the circle |z - z0| = rho,
    trapezoid rule with n nodes: exact up to the aliased Taylor terms
    a_(1+jn) rho^(jn) and a rounding error ~ 1e-16 max|f| / rho.
    Returns the derivative and a bound on that rounding error."""
    w = np.exp(2j * np.pi * np.arange(n) / n)
    vals = [fn(z0 + rho * wk) for wk in w]
    der = sum(v / wk for v, wk in zip(vals, w)) / (n * rho)
    return der, 64 * np.finfo(float).eps * max(abs(v) for v in vals) / rho


@pytest.mark.parametrize("axis,degree", [("ij", 2), ("k", 2), ("ij", 3), ("k", 3), ("ij", 4), ("ij", 6)])
def test_julia_complex_slice_matches_complex_dynamics(orc, axis, degree):
    """In span{1, u} the quaternion map is the complex map z^p+c' (a complex
    subalgebra), so orbit, escape count and running derivative must equal
    the complex ones; the derivative is checked against a contour-integral
    derivative of the complex orbit map."""
    rng = np.random.default_rng((21 if axis == "ij" else 22) + 100 * degree)
    if axis == "k":
        u = np.array([0.0, 0.0, 0.0, 1.0])      # the k axis: slice points must be real
    else:
        v = rng.normal(size=2)
        v /= np.linalg.norm(v)
        u = np.array([0.0, v[0], v[1], 0.0])
    c0, s = -0.3, 0.55
    c = np.array([c0, 0, 0, 0]) + s * u
    max_iter = {2: 11, 3: 8, 4: 6, 6: 5}[degree]
    fr = W.julia(c, max_iter, degree=degree)
    fr["c"] = list(c)                      # keep doubles for this pin
    for _ in range(60):
        x = rng.uniform(-1.5, 1.5)
        y = 0.0 if axis == "k" else rng.uniform(-1.5, 1.5)
        p = np.array([x, y * u[1], y * u[2]])
        d, it, m2, dz2 = (a[0] for a in orc.de(fr, p[None, :]))
        zN, n, bodies = _complex_orbit(complex(x, y), complex(c0, s), max_iter, 256.0, degree)
        assert it == n
        assert m2 == pytest.approx(abs(zN) ** 2, rel=1e-11)
        dzN, err = _holomorphic_derivative(lambda z: _complex_iter_fixed(z, complex(c0, s), bodies, degree),
                                           complex(x, y))
        rel = 1e-9 + err / abs(dzN)
        assert abs(math.sqrt(dz2) - abs(dzN)) <= rel * abs(dzN)
        ref_d = 0.5 * abs(zN) * math.log(abs(zN)) / abs(dzN)
        assert abs(d - ref_d) <= 2 * rel * abs(ref_d) + 1e-15


def test_julia_estimate_is_even(orc):
    """(-z)^2 = z^2 exactly, so the estimate is even, bit for bit."""
    rng = np.random.default_rng(30)
    pts = rng.uniform(-1.6, 1.6, size=(2000, 3))
    fr = W.julia(W.JULIA_C1, 11)
    a = orc.de(fr, pts)
    b = orc.de(fr, -pts)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# -------------------------------------------------------------- Mandelbulb map
def test_bulb_square_closed_form(orc):
    """n = 2 in Listing 7's axes: p^2 = (4xyz/rho, y^2 - rho^2, 2y(z^2 - x^2)/rho), rho = |(x, z)|."""
    rng = np.random.default_rng(40)
    for _ in range(300):
        x, y, z = rng.normal(size=3)
        rho = math.hypot(x, z)
        ref = np.array([4 * x * y * z / rho, y * y - rho * rho, 2 * y * (z * z - x * x) / rho])
        np.testing.assert_allclose(orc.bulb_power([x, y, z], 2.0), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 9, 16])
def test_bulb_integer_power_complex_form(orc, n):
    """Integer n: (y + i rho)^n = r^n e^(i n theta) and ((z + i x)/rho)^n = e^(i n phi)."""
    rng = np.random.default_rng(50 + n)
    for _ in range(200):
        w = rng.normal(size=3) * 0.7
        x, y, z = w
        rho = math.hypot(x, z)
        Y = complex(y, rho) ** n
        Z = (complex(z, x) / rho) ** n
        ref = np.array([Y.imag * Z.imag, Y.real, Y.imag * Z.real])
        scale = np.linalg.norm(w) ** n
        np.testing.assert_allclose(orc.bulb_power(w, float(n)), ref, rtol=1e-9, atol=1e-11 * scale)


@pytest.mark.parametrize("n", [2.3, 5.5, 8.0, 11.7])
def test_bulb_real_power_multiplies_angles(orc, n):
    """Real n: |p^n| = r^n and, where n*theta < pi and |n*phi| < pi, the polar
    and azimuthal angles of p^n are n*theta and n*phi (Eq. 1)."""
    rng = np.random.default_rng(int(n * 10))
    for _ in range(200):
        r = rng.uniform(0.2, 1.5)
        th = rng.uniform(0.01, math.pi / n - 0.01)
        ph = rng.uniform(-math.pi / n + 0.01, math.pi / n - 0.01)
        w = r * np.array([math.sin(th) * math.sin(ph), math.cos(th), math.sin(th) * math.cos(ph)])
        out = orc.bulb_power(w, n)
        rn = np.linalg.norm(out)
        assert rn == pytest.approx(r ** n, rel=1e-12)
        assert math.acos(out[1] / rn) == pytest.approx(n * th, rel=1e-9, abs=1e-12)
        assert math.atan2(out[0], out[2]) == pytest.approx(n * ph, rel=1e-9, abs=1e-12)


def test_bulb_polar_axis_is_the_real_quadratic_map(orc):
    """n = 2 on the polar axis: w -> (0, w_y^2, 0) + c, the real map x -> x^2 + c
    from x0 = c.  Short orbits agree to rounding; over 30 iterations rounding is
    amplified by the chaotic real map, so there only escape counts are compared."""
    rng = np.random.default_rng(60)
    ys = rng.uniform(-2.5, 0.6, size=200)

    def real_orbit(y, iters):
        x, n = y, 0
        for _ in range(iters):
            x = x * x + y
            if x * x > 4.0:
                break
            n += 1
        return x, n

    for iters in (1, 2, 4, 6):
        fr = W.bulb(2.0, iters)
        _, it, m2, _ = orc.de(fr, np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1))
        for k, y in enumerate(ys):
            x, n = real_orbit(y, iters)
            assert it[k] == n
            assert m2[k] == pytest.approx(x * x, rel=1e-10, abs=1e-14)
    fr = W.bulb(2.0, 30)
    _, it, _, _ = orc.de(fr, np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1))
    agree = np.mean([it[k] == real_orbit(y, 30)[1] for k, y in enumerate(ys)])
    assert agree >= 0.98


def test_bulb_axis_slice_is_mandelbrot_interval(orc):
    """n = 2, real axis: points of [-2, 1/4] stay bounded for 10^4 iterations,
    points outside escape (textbook real slice of the Mandelbrot set)."""
    lo, hi = GOLDEN["mandelbrot_real_axis"]["interval"]
    fr = W.bulb(2.0, 10000)
    fr["power"] = 2.0
    inside = np.linspace(lo + 1e-3, hi - 1e-3, 101)
    pts = np.stack([np.zeros_like(inside), inside, np.zeros_like(inside)], 1)
    assert np.all(orc.escape_iters(fr, pts, 10000) == 10000)
    outside = np.array([lo - 1e-2, lo - 1e-3, hi + 1e-2, hi + 1e-3, hi + 1e-4, 0.5, -2.5])
    pts = np.stack([np.zeros_like(outside), outside, np.zeros_like(outside)], 1)
    assert np.all(orc.escape_iters(fr, pts, 10000) < 10000)


@pytest.mark.parametrize("n", [3, 8])
def test_bulb_rotational_symmetry(orc, n):
    """Integer n: rotation by 2 pi/(n-1) about the polar axis commutes with the
    map, (R p)^n + R c = R (p^n + c), so the estimate is invariant."""
    a = 2 * math.pi / (n - 1)
    rng = np.random.default_rng(70 + n)
    pts = rng.uniform(-1.2, 1.2, size=(2000, 3))
    rot = np.stack([pts[:, 0] * math.cos(a) + pts[:, 2] * math.sin(a), pts[:, 1],
                    pts[:, 2] * math.cos(a) - pts[:, 0] * math.sin(a)], 1)
    fr = W.bulb(float(n), 10)
    d0, i0, _, _ = orc.de(fr, pts)
    d1, i1, _, _ = orc.de(fr, rot)
    same = i0 == i1
    assert same.mean() > 0.99
    np.testing.assert_allclose(d1[same], d0[same], rtol=1e-7, atol=1e-10)


# --------------------------------------------------------------- escape radii
def test_bound_radius_values(orc):
    assert orc.bound_radius(W.julia([0, 0, 0, 0], 11)) == pytest.approx(1.0, rel=1e-15)
    assert orc.bound_radius(W.julia([0, 0, 0, 0], 11, bound_radius=1.5)) == 1.5
    assert orc.bound_radius(W.bulb(8.0, 10, bound_radius=0.5)) == pytest.approx(2 ** (1 / 7), rel=1e-15)
    assert orc.bound_radius(W.bulb(2.0, 10)) == pytest.approx(2.0, rel=1e-15)
    assert orc.bound_radius(W.bulb(8.0, 10)) == pytest.approx(2 ** (1 / 7), rel=1e-15)
    c = W.JULIA_C1
    cn = math.sqrt(sum(x * x for x in c))
    R = orc.bound_radius(W.julia(c, 11))
    assert R * R - R - cn == pytest.approx(0.0, abs=1e-14)


@pytest.mark.parametrize("degree", [3, 4, 5, 7])
def test_julia_degree_bound_radius_is_the_tight_escape_radius(orc, degree):
    """R solves R^p - R - |c| = 0; for c = -|c| on the real axis the point
    (R, 0, 0) is a fixed point of x^p - |c| (x^p - |c| = x), so just inside R
    the orbit stays put for a few bodies while just outside it escapes."""
    for cn in (0.0, 0.2, 0.7, 1.3):
        fr = W.julia([-cn, 0, 0, 0], 6, degree=degree)
        fr["c"] = [-cn, 0.0, 0.0, 0.0]
        R = orc.bound_radius(fr)
        assert R >= 1.0
        assert abs(R ** degree - R - cn) <= 1e-13 * R ** degree
        assert orc.escape_iters(fr, np.array([[R * (1.0 - 1e-13), 0.0, 0.0]]), 6)[0] == 6
        assert orc.escape_iters(fr, np.array([[R * (1.0 + 1e-9), 0.0, 0.0]]), 10000)[0] < 10000


@pytest.mark.parametrize("kind", ["julia", "bulb"])
def test_points_beyond_bound_radius_escape(orc, kind):
    rng = np.random.default_rng(80)
    for trial in range(20):
        if kind == "julia":
            fr = W.julia(rng.uniform(-0.8, 0.8, size=4), 10000, degree=int(rng.integers(2, 8)))
        else:
            fr = W.bulb(rng.uniform(2.0, 16.0), 10000)
        R = orc.bound_radius(fr)
        dirs = rng.normal(size=(20, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        pts = dirs * R * 1.01
        assert np.all(orc.escape_iters(fr, pts, 10000) < 10000)


# ----------------------------------------------------- the c = 0 ball renders
def _ball_job(width=96, height=96, eps_abs=1e-3, eps_rel=0.0, normal_mode="tetra", planes=(), shadow=False,
              bound_radius=1.5):
    """c = 0 Julia view.  The provable escape radius (1) lies inside the
    eps-level sphere, so a looser caller radius is given to make the rays
    march from outside it."""
    jb = W.julia_view(c=[0, 0, 0, 0], width=width, height=height, eps_abs=eps_abs, planes=planes,
                      shadow=shadow, normal_mode=normal_mode)
    jb["march"]["eps_rel"] = W.f32(eps_rel)
    jb["fractal"]["bound_radius"] = W.f32(bound_radius)
    return jb


def _rho(eps):
    return brentq(lambda r: 0.5 * r * math.log(r) - eps, 1.0, 2.0, xtol=1e-15)


@pytest.mark.parametrize("normal_mode", ["tetra", "central", "analytic"])
def test_c0_ball_hit_depth_normal_colour(orc, normal_mode):
    """c = 0: the estimate is 0.5 r ln r, the eps-level set is the sphere of
    radius rho_eps, so the refined depth is the ray's entry into it, the hit
    mask is 'closest approach < rho_eps', the normal is radial and the colour
    is Lambert of the radial normal."""
    jb = _ball_job(normal_mode=normal_mode)
    eps = jb["march"]["eps_abs"]
    rho = _rho(eps)
    out = orc.render(jb)
    n = 96 * 96
    o, d = orc.camera_rays(jb["camera"], np.arange(n))
    b_par = np.einsum("ij,ij->i", o, d)
    b2 = np.einsum("ij,ij->i", o, o) - b_par ** 2
    b = np.sqrt(np.maximum(b2, 0))
    cls = out["status"] & 7
    clear = np.abs(b - rho) > 3e-3
    assert np.all((cls[clear] == orc.STATUS_HIT) == (b[clear] < rho))
    hit = clear & (b < rho)
    assert hit.sum() > 1000
    t_ref = -b_par[hit] - np.sqrt(b_par[hit] ** 2 - (np.einsum("ij,ij->i", o, o)[hit] - rho * rho))
    np.testing.assert_allclose(out["depth"][hit], t_ref, atol=1e-9)
    p = o[hit] + out["depth"][hit, None] * d[hit]
    nref = p / np.linalg.norm(p, axis=1, keepdims=True)
    cosang = np.clip(np.einsum("ij,ij->i", out["normal"][:, hit].T, nref), -1, 1)
    assert np.max(np.arccos(cosang)) < (1e-7 if normal_mode == "analytic" else 1e-5)
    L = np.array(jb["march"]["light_dir"], dtype=np.float64)
    L /= np.linalg.norm(L)
    lam = jb["march"]["k_ambient"] + jb["march"]["k_diffuse"] * np.maximum(0, nref @ L)
    np.testing.assert_allclose(out["colour"][0, hit], lam, atol=1e-6)
    miss = clear & (b >= rho)
    assert np.all(out["depth"][miss] == -1.0) and np.all(out["colour"][:, miss] == 0.0)


def test_c0_ball_brackets_hold_one_crossing(orc):
    """c = 0: d - eps falls monotonically through the eps-level sphere, so
    every refinable hit's final bracket holds exactly one crossing and the
    refined depth lies inside it."""
    jb = _ball_job()
    out = orc.render(jb)
    hit = np.nonzero(((out["status"] & 7) == orc.STATUS_HIT) & ((out["status"] & orc.FLAG_UNREFINED) == 0))[0]
    assert hit.size > 1000
    lt, t, cr = orc.bracket_crossings(jb, hit)
    assert np.all(cr == 1)
    assert np.all((lt <= out["depth"][hit]) & (out["depth"][hit] <= t))


def test_c0_ball_relative_eps_depth(orc):
    """eps = eps_rel * t: the refined depth solves 0.5 r(t) ln r(t) = eps_rel t."""
    jb = _ball_job(width=48, height=48, eps_abs=0.0, eps_rel=5e-4)
    out = orc.render(jb)
    o, d = orc.camera_rays(jb["camera"], np.arange(48 * 48))
    cls = out["status"] & 7
    checked = 0
    er = jb["march"]["eps_rel"]
    for k in np.nonzero(cls == orc.STATUS_HIT)[0]:
        f = lambda t: 0.5 * np.linalg.norm(o[k] + t * d[k]) * math.log(np.linalg.norm(o[k] + t * d[k])) - er * t
        bpar = -np.dot(o[k], d[k])
        if f(bpar) > -1e-4:           # grazing: skip
            continue
        t_ref = brentq(f, 1.0, bpar, xtol=1e-14)
        assert out["depth"][k] == pytest.approx(t_ref, abs=1e-9)
        checked += 1
    assert checked > 300


def test_c0_ball_shadow_is_never_cast_on_lit_side(orc):
    """The ball is convex: a shadow ray from a lit point never hits it again,
    so shadows change nothing."""
    a = orc.render(_ball_job(shadow=False))
    b = orc.render(_ball_job(shadow=True))
    assert not np.any(b["status"] & orc.FLAG_SHADOWED)
    np.testing.assert_array_equal(a["colour"], b["colour"])


def test_c0_ball_cut_face_closed_form(orc):
    """Ball cut by z <= 0.3 seen from z = 3: rays cross the plane first; the
    face is the disk |p0| < rho_eps, depth (d - n.o)/(n.dir), normal +z."""
    pl = W.plane([0.0, 0.0, 3.0], 0.3)       # raw normal, normalised by the renderer
    jb = _ball_job(planes=[pl])
    rho = _rho(jb["march"]["eps_abs"])
    out = orc.render(jb)
    o, d = orc.camera_rays(jb["camera"], np.arange(96 * 96))
    t0 = (pl["d"] - o[:, 2]) / d[:, 2]
    p0 = o + t0[:, None] * d
    r0 = np.linalg.norm(p0, axis=1)
    cls = out["status"] & 7
    clear = (r0 < 0.999) | (r0 > rho + 1e-3)
    inside = clear & (r0 < 0.999)
    assert inside.sum() > 500
    assert np.all(cls[inside] == orc.STATUS_HIT_CUT)
    assert np.all(cls[clear & ~inside] != orc.STATUS_HIT_CUT)
    np.testing.assert_allclose(out["depth"][inside], t0[inside], rtol=1e-14)
    np.testing.assert_allclose(out["normal"][:, inside].T, np.tile([0, 0, 1.0], (inside.sum(), 1)), atol=0)
    # the same plane with a unit normal renders identically
    out2 = orc.render(_ball_job(planes=[W.plane([0.0, 0.0, 1.0], 0.3)]))
    np.testing.assert_array_equal(out["status"], out2["status"])
    np.testing.assert_allclose(out["depth"], out2["depth"], rtol=1e-14)


# --------------------------------------------------------------- march pins
def test_refined_depth_is_a_root(orc):
    jb = W.julia_view(width=64, height=64)
    out = orc.render(jb)
    hit = (out["status"] == orc.STATUS_HIT)
    o, d = orc.camera_rays(jb["camera"], np.nonzero(hit)[0])
    p = o + out["depth"][hit, None] * d
    dv, _, _, _ = orc.de(jb["fractal"], p)
    assert hit.sum() > 1000
    off = np.abs(dv - jb["march"]["eps_abs"]) >= 1e-9
    assert off.mean() < 0.01
    # the estimate is discontinuous where the escape count changes; a root
    # bracket around such a jump converges onto the jump itself
    for k in np.nonzero(off)[0]:
        pa = o[k] + (out["depth"][hit][k] - 1e-11) * d[k]
        pb = o[k] + (out["depth"][hit][k] + 1e-11) * d[k]
        ia = orc.de(jb["fractal"], pa[None])[1][0]
        ib = orc.de(jb["fractal"], pb[None])[1][0]
        assert ia != ib


def test_julia_render_is_symmetric_under_point_reflection(orc):
    """Rendering from -eye (up kept +y) shoots exactly the negated rays of the
    vertically flipped image; the estimate is even, so the images agree."""
    jb = W.julia_view(width=64, height=64)
    jb2 = W.julia_view(width=64, height=64, eye=(0.0, 0.0, -3.0))
    a = orc.render(jb)
    b = orc.render(jb2)
    sa = a["status"].reshape(64, 64)
    sb = b["status"].reshape(64, 64)[::-1]
    assert (sa != sb).mean() <= 1e-3
    same = (sa == sb) & ((sa & 7) == orc.STATUS_HIT)
    np.testing.assert_allclose(a["depth"].reshape(64, 64)[same], b["depth"].reshape(64, 64)[::-1][same], atol=1e-9)


def _bounded_along(orc, fr, o, d, t_lo, t_hi, step, nb, planes=()):
    ts = np.arange(t_lo, t_hi, step)
    if ts.size == 0:
        return 0
    pts = o[None, :] + ts[:, None] * d[None, :]
    for pl in planes:
        nh = np.array(pl["n"], dtype=np.float64)
        nh /= np.linalg.norm(nh)
        pts = pts[pts @ nh <= pl["d"]]
    if pts.shape[0] == 0:
        return 0
    g = dict(fr)
    g["max_iter"] = nb
    _, it, _, _ = orc.de(g, pts)
    return int(np.sum(it == nb))


@pytest.mark.parametrize("case", ["julia", "julia_cut", "bulb"])
def test_march_never_passes_a_bounded_point(orc, case):
    """Brute force on tiny images: sample every eps/4 along each ray up to the
    refined hit (or through the whole interval for misses); no sample may be
    a bounded point (no escape within max(200, 8N) iterations)."""
    if case == "julia":
        jb = W.julia_view(width=12, height=12)
    elif case == "julia_cut":
        jb = W.julia_view(width=12, height=12, planes=[W.plane([0.3, 0.2, 1.0], 0.05)])
    else:
        jb = W.bulb_view(0.7, 0.2, width=10, height=10, shadow=False)
    fr, mc = jb["fractal"], jb["march"]
    nb = max(200, 8 * fr["max_iter"])
    out = orc.render(jb)
    n = jb["camera"]["width"] * jb["camera"]["height"]
    o, d = orc.camera_rays(jb["camera"], np.arange(n))
    R = orc.bound_radius(fr)
    bad = 0
    for k in range(n):
        bp = np.dot(o[k], d[k])
        disc = bp * bp - (np.dot(o[k], o[k]) - R * R)
        if disc <= 0:
            continue
        t_in, t_out = -bp - math.sqrt(disc), -bp + math.sqrt(disc)
        cls = out["status"][k] & 7
        if cls == orc.STATUS_HIT:
            t_end = out["depth"][k]
        elif cls in (orc.STATUS_MISS_TMAX, orc.STATUS_MISS_BOUNDS):
            t_end = t_out
        else:
            continue
        eps = mc["eps_abs"] + mc["eps_rel"] * t_end
        bad += _bounded_along(orc, fr, o[k], d[k], max(t_in, 0.0), t_end - eps / 4, eps / 4, nb, jb["planes"])
    assert bad == 0


# ----------------------------------------------- analytic normals (R10, mode 2)
@pytest.mark.parametrize("degree", [2, 3, 5])
def test_analytic_normal_c0_is_radial(orc, degree):
    """c = 0: d = 0.5 r ln r depends on r alone, so its gradient is radial
    (three bodies keep |z|^(p^k) well inside double range)."""
    rng = np.random.default_rng(60 + degree)
    pts = rng.normal(size=(500, 3))
    pts *= (rng.uniform(0.85, 1.4, size=500) / np.linalg.norm(pts, axis=1))[:, None]
    ref = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    fr = W.julia([0, 0, 0, 0], 3, degree=degree)
    n = orc.normal_at(fr, pts, -ref, np.full(500, 1e-3), "analytic")
    assert np.max(np.linalg.norm(n - ref, axis=1)) < 1e-12


ANALYTIC_CASES = {
    "julia": W.julia(W.JULIA_C1, 11),
    "julia3": W.julia(W.JULIA_C3, 9, degree=3),
    "bulb8": W.bulb(8.0, 10),
    "bulb5": W.bulb(5.0, 10),
    "bulb_real": W.bulb(6.37, 10),
}


@pytest.mark.parametrize("name", sorted(ANALYTIC_CASES))
def test_analytic_normal_matches_converged_differences(orc, name):
    """The dual-number gradient of the estimate against Richardson-
    extrapolated central differences of the plain FP64 estimate (a different
    code path), on points whose escape count is the same at every stencil
    point and whose quotients at h and h/2 agree to 1e-4 (near the polar
    axis the bulb's map has large higher derivatives)."""
    fr = ANALYTIC_CASES[name]
    rng = np.random.default_rng(3)
    R = orc.bound_radius(fr)
    dirs = rng.normal(size=(3000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = dirs * R * rng.uniform(0.5, 1.0, size=(3000, 1))
    d, it, _, _ = orc.de(fr, pts)
    mg, esc = orc.escape_margin(fr, pts)
    ok = esc & (mg > 1e-3) & (d > 1e-3)

    def quotient(h):
        g = np.zeros_like(pts)
        same = np.ones(len(pts), bool)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            dp, ip, _, _ = orc.de(fr, pts + e)
            dm, im, _, _ = orc.de(fr, pts - e)
            g[:, k] = (dp - dm) / (2 * h)
            same &= (ip == it) & (im == it)
        return g, same

    g1, s1 = quotient(1e-4)
    g2, s2 = quotient(5e-5)
    conv = np.linalg.norm(g1 - g2, axis=1) <= 1e-4 * np.linalg.norm(g2, axis=1)
    ok &= s1 & s2 & conv
    assert ok.sum() > 1000
    g = (4 * g2 - g1) / 3
    gn = g / np.linalg.norm(g, axis=1, keepdims=True)
    n = orc.normal_at(fr, pts, -dirs, np.full(len(pts), 1e-3), "analytic")
    ang = np.arccos(np.clip(np.einsum("ij,ij->i", n[ok], gn[ok]), -1, 1))
    assert ang.max() < 1e-5, ang.max()


def test_analytic_normal_jacobian_is_not_provided(orc):
    jb = W.julia_view(width=8, height=8, normal_mode="analytic")
    with pytest.raises(NotImplementedError):
        orc.pixel_jacobian(jb, np.arange(64))


@pytest.mark.parametrize("degree", [2, 3, 5])
def test_escape_margin_julia_c0_closed_form(orc, degree):
    """With c = 0 the orbit of x is x^(p^k), so |z_k|^2 = |x|^(2 p^k): the
    margin is the smallest |m_k - B| / B up to the first m_k > B."""
    fr = W.julia([0, 0, 0, 0], max_iter=9, bailout2=256.0, degree=degree)
    rng = np.random.default_rng(5)
    pts = rng.normal(size=(200, 3)) * rng.uniform(0.5, 1.6, size=(200, 1))
    margin, esc = orc.escape_margin(fr, pts)
    for p, mg, e in zip(pts, margin, esc):
        m0, B = float(p @ p), 256.0
        best, escaped = np.inf, False
        for k in range(1, 10):
            mk = m0 ** (degree ** k)
            best = min(best, abs(mk - B) / B)
            if mk > B:
                escaped = True
                break
        assert e == escaped
        assert mg == pytest.approx(best, rel=1e-9, abs=1e-12)


def test_escape_margin_bulb_polar_axis(orc):
    """On the polar (y) axis the n = 8 Mandelbulb map sends (0, y, 0) to
    (0, |y|^8, 0) (theta is 0 or pi, and 8 theta a multiple of 2 pi), so the
    orbit follows the 1-D recurrence y <- |y|^8 + y0."""
    fr = W.bulb(8.0, 10)
    ys = np.linspace(-1.3, 1.3, 131)
    pts = np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1)
    margin, esc = orc.escape_margin(fr, pts)
    B = float(fr["bailout2"])
    for y0, mg, e in zip(ys, margin, esc):
        y, best, escaped = y0, np.inf, False
        for _ in range(10):
            y = abs(y) ** 8 + y0
            best = min(best, abs(y * y - B) / B)
            if y * y > B:
                escaped = True
                break
        assert e == escaped, y0
        assert mg == pytest.approx(best, rel=1e-9, abs=1e-12), y0


# ------------------------------------------------- Mandelbulb running derivative
def _axis_map_complex_step(y0, n, max_iter, bailout2, h=1e-30):
    """The real map y <- y^n + c from y = c (c = y0 > 0), run with c = y0 + i h
    (complex step): Re(y) is the orbit, Im(y)/h its exact c-derivative to
    rounding, with no difference quotient.  Returns (y, dy/dc, bodies that
    stayed within the bailout)."""
    c = complex(y0, h)
    y, k = c, 0
    for _ in range(max_iter):
        y = y ** n + c
        if y.real * y.real > bailout2:
            break
        k += 1
    return y.real, y.imag / h, k


@pytest.mark.parametrize("n", [2.0, 5.0, 8.0, 6.37])
def test_bulb_running_derivative_is_the_axis_map_c_derivative(orc, n):
    """On the positive polar axis, c = (0, y0, 0) with y0 > 0, every body has
    theta = 0, so w^n = (0, r^n, 0) and the orbit is the real map y <- y^n + c
    started at y = c (Listing 7 starts the orbit at the point itself).  The
    running derivative dr <- n r^(n-1) dr + 1, dr = 1 (Sec. 2, Eq. 4 in norm,
    with the +1 of the added point) is then exactly the c-derivative of that
    map, which the test takes by complex step; the estimate is
    d = 0.5 |y| ln|y| / y' (the constant of Listings 4 and 7).  n = 2 with
    c in (0, 1/4] stays bounded (the Mandelbrot interval), so the estimate
    there is negative; larger c and n = 5, 8 cover every escape body."""
    if n == 2.0:
        ys = np.concatenate([np.linspace(0.01, 0.25, 25), np.linspace(0.26, 1.2, 48)])
    else:
        ys = np.linspace(0.02, 1.2, 119)
    for max_iter in (1, 3, 10, 15):
        fr = W.bulb(n, max_iter)
        B = float(fr["bailout2"])
        pts = np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1)
        d, it, m2, dr = orc.de(fr, pts)
        bodies = set()
        for k, y0 in enumerate(ys):
            y, dy, esc = _axis_map_complex_step(float(y0), float(fr["power"]), max_iter, B)
            bodies.add(esc)
            assert it[k] == esc, (n, max_iter, y0)
            assert m2[k] == pytest.approx(y * y, rel=1e-11), (n, max_iter, y0)
            assert dr[k] == pytest.approx(dy, rel=1e-11), (n, max_iter, y0)
            assert d[k] == pytest.approx(0.5 * abs(y) * math.log(abs(y)) / dy, rel=1e-10, abs=1e-300), (n, max_iter, y0)
        if max_iter >= 10:
            # the sample reaches escapes after 1, 2, ... bodies and non-escapes
            assert len(bodies) >= 4, (n, max_iter, sorted(bodies))


def test_bulb_running_derivative_is_not_the_orbit_derivative_without_the_plus_one(orc):
    """The +1 of the recurrence is the derivative of the added point: for
    the Mandelbulb the point is both the start and the constant.  Without it
    dr would be prod n r_k^(n-1), the derivative of the map with c held
    fixed.  On the axis with n = 2, one body from y0: dr = 2 y0 + 1 (with),
    against 2 y0 (without)."""
    ys = np.linspace(0.05, 1.3, 26)
    fr = W.bulb(2.0, 1)
    _, _, _, dr = orc.de(fr, np.stack([np.zeros_like(ys), ys, np.zeros_like(ys)], 1))
    np.testing.assert_allclose(dr, 2.0 * ys + 1.0, rtol=1e-14)


# ---------------------------------------------------------- rounding probes
@pytest.mark.parametrize("rel", [2.0 ** -20, 1e-3, 0.25])
def test_probe_noise_is_uniform_on_the_stated_interval(orc, rel):
    """The probes' factor is uniform on [1 - rel, 1 + rel]: range, mean,
    variance rel^2/3, a Kolmogorov-Smirnov test, and no correlation between
    neighbouring components, bodies and points."""
    from scipy import stats as sst
    keys = [(s, p, b, c) for s in (1000, 1003) for p in range(40) for b in range(5) for c in range(4)]
    v = np.array([orc.probe_noise(s, p, b, c, rel) for s, p, b, c in keys])
    assert v.min() >= 1.0 - rel and v.max() <= 1.0 + rel
    u = (v - (1.0 - rel)) / (2.0 * rel)
    N = u.size
    assert abs(u.mean() - 0.5) < 4.0 * math.sqrt(1.0 / 12.0 / N)
    assert abs(u.var() - 1.0 / 12.0) < 0.1 / 12.0
    assert sst.kstest(u, "uniform").pvalue > 1e-3
    grid = u.reshape(2, 40, 5, 4)
    for ax in (1, 2, 3):
        a = np.moveaxis(grid, ax, -1)
        r = np.corrcoef(a[..., :-1].ravel(), a[..., 1:].ravel())[0, 1]
        assert abs(r) < 0.1, (ax, r)
    # same key, same draw; another seed, another draw
    assert orc.probe_noise(7, 3, 2, 1, rel) == orc.probe_noise(7, 3, 2, 1, rel)
    assert orc.probe_noise(7, 3, 2, 1, rel) != orc.probe_noise(8, 3, 2, 1, rel)


@pytest.mark.parametrize("kind", ["julia", "cubic", "bulb8", "bulb_real"])
@pytest.mark.parametrize("mode", ["tetra", "central", "analytic"])
def test_probes_at_zero_perturbation_are_the_plain_functions(orc, kind, mode):
    """With rel = 0 every factor is exactly 1, so the perturbed normal and
    trap must reproduce normal_at and orbit_trap bit for bit; and as rel
    shrinks the perturbed normal must converge to the plain one."""
    fr = {"julia": W.julia([-0.2, 0.6, 0.2, 0.2], max_iter=11), "cubic": W.julia([-0.45, 0.1, 0.4, 0.2], 10, degree=3),
          "bulb8": W.bulb(8.0, 10), "bulb_real": W.bulb(6.37, 10)}[kind]
    rng = np.random.default_rng(17)
    pts = rng.normal(size=(300, 3))
    pts *= (rng.uniform(0.6, 1.3, size=(300, 1)) / np.linalg.norm(pts, axis=1, keepdims=True))
    dirs = -pts / np.linalg.norm(pts, axis=1, keepdims=True)
    eps = np.full(300, 1e-3)
    ref = orc.normal_at(fr, pts, dirs, eps, mode)
    np.testing.assert_array_equal(orc.normal_perturbed(fr, pts, dirs, eps, mode, 0.0, 1234), ref)
    np.testing.assert_array_equal(orc.orbit_trap_perturbed(fr, pts, 0.0, 1234), orc.orbit_trap(fr, pts))
    from parity import angle
    prev = None
    for rel in (1e-6, 1e-9, 1e-12):
        a = np.median(angle(orc.normal_perturbed(fr, pts, dirs, eps, mode, rel, 99), ref))
        if prev is not None:
            assert a <= prev * 0.1 + 1e-15, (rel, a, prev)
        prev = a
    assert prev < 1e-6
