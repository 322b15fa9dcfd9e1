"""Host-side checks of the numerical building blocks that need no GPU.

1. The normal-tap tables: the tetrahedral taps of Eq. 5 (Sec. 2) and the
   central-difference taps.  Their first and second moments (sum of the taps
   zero, sum of nu nu^T a multiple of the identity) are what make the
   weighted tap sum a gradient estimate; the oracle's C normal estimator is
   then tied to these tables by recomputing its normals from its own
   distance estimates at the tap points.
2. The library's fast acos / atan polynomials (the float32 coefficients
   written in the kernel header): evaluated here in double and in emulated
   float32 against numpy's double-precision libm, over dense grids of
   [-1, 1] and of the four quadrants, with the special cases the kernels
   rely on (atan2(0, 0) = 0, signed zeros, the endpoints).  The fitting
   script is re-run and must give the same float32 coefficients.
"""
import os
import re
import sys

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_01747_amd", "csrc")
MATH_HPP = os.path.join(CSRC, "frt_math.hpp")


# ---------------------------------------------------------------- taps
def test_tetra_tap_moments(orc):
    T = orc.TETRA_TAPS
    assert T.shape == (4, 3)
    np.testing.assert_array_equal(T.sum(axis=0), 0.0)
    # sum of nu_x nu over the taps is (4, 0, 0), and likewise per axis
    np.testing.assert_array_equal(T.T @ T, 4.0 * np.eye(3))
    # vertices of a regular tetrahedron: equal length, pairwise dot -1
    G = T @ T.T
    np.testing.assert_array_equal(np.diag(G), 3.0)
    np.testing.assert_array_equal(G[~np.eye(4, dtype=bool)], -1.0)


def test_central_tap_moments(orc):
    C = orc.CENTRAL_TAPS
    assert C.shape == (6, 3)
    np.testing.assert_array_equal(C.sum(axis=0), 0.0)
    np.testing.assert_array_equal(C.T @ C, 2.0 * np.eye(3))


def test_tap_sum_recovers_linear_gradient(orc):
    """With these moments the weighted tap sum of a linear function a.x + b
    is exactly a scaled: sum nu (a . (p + h nu) + b) = h (T^T T) a, that is
    4 h a for the tetrahedral and 2 h a for the central taps."""
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=3), rng.normal()
    p = rng.normal(size=(5, 3))
    for mode, T, scale in (("tetra", orc.TETRA_TAPS, 4.0), ("central", orc.CENTRAL_TAPS, 2.0)):
        eps = np.full(5, 1e-3)
        q = orc.tap_points(p, eps, mode)                  # [5, taps, 3]
        h = np.linalg.norm(q[:, 0] - p, axis=1) / np.linalg.norm(T[0])
        g = np.einsum("tk,nt->nk", T, q @ a + b)
        np.testing.assert_allclose(g, scale * h[:, None] * a[None], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("mode", ["tetra", "central"])
@pytest.mark.parametrize("kind", ["julia", "bulb"])
def test_oracle_normal_uses_the_tap_tables(orc, mode, kind):
    """The C normal estimator equals the normalised tap sum of the C distance
    estimate at the tap points formed from the moment-checked tables."""
    fr = (W.julia_view() if kind == "julia" else W.bulb_view(0.4, 0.25))["fractal"]
    rng = np.random.default_rng(11)
    p = rng.uniform(-1.2, 1.2, size=(64, 3))
    eps = rng.uniform(1e-4, 1e-2, size=64)
    dirs = np.tile([0.0, 0.0, 1.0], (64, 1))
    n = orc.normal_at(fr, p, dirs, eps, mode)
    q = orc.tap_points(p, eps, mode)
    d = orc.de(fr, q.reshape(-1, 3))[0].reshape(q.shape[:2])
    T = orc.TETRA_TAPS if mode == "tetra" else orc.CENTRAL_TAPS
    g = np.einsum("tk,nt->nk", T, d)
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    np.testing.assert_allclose(n, g, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- fast acos / atan
def _coefficients(fn):
    """Horner coefficients (highest degree first) of the polynomial in the
    body of the named device function of the kernel math header."""
    src = open(MATH_HPP).read()
    body = src[src.index(fn + "("):]
    body = body[:body.index("\n}\n")]
    lit = r"(-?\d\.\d+e[+-]\d+)f"
    first = re.search(r"float [pq] = " + lit + ";", body)
    rest = re.findall(r"fmaf\([pq], \w+, " + lit + r"\)", body)
    assert first is not None and len(rest) >= 6
    return np.array([float(first.group(1))] + [float(v) for v in rest], dtype=np.float32)


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _fma32(a, b, c):
    # a*b of two float32 values is exact in double; one rounding of the sum
    # to double and one to float32 (double rounding is at most 1/2 ulp more)
    return _f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def _horner32(c, x):
    r = np.full_like(x, c[0], dtype=np.float32)
    for v in c[1:]:
        r = _fma32(r, x, np.float32(v))
    return r


def _acos32(x):
    c = _coefficients("fast_acos")
    ax = np.abs(x)
    r = _f32(np.sqrt(_f32(np.float32(1.0) - ax).astype(np.float64))) * _horner32(c, ax)
    r = r.astype(np.float32)
    return np.where(x < 0, _f32(np.float32(np.pi) - r), r)


def _atan2_32(y, x):
    c = _coefficients("fast_atan2")
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(mx > 0, _f32(mn.astype(np.float64) / mx.astype(np.float64)), np.float32(0.0)).astype(np.float32)
    r = (s * _horner32(c, (s * s).astype(np.float32))).astype(np.float32)
    r = np.where(ay > ax, _f32(np.float32(np.pi / 2) - r), r)
    r = np.where(x < 0, _f32(np.float32(np.pi) - r), r)
    return np.copysign(r, y).astype(np.float32)


def test_acos_polynomial_error():
    c = _coefficients("fast_acos").astype(np.float64)
    assert c.size == 8
    x = np.linspace(0.0, 1.0, 2_000_001)
    pd = np.polyval(c, x)
    # the header's bound for the float32 coefficients evaluated in double
    assert np.max(np.abs(np.sqrt(1.0 - x) * pd - np.arccos(x))) < 6.9e-8
    # float32 evaluation over [-1, 1] (the kernels clamp their argument)
    xs = _f32(np.concatenate([np.linspace(-1.0, 1.0, 2_000_001), [-1.0, -0.0, 0.0, 1.0],
                              np.nextafter(np.float32(1.0), np.float32(0.0)) * np.array([1.0, -1.0])]))
    err = np.abs(_acos32(xs).astype(np.float64) - np.arccos(xs.astype(np.float64)))
    print("fast_acos float32 max error %.3e rad" % err.max())
    # bound: polynomial 6.8e-8, sqrt and product roundings (half an ulp of
    # numbers below pi/2 each, 6e-8), and for x < 0 pi in float32 (8.7e-8)
    # plus the rounding of pi - r (half an ulp in [2, 4), 1.2e-7)
    assert err[xs >= 0].max() < 2.5e-7
    assert err.max() < 4.0e-7
    assert _acos32(_f32([1.0]))[0] == 0.0
    assert _acos32(_f32([-1.0]))[0] == np.float32(np.pi)


def test_atan_polynomial_error():
    c = _coefficients("fast_atan2").astype(np.float64)
    assert c.size == 9
    s = np.linspace(0.0, 1.0, 2_000_001)
    assert np.max(np.abs(s * np.polyval(c, s * s) - np.arctan(s))) < 2.3e-8
    rng = np.random.default_rng(3)
    th = rng.uniform(-np.pi, np.pi, 1_000_000)
    rad = np.exp(rng.uniform(-20, 20, th.size))
    y, x = _f32(rad * np.sin(th)), _f32(rad * np.cos(th))
    # axes and diagonals in every quadrant
    ax = _f32([1, -1, 0, 0, 1, -1, 1, -1, 3e-30, -3e-30])
    ay = _f32([0, 0, 1, -1, 1, 1, -1, -1, 2e30, 2e30])
    x, y = np.concatenate([x, ax]), np.concatenate([y, ay])
    err = np.abs(_atan2_32(y, x).astype(np.float64) - np.arctan2(y.astype(np.float64), x.astype(np.float64)))
    print("fast_atan2 float32 max error %.3e rad" % err.max())
    assert err.max() < 3.0e-7


def test_atan2_special_cases():
    z, nz = np.float32(0.0), np.float32(-0.0)
    y = np.array([z, nz, z, nz, 1, -1], dtype=np.float32)
    x = np.array([z, z, np.float32(-1), np.float32(-1), z, z], dtype=np.float32)
    r = _atan2_32(y, x)
    assert r[0] == 0.0 and not np.signbit(r[0])       # atan2(0, 0) = 0
    assert r[1] == 0.0 and np.signbit(r[1])           # atan2(-0, 0) = -0
    assert r[2] == np.float32(np.pi) and r[3] == -np.float32(np.pi)
    assert r[4] == np.float32(np.pi / 2) and r[5] == -np.float32(np.pi / 2)


def test_fit_script_reproduces_header_coefficients():
    sys.path.insert(0, CSRC)
    try:
        import fit_fastmath as fit
    finally:
        sys.path.remove(CSRC)
    ca, ea = fit.fit_acos()
    ct, et = fit.fit_atan()
    assert ea < 6.9e-8 and et < 2.3e-8
    # the script returns coefficients lowest degree first
    np.testing.assert_allclose(ca[::-1].astype(np.float32), _coefficients("fast_acos"), rtol=2.4e-7, atol=0)
    np.testing.assert_allclose(ct[::-1].astype(np.float32), _coefficients("fast_atan2"), rtol=2.4e-7, atol=0)
