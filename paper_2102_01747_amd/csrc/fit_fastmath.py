"""Fit the polynomial cores of the library's fast acos and atan (float32).

Method: weighted least squares on Chebyshev nodes refined by Lawson's
iteration (reweighting by the error magnitude), which converges to the
minimax (equioscillating) polynomial.  Coefficients are fitted in double,
rounded to float32, and the error of the rounded polynomial is measured on a
dense grid against numpy's double-precision acos/atan.

    acos(x) = sqrt(1 - x) * P(x),       x in [0, 1], P of degree 7
    atan(s) = s * Q(s^2),               s in [0, 1], Q of degree 8

Run:  python fit_fastmath.py   (prints the C initialisers used in frt_math.hpp)
"""
import numpy as np


def lawson(f, basis, lo, hi, n_nodes=4000, iters=300):
    k = np.arange(n_nodes)
    x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(np.pi * (k + 0.5) / n_nodes)
    A = basis(x)
    y = f(x)
    w = np.ones_like(x) / n_nodes
    coef = None
    for _ in range(iters):
        sw = np.sqrt(w)
        coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
        err = np.abs(A @ coef - y)
        w = w * err
        w /= w.sum()
    return coef


def horner(c, x):
    r = np.zeros_like(x) + c[-1]
    for a in c[-2::-1]:
        r = r * x + a
    return r


def fit_acos():
    deg = 7
    # P(x) = acos(x)/sqrt(1-x); absolute error of acos = sqrt(1-x)|dP|, so weight by sqrt(1-x)
    f = lambda x: np.arccos(x) / np.sqrt(1 - x)
    basis = lambda x: np.sqrt(1 - x)[:, None] * np.vander(x, deg + 1, increasing=True)
    g = lambda x: np.arccos(x)
    c = lawson(g, basis, 0.0, 1.0 - 1e-12)
    c32 = c.astype(np.float32).astype(np.float64)
    x = np.linspace(0, 1, 2_000_001)
    err = np.max(np.abs(np.sqrt(1 - x) * horner(c32, x) - np.arccos(x)))
    _ = f
    return c32, err


def fit_atan():
    deg = 8
    basis = lambda s: s[:, None] * np.vander(s * s, deg + 1, increasing=True)
    c = lawson(np.arctan, basis, 0.0, 1.0)
    c32 = c.astype(np.float32).astype(np.float64)
    s = np.linspace(0, 1, 2_000_001)
    err = np.max(np.abs(s * horner(c32, s * s) - np.arctan(s)))
    return c32, err


def main():
    ca, ea = fit_acos()
    ct, et = fit_atan()
    fmt = lambda c: ", ".join("%.9ef" % v for v in c)
    print("// acos(x) = sqrt(1-x) * P(x), x in [0,1]; max abs error of the float32 coefficients %.2e rad" % ea)
    print("ACOS_P = { %s };" % fmt(ca))
    print("// atan(s) = s * Q(s^2), s in [0,1]; max abs error of the float32 coefficients %.2e rad" % et)
    print("ATAN_Q = { %s };" % fmt(ct))


if __name__ == "__main__":
    main()
