"""Accuracy of the library's fast float32 math and of its distance estimate
at single points, on the GPU, against double-precision references (numpy
for the functions, the FP64 oracle for the estimate)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


def _eval(frt, name, x, y=None):
    out = frt.math_eval(name, x, y)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def test_fast_acos_atan2(frt):
    x = np.linspace(-1, 1, 200001, dtype=np.float32)
    err = np.abs(_eval(frt, "acos", x) - np.arccos(x.astype(np.float64)))
    print("acos max abs err", err.max())
    assert err.max() < 4e-7
    rng = np.random.default_rng(0)
    a = rng.normal(size=200000).astype(np.float32)
    b = rng.normal(size=200000).astype(np.float32)
    err = np.abs(_eval(frt, "atan2", a, b) - np.arctan2(a.astype(np.float64), b.astype(np.float64)))
    print("atan2 max abs err", err.max())
    assert err.max() < 4e-7
    assert _eval(frt, "atan2", np.zeros(1, np.float32), np.zeros(1, np.float32))[0] == 0.0


@pytest.mark.parametrize("lim", [0.5, 2.0, 8.0])
def test_hardware_sin_cos_in_revolutions(frt, lim):
    x = np.linspace(-lim, lim, 400001, dtype=np.float32)
    ref = 2 * np.pi * x.astype(np.float64)
    es = np.abs(_eval(frt, "sin_rev", x) - np.sin(ref))
    ec = np.abs(_eval(frt, "cos_rev", x) - np.cos(ref))
    print("revolutions +-%g: sin max abs err %.3e, cos %.3e" % (lim, es.max(), ec.max()))
    assert es.max() < 2e-6 and ec.max() < 2e-6


def test_hardware_log2_exp2_rsq_rcp(frt):
    x = np.geomspace(1e-6, 1e6, 200001).astype(np.float32)
    xd = x.astype(np.float64)
    rel = lambda a, b: np.max(np.abs(a - b) / np.abs(b))
    e_log = np.max(np.abs(_eval(frt, "log2", x) - np.log2(xd)) / np.maximum(1.0, np.abs(np.log2(xd))))
    e_rsq = rel(_eval(frt, "rsq", x), 1 / np.sqrt(xd))
    e_rcp = rel(_eval(frt, "rcp", x), 1 / xd)
    y = np.linspace(-30, 30, 200001, dtype=np.float32)
    e_exp = rel(_eval(frt, "exp2", y), np.exp2(y.astype(np.float64)))
    print("log2 err/max(1,|log2|) %.3e exp2 rel %.3e rsq rel %.3e rcp rel %.3e" % (e_log, e_exp, e_rsq, e_rcp))
    assert e_log < 1e-6 and e_exp < 1e-6 and e_rsq < 1e-6 and e_rcp < 1e-6


FRACTALS = {
    "julia": W.julia(W.JULIA_C1, 11),
    "julia3": W.julia(W.JULIA_C3, 11, degree=3),
    "julia5": W.julia([-0.5, 0.3, 0.1, 0.0], 8, degree=5),
    "bulb8": W.bulb(8.0, 10),
    "bulb5": W.bulb(5.0, 10),
    "bulb_real": W.bulb(6.37, 10),
}


@pytest.mark.parametrize("name", sorted(FRACTALS))
def test_distance_matches_oracle(frt, orc, name):
    """Estimate at points spread through the bounding ball, on points whose
    orbit escapes away from the bailout decision (elsewhere the escape count,
    and with it the estimate, is decided by rounding).  Near the set z^p + c
    cancels and the next body multiplies the relative rounding error by p, so
    float32 carries a heavy tail; the bounds are on quantiles."""
    fr = FRACTALS[name]
    rng = np.random.default_rng(5)
    R = orc.bound_radius(fr)
    dirs = rng.normal(size=(100000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = (dirs * R * rng.uniform(0.3, 1.0, size=(100000, 1))).astype(np.float32)
    d, it = frt.distance(fr, pts)
    torch.cuda.synchronize()
    d, it = d.cpu().numpy().astype(np.float64), it.cpu().numpy()
    od, oit, _, _ = orc.de(fr, pts.astype(np.float64))
    mg, esc = orc.escape_margin(fr, pts.astype(np.float64))
    clean = esc & (mg > 1e-3)
    same = it == oit
    rel = np.abs(d - od) / np.maximum(np.abs(od), 1e-6)
    q = np.percentile(rel[clean], [50, 99, 99.9])
    print(name, "escape-count agreement %.5f (clean %.5f)" % (same.mean(), same[clean].mean()),
          "rel err p50 %.2e p99 %.2e p99.9 %.2e" % tuple(q))
    assert same[clean].mean() > 0.9999
    assert q[0] < 1e-6 and q[1] < 2e-3


@pytest.mark.parametrize("mode", ["tetra", "central", "analytic"])
@pytest.mark.parametrize("name", sorted(FRACTALS))
def test_normal_query_matches_oracle(frt, orc, name, mode):
    """The renderer's normal rule at points near the set (on rays toward the
    origin, where the orbit escapes, with a tap scale of 1e-3), against the
    oracle's normal at the same float32 points, on the points whose normal
    is well conditioned at float32 resolution."""
    from parity import angle, normal_ill_conditioned
    fr = FRACTALS[name]
    rng = np.random.default_rng(7)
    R = orc.bound_radius(fr)
    dirs = rng.normal(size=(4000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = (dirs * R * rng.uniform(0.5, 1.0, size=(4000, 1))).astype(np.float32)
    d, _, _, _ = orc.de(fr, pts.astype(np.float64))
    keep = (d > 2e-3) & (d < 0.05)           # near the set, outside the tap spacing
    pts, dirs = pts[keep], dirs[keep]
    eps = np.full(len(pts), 1e-3)
    g = frt.normal_at(fr, pts, mode, eps=eps.astype(np.float32)).cpu().numpy()
    p64 = pts.astype(np.float64)
    ref = orc.normal_at(fr, p64, -dirs, eps, mode)
    ill = normal_ill_conditioned(orc, fr, {"normal_mode": mode}, p64, -dirs, eps)
    ok = ~ill & (np.linalg.norm(g, axis=1) > 0)
    ang = angle(g[ok], ref[ok])
    q = np.percentile(ang, [50, 99, 100])
    print(name, mode, "points %d (well conditioned %d)" % (len(pts), ok.sum()),
          "angle p50 %.2e p99 %.2e max %.2e" % tuple(q))
    assert ok.sum() > 200
    assert np.mean(ang <= 1e-3) >= 0.999 and q[1] < 3e-4
