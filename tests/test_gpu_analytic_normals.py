"""Analytic normals (normal_mode "analytic"): the gradient of the estimate at
the hit point from forward-mode orbit tangents, against the oracle's FP64
dual-number gradient at the GPU's own hit point, on every kernel variant
(Julia of degree 2 and 3, Mandelbulb with n = 8, run-time integer n and real
n), with cut planes and shadows; the c = 0 ball's radial normals; the
benchmark views on a pixel sample; the refusal of the adjoint; and the cost
of the normal stage against the tap modes.
"""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from parity import angle, assert_parity, compare, neighbour_flags, sampled_compare, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


def _analytic(job):
    job = copy.deepcopy(job)
    job["march"]["normal_mode"] = "analytic"
    return job


def _full_parity(frt, orc, job):
    fr = frt.render(job, "cuda", counters=True)
    torch.cuda.synchronize()
    g = to_numpy(fr)
    o = orc.render(job)
    cam = job["camera"]
    nd = neighbour_flags(o["status"].reshape(cam["height"], cam["width"])).ravel()
    st = compare(orc, job, g, o, nd)
    print(job["fractal"]["kind"], job["fractal"]["power"], cam["width"], cam["height"], st, flush=True)
    assert st["oracle_hits"] > 0
    assert_parity(st)
    # one estimate per normal instead of 4 or 6 taps
    hit = (g["status"] & 7) == 2
    assert np.all(g["counters"][4][hit] == 1)
    return st


def test_julia_view_analytic(frt, orc):
    _full_parity(frt, orc, _analytic(W.julia_view()))


def test_cubic_cut_shadow_analytic(frt, orc):
    _full_parity(frt, orc, _analytic(W.julia_view(c=W.JULIA_C3, degree=3, width=200, height=150, shadow=True,
                                                  planes=[W.plane([-0.2, 0.3, 1.0], 0.1)])))


def test_bulb8_shadow_analytic(frt, orc):
    _full_parity(frt, orc, _analytic(W.bulb_views(width=400, height=224)[0]))


def test_bulb_integer_power_analytic(frt, orc):
    _full_parity(frt, orc, _analytic(W.bulb_view(0.4, 0.25, width=160, height=120, power=5.0, max_iter=12)))


def test_bulb_real_power_cut_analytic(frt, orc):
    _full_parity(frt, orc, _analytic(W.bulb_view(2.1, -0.3, width=240, height=180, power=6.37, shadow=True,
                                                 planes=[W.plane([0.2, 1.0, 0.1], 0.1)])))


def test_c0_ball_analytic_normals_are_radial(frt, orc):
    job = _analytic(W.julia_view(c=[0, 0, 0, 0], width=96, height=96))
    job["fractal"]["bound_radius"] = 1.5
    fr = frt.render(job, "cuda")
    torch.cuda.synchronize()
    g = to_numpy(fr)
    hit = (g["status"] & 7) == 2
    assert hit.sum() > 1000
    o, d = orc.camera_rays(job["camera"], np.nonzero(hit)[0])
    p = o + g["depth"][hit, None].astype(np.float64) * d
    ang = angle(g["normal"][:, hit].T, p)
    print("c = 0 ball: max angle to the radial normal %.2e rad" % ang.max())
    assert ang.max() < 2e-6


@pytest.mark.parametrize("view", [1, 5])
def test_bulb_1080p_views_analytic_sampled(frt, orc, view):
    job = _analytic(W.bulb_views()[view])
    fr = frt.render(job, "cuda", counters=True)
    torch.cuda.synchronize()
    pix = W.stratified_pixels(1920, 1080, 16, seed=300 + view)
    st = sampled_compare(orc, job, fr, pix)
    print("view", view, st)
    assert st["oracle_hits"] > 1000
    assert_parity(st)


def test_backward_refuses_analytic_normals(frt):
    job = _analytic(W.julia_view(width=16, height=16))
    fr = frt.render(job, "cuda")
    gc = torch.zeros(3, 256, device="cuda")
    with pytest.raises(frt.FrtError, match="unsupported"):
        frt.render_backward([job], [fr], [gc], None, None, "cuda")


def test_normal_stage_cost_by_mode(frt):
    """Times the normal stage of the eight 1080p views with tetrahedral,
    central and analytic normals (the march stages are identical)."""
    base = W.bulb_views()
    out = {}
    for mode in ("tetra", "central", "analytic"):
        jobs = copy.deepcopy(base)
        for j in jobs:
            j["march"]["normal_mode"] = mode
            j["march"]["shadow"] = False
        frames = [frt.alloc_frame(j, "cuda") for j in jobs]
        ws = frt.alloc_workspace(len(jobs), "cuda")
        frt.render_batch(jobs, "cuda", outs=frames, workspace=ws)
        torch.cuda.synchronize()
        frt.set_stage_timing(True)
        acc = np.zeros(3)
        for _ in range(5):
            frt.render_batch(jobs, "cuda", outs=frames, workspace=ws)
            acc += np.array(frt.stage_times())
        frt.set_stage_timing(False)
        out[mode] = acc / 5
        del frames
    print("normal stage ms:", {m: round(float(s[1]), 3) for m, s in out.items()},
          "primary march ms:", {m: round(float(s[0]), 3) for m, s in out.items()})
