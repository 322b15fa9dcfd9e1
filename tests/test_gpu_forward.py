"""Forward parity: HIP kernels (through the C ABI) vs the FP64 oracle.

Sizes are chosen so the oracle finishes in seconds while covering several
8x8 ray tiles and ragged image edges; the 1080p Mandelbulb views (the
benchmark workload, same launch configuration) are compared on a stratified
pixel sample with the oracle's 3x3 neighbourhoods for the boundary rule.
"""
import numpy as np
import pytest
import torch

import workloads as W
from parity import assert_parity, boundary_set, compare, neighbour_flags, sampled_compare, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


def _gpu(frt, job, counters=True):
    fr = frt.render(job, "cuda", counters=counters)
    torch.cuda.synchronize()
    return to_numpy(fr)


def _full_parity(frt, orc, job, **kw):
    g = _gpu(frt, job)
    o = orc.render(job)
    cam = job["camera"]
    nd = neighbour_flags(o["status"].reshape(cam["height"], cam["width"])).ravel()
    st = compare(orc, job, g, o, nd)
    print(job["fractal"]["kind"], cam["width"], cam["height"], st, flush=True)
    assert_parity(st, **kw)
    return g, o, st


def _hit_disagreements_outside_boundary(orc, job, g, o):
    """Pixels where the GPU and the oracle disagree on hit or miss, outside
    the boundary set B that the oracle's render alone decides."""
    cam = job["camera"]
    nd = neighbour_flags(o["status"].reshape(cam["height"], cam["width"])).ravel()
    _, dirs = orc.camera_rays(cam, np.arange(o["depth"].size))
    B = boundary_set(o, nd, dirs)
    dis = ((g["status"] & 7) >= 2) != ((o["status"] & 7) >= 2)
    return np.flatnonzero(dis & ~B)


def test_julia_view_parity(frt, orc):
    _full_parity(frt, orc, W.julia_view())


def test_julia_cut_plane_parity(frt, orc):
    _full_parity(frt, orc, W.julia_view(planes=[W.plane([0.3, 0.2, 1.0], 0.05)]))


def test_julia_two_planes_shadow_ragged(frt, orc):
    job = W.julia_view(width=250, height=190, shadow=True,
                       planes=[W.plane([0.3, 0.2, 1.0], 0.05), W.plane([-1.0, 0.4, 0.2], 0.3)])
    _full_parity(frt, orc, job)


def test_julia_central_normals_parity(frt, orc):
    _full_parity(frt, orc, W.julia_view(width=200, height=136, normal_mode="central"))


def test_bulb_view_parity(frt, orc):
    _full_parity(frt, orc, W.bulb_views(width=480, height=270)[0])


def test_bulb_real_power_cut_parity(frt, orc):
    job = W.bulb_view(2.1, -0.3, width=320, height=240, power=6.37, shadow=True,
                      planes=[W.plane([0.2, 1.0, 0.1], 0.1)])
    _full_parity(frt, orc, job)


def test_bulb_integer_power_16_tetra(frt, orc):
    job = W.bulb_view(0.4, 0.25, width=160, height=120, power=16.0, max_iter=15, normal_mode="tetra")
    _full_parity(frt, orc, job)


@pytest.mark.parametrize("view", range(8))
def test_bulb_1080p_views_sampled(frt, orc, view):
    """The benchmark workload itself (1920x1080, n = 8, shadows), compared on
    one pixel per 16x16 cell."""
    job = W.bulb_views()[view]
    g = _gpu(frt, job)
    pix = W.stratified_pixels(1920, 1080, 16, seed=view)
    st = sampled_compare(orc, job, g, pix)
    print("view", view, st, flush=True)
    assert_parity(st)


def test_c0_ball_closed_form_on_gpu(frt, orc):
    """c = 0 with a loose bounding radius: refined depth = entry into the
    sphere 0.5 r ln r = eps, normal radial."""
    from scipy.optimize import brentq
    job = W.julia_view(c=[0, 0, 0, 0], width=96, height=96)
    job["fractal"]["bound_radius"] = 1.5
    eps = job["march"]["eps_abs"]
    rho = brentq(lambda r: 0.5 * r * np.log(r) - eps, 1.0, 2.0, xtol=1e-15)
    g = _gpu(frt, job)
    o, d = orc.camera_rays(job["camera"], np.arange(96 * 96))
    bp = np.einsum("ij,ij->i", o, d)
    b = np.sqrt(np.maximum(np.einsum("ij,ij->i", o, o) - bp * bp, 0))
    clear = np.abs(b - rho) > 3e-3
    hit = clear & (b < rho)
    assert np.all(((g["status"] & 7) == 2)[clear] == (b < rho)[clear])
    t_ref = -bp[hit] - np.sqrt(bp[hit] ** 2 - (np.einsum("ij,ij->i", o, o)[hit] - rho * rho))
    assert np.max(np.abs(g["depth"][hit] - t_ref)) < 2e-5
    p = o[hit] + t_ref[:, None] * d[hit]
    nref = p / np.linalg.norm(p, axis=1, keepdims=True)
    ang = np.arccos(np.clip(np.einsum("ij,ij->i", g["normal"][:, hit].T, nref), -1, 1))
    assert ang.max() < 1e-3


@pytest.mark.parametrize("wh", [(1, 1), (3, 5), (9, 7), (17, 8), (64, 1)])
def test_tiny_and_ragged_images(frt, orc, wh):
    w, h = wh
    job = W.julia_view(width=w, height=h, planes=[W.plane([0.3, 0.2, 1.0], 0.05)], shadow=True)
    fr = frt.alloc_frame(job, "cuda", counters=True)
    fr["status"].fill_(0xFF)
    frt.render(job, "cuda", out=fr)
    torch.cuda.synchronize()
    g = to_numpy(fr)
    assert np.all(g["status"] != 0xFF)          # every pixel written exactly by its lane
    o = orc.render(job)
    assert _hit_disagreements_outside_boundary(orc, job, g, o).size == 0


def test_degenerate_parameters(frt, orc):
    """max_iter = 1, max_steps = 1, no refinement, camera looking away."""
    job = W.julia_view(width=40, height=40, max_iter=1, max_steps=1)
    job["march"]["refine_iters"] = 0
    g = _gpu(frt, job)
    o = orc.render(job)
    assert _hit_disagreements_outside_boundary(orc, job, g, o).size == 0
    away = W.julia_view(width=33, height=21)
    away["camera"]["target"] = [0.0, 0.0, 6.0]
    g = _gpu(frt, away)
    assert np.all(g["status"] == 0) and np.all(g["depth"] == -1.0)
    assert np.all(g["counters"] == 0)


def test_invalid_arguments_raise_and_write_nothing(frt):
    job = W.julia_view(width=16, height=16)
    fr = frt.alloc_frame(job, "cuda")
    fr["depth"].fill_(7.0)
    bad = [("fractal", "max_iter", 0), ("march", "eps_abs", -1.0), ("march", "max_steps", 0),
           ("camera", "width", 0), ("fractal", "bailout2", float("nan")), ("march", "normal_mode", 5)]
    for blk, key, val in bad:
        j = {k: (dict(v) if isinstance(v, dict) else list(v)) for k, v in job.items()}
        j[blk][key] = val
        if key == "width":
            with pytest.raises(frt.FrtError):
                frt.render(j, "cuda")
            continue
        with pytest.raises(frt.FrtError, match="invalid argument"):
            frt.render(j, "cuda", out=fr)
    j = {k: (dict(v) if isinstance(v, dict) else list(v)) for k, v in job.items()}
    j["planes"] = [W.plane([0.0, 0.0, 0.0], 0.1)]
    with pytest.raises(frt.FrtError, match="plane normal is zero"):
        frt.render(j, "cuda", out=fr)
    torch.cuda.synchronize()
    assert torch.all(fr["depth"] == 7.0)


def test_counters_match_oracle_steps(frt, orc):
    job = W.julia_view(width=128, height=128)
    g = _gpu(frt, job)
    o = orc.render(job)
    same = (g["status"] & 7) == (o["status"] & 7)
    agree = np.mean(g["counters"][0][same] == o["steps"][same])
    assert agree > 0.97
