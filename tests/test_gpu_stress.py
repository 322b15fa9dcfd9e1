"""The stress sweep: 64 frames of 3840x2160, frame f with Mandelbulb power
n = 2 + 14 f / 63 (integer at every 9th frame, real otherwise), cut plane
z <= 0.1, 15 orbit iterations, 1024 steps, eps = 2e-4 t, central normals.

All 64 frames (530 M rays) are rendered in one batch call, traced as two
groups: the 8 integer-power frames by the integer-power kernels and the 56
real-power frames by the real-power kernels.  Five frames (0, 20, 45, 50
and 63: three integer and two real powers) are compared with the FP64
oracle on one pixel per 16x16 cell.  The
adjoint with respect to n is checked against FP64 central differences on two
frames at reduced resolution (same cameras), with a seeded N(0, 1) cotangent
on the colour (L = sum w . colour).
"""
import numpy as np
import pytest
import torch

import workloads as W
from gradcheck import finite_differences
from parity import adjoint_mask, assert_parity, sampled_compare, to_numpy

pytestmark = pytest.mark.gpu

FRAMES = (0, 20, 45, 50, 63)   # n = 2, 6.44, 12, 13.11, 16: three integer and two real powers


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def sweep(frt):
    jobs = W.stress_sweep()
    frames = frt.render_batch(jobs, "cuda", counters=True)
    torch.cuda.synchronize()
    yield jobs, frames
    del frames
    torch.cuda.empty_cache()


@pytest.mark.parametrize("f", FRAMES)
def test_stress_frames_sampled_parity(frt, orc, sweep, f):
    jobs, frames = sweep
    pix = W.stratified_pixels(3840, 2160, 16, seed=500 + f)
    st = sampled_compare(orc, jobs[f], frames[f], pix)
    print("frame %d (n = %.4f)" % (f, jobs[f]["fractal"]["power"]), st, flush=True)
    assert st["oracle_hits"] > 1000
    # powers up to 16 at eps = 2e-4 t: a quarter of the normals are
    # sensitive beyond 2e-4 rad to float32 changes of their inputs
    assert_parity(st, max_normal_boundary=0.35)


def test_stress_sweep_throughput(frt, sweep):
    """Times the 64-frame batch (no counters) and checks it renders the same
    status and depth as the counting launch the parity tests use."""
    jobs, ref = sweep
    frames = [frt.alloc_frame(j, "cuda") for j in jobs]
    ws = frt.alloc_workspace(len(jobs), "cuda")
    frt.render_batch(jobs, "cuda", outs=frames, workspace=ws)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    reps = 2
    for _ in range(reps):
        frt.render_batch(jobs, "cuda", outs=frames, workspace=ws)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    rays = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    print("stress sweep: 64 x 3840x2160, %.1f ms per batch, %.0f Mrays/s" % (ms, rays / (ms * 1e-3) / 1e6))
    for f in FRAMES:
        assert torch.equal(frames[f]["status"], ref[f]["status"])
        assert torch.equal(frames[f]["depth"], ref[f]["depth"])
    del frames


@pytest.mark.parametrize("f", (10, 50))
def test_stress_adjoint_power_vs_fp64_fd(frt, orc, f):
    job = W.with_size(W.stress_frame(f), 256, 144)
    fr = frt.render(job, "cuda", counters=True)
    torch.cuda.synchronize()
    g = to_numpy(fr)
    o = orc.render(job)
    M = adjoint_mask(orc, job, g, o)
    idx = np.nonzero(M)[0]
    assert idx.size > 500, idx.size
    J, taps = orc.pixel_jacobian(job, idx)
    scale = 1.0 + np.abs(J.transpose(1, 0, 2))
    fd, stable = finite_differences(orc, job, idx, [4], o["status"][idx], taps, scale)
    keep = stable[4]
    assert keep.mean() > 0.95, keep.mean()
    P = job["camera"]["width"] * job["camera"]["height"]
    w = np.random.default_rng(5).normal(size=(3, P)).astype(np.float32)
    M2 = np.zeros(P, bool)
    M2[idx[keep]] = True
    w[:, ~M2] = 0.0
    gc = torch.from_numpy(w).cuda()
    grads = frt.render_backward([job], [fr], [gc], None, None, "cuda")
    torch.cuda.synchronize()
    gpu = float(grads[1].cpu()[0])
    ref = float(np.sum(w[:, idx] * fd[4][4:7]))
    scale_sum = float(np.sum(np.abs(w[:, idx] * fd[4][4:7])))
    rel = abs(gpu - ref) / abs(ref)
    print("frame %d (n = %.4f): dL/dn GPU %.8e FD %.8e rel %.2e (sum |terms| %.3e)"
          % (f, job["fractal"]["power"], gpu, ref, rel, scale_sum))
    assert rel < 1e-3


def test_sweep_batched_adjoint_power_vs_fp64_fd(frt, orc, sweep):
    """The stress sweep's batched adjoint: dL/dn of all 64 frames of 3840 x
    2160 (n = 2 + 14 f / 63) in ONE backward call, L = sum w . colour with a
    seeded normal cotangent w per pixel (seed 5), timed beside the forward
    batch.  Frames 10 and 50 are checked through that same call: their
    cotangent is kept only on the stable pixels of a seeded stratified
    sample (one per 32 x 32 cell), whose FP64 central differences of the
    oracle give dL/dn to compare with (relative 1e-3)."""
    from gradcheck import finite_differences
    from parity import sampled_adjoint_mask

    jobs, frames = sweep
    P = 3840 * 2160
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    gcs = [torch.randn(3, P, device="cuda", generator=gen) for _ in jobs]
    refs = {}
    for f in (10, 50):
        pix = W.stratified_pixels(3840, 2160, 32, seed=700 + f)
        M, g, o = sampled_adjoint_mask(orc, jobs[f], frames[f], pix)
        idx = pix[M]
        J, taps = orc.pixel_jacobian(jobs[f], idx)
        scale = 1.0 + np.abs(J.transpose(1, 0, 2))
        fd, stable = finite_differences(orc, jobs[f], idx, [4], o["status"][M], taps, scale)
        kp = idx[stable[4]]
        ki = torch.as_tensor(kp, device="cuda")
        w = gcs[f][:, ki].clone()
        gcs[f].zero_()
        gcs[f][:, ki] = w
        refs[f] = (float(np.sum(w.cpu().numpy().astype(np.float64) * fd[4][4:7][:, stable[4]])), kp.size, M.mean())
    ws_f = frt.alloc_workspace(len(jobs), "cuda")
    ws_b = frt.alloc_workspace(len(jobs), "cuda")

    def timed(fn, reps=2):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            out = fn()
        e.record()
        e.synchronize()
        return s.elapsed_time(e) / reps, out

    fwd = [frt.alloc_frame(j, "cuda") for j in jobs]
    frt.render_batch(jobs, "cuda", outs=fwd, workspace=ws_f)
    t_f, _ = timed(lambda: frt.render_batch(jobs, "cuda", outs=fwd, workspace=ws_f))
    del fwd
    frt.render_backward(jobs, frames, gcs, None, None, "cuda", workspace=ws_b)
    t_b, grads = timed(lambda: frt.render_backward(jobs, frames, gcs, None, None, "cuda", workspace=ws_b))
    torch.cuda.synchronize()
    gn = grads[1].cpu().numpy().astype(np.float64)
    print("sweep (64 x 3840x2160): forward %.1f ms, batched backward w.r.t. n %.1f ms (x%.2f), %.0f gradients/s"
          % (t_f, t_b, t_b / t_f, len(jobs) / ((t_f + t_b) * 1e-3)))
    for f, (ref, n, frac) in refs.items():
        rel = abs(gn[f] - ref) / abs(ref)
        print("frame %d (n = %.4f): %d stable sampled pixels (mask %.2f); dL/dn GPU %.8e FD %.8e rel %.2e"
              % (f, jobs[f]["fractal"]["power"], n, frac, gn[f], ref, rel))
        assert n > 1000
        assert rel < 1e-3
    assert np.all(np.isfinite(gn)) and np.count_nonzero(gn) == len(jobs)
    assert t_b <= 3.0 * t_f
    del gcs
