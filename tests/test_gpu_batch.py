"""Batched persistent launch: 64 uneven quaternion Julia renders (seeded c,
cut plane, resolution, iteration count and eps) drained by one launch per
kernel, with and without HIP-graph replay, against one-by-one renders and
the FP64 oracle."""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from parity import assert_aggregate_exclusions, assert_parity, compare, neighbour_flags, sampled_compare, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def batch_jobs():
    return W.julia_batch()


def _same(a, b):
    """Fraction of pixels with identical status and depth."""
    return float(np.mean((a["status"] == b["status"]) & (a["depth"] == b["depth"])))


def test_batch_equals_one_by_one(frt, batch_jobs):
    outs = frt.render_batch(batch_jobs, "cuda", counters=True)
    singles = [frt.render(j, "cuda", counters=True) for j in batch_jobs]
    torch.cuda.synchronize()
    worst = 1.0
    for k, (a, b) in enumerate(zip(outs, singles)):
        a, b = to_numpy(a), to_numpy(b)
        s = _same(a, b)
        worst = min(worst, s)
        assert s >= 0.9999, (k, s)
    print("worst identical-pixel fraction over 64 jobs: %.6f" % worst)


def test_batch_parity_against_oracle(frt, orc, batch_jobs):
    outs = frt.render_batch(batch_jobs, "cuda", counters=True)
    torch.cuda.synchronize()
    checked = 0
    stats = []
    for k, (job, fr) in enumerate(zip(batch_jobs, outs)):
        g = to_numpy(fr)
        cam = job["camera"]
        W_, H = cam["width"], cam["height"]
        if W_ * H <= 256 * 256:
            o = orc.render(job)
            nd = neighbour_flags(o["status"].reshape(H, W_)).ravel()
            st = compare(orc, job, g, o, nd)
        else:
            pix = W.stratified_pixels(W_, H, 8, seed=k)
            st = sampled_compare(orc, job, g, pix)
        if st["oracle_hits"] == 0 and st["gpu_hits"] == 0:
            continue
        # single jobs of this set may be mostly chaotic (eps down to 1e-4, up
        # to 24 orbit iterations): their exclusions are bounded in aggregate
        assert_parity(st, max_boundary=0.4, max_normal_boundary=1.0)
        stats.append(st)
        checked += 1
    print("jobs with hits compared:", checked)
    assert checked >= 10
    assert_aggregate_exclusions(stats, max_boundary=0.10, max_normal_boundary=0.45)


def test_graph_replay_matches_eager(frt, batch_jobs):
    """Capture once, replay with changed parameters and with the program's
    own eager work and synchronisations between replays; every replay must
    equal a fresh eager render of the same jobs."""
    jobs = copy.deepcopy(batch_jobs[:16])
    frames = [frt.alloc_frame(j, "cuda") for j in jobs]
    ref_frames = [frt.alloc_frame(j, "cuda") for j in jobs]
    ws = frt.alloc_workspace(len(jobs), "cuda")
    frt.graph_reset()
    rng = np.random.default_rng(7)
    for rep in range(4):
        if rep > 0:
            for j in jobs:   # new parameters between replays
                j["fractal"]["c"] = W.f32v(np.array(j["fractal"]["c"]) + rng.normal(0, 0.01, 4))
        frt.render_batch(jobs, "cuda", outs=frames, workspace=ws, use_graph=True)
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2).sum()            # eager work on the same stream
        torch.cuda.synchronize()
        frt.render_batch(jobs, "cuda", outs=ref_frames, workspace=frt.alloc_workspace(len(jobs), "cuda"))
        torch.cuda.synchronize()
        for a, b in zip(frames, ref_frames):
            a, b = to_numpy(a), to_numpy(b)
            assert np.array_equal(a["status"], b["status"])
            assert np.array_equal(a["depth"], b["depth"])
            assert np.array_equal(a["colour"], b["colour"])
    frt.graph_reset()


def test_mixed_kind_batch(frt, orc):
    jobs = [W.julia_view(width=120, height=90), W.bulb_view(0.3, 0.1, width=100, height=80),
            W.bulb_view(1.3, -0.2, width=64, height=64, power=6.37, planes=[W.plane([0.1, 1, 0], 0.05)]),
            W.julia_view(width=50, height=70, planes=[W.plane([0.3, 0.2, 1.0], 0.05)], shadow=True)]
    outs = frt.render_batch(jobs, "cuda", counters=True)
    torch.cuda.synchronize()
    for job, fr in zip(jobs, outs):
        g = to_numpy(fr)
        o = orc.render(job)
        cam = job["camera"]
        nd = neighbour_flags(o["status"].reshape(cam["height"], cam["width"])).ravel()
        st = compare(orc, job, g, o, nd)
        assert_parity(st, max_boundary=0.2)


def _tiny_jobs():
    """27 small renders (1x1 to 17x13) over all five kernel variants, some
    with shadows and cut planes: several jobs fall inside one queue claim,
    and job ranges end inside claims and tile groups."""
    sizes = [(1, 1), (7, 5), (9, 9), (17, 3), (8, 8), (3, 17), (16, 9), (5, 13), (17, 13)]
    jobs = []
    for k, (w, h) in enumerate(sizes):
        shadow = k % 2 == 0
        planes = [W.plane([0.2, 1.0, 0.3], 0.05)] if k % 3 == 1 else []
        jobs.append(W.julia_view(width=w, height=h, shadow=shadow, planes=planes))
        jobs.append(W.bulb_view(0.3 + 0.5 * k, 0.2, width=h, height=w, shadow=not shadow, planes=planes,
                                power=[8.0, 5.0, 6.37][k % 3]))
        jobs.append(W.julia_view(c=W.JULIA_C3, degree=3, width=w + 2, height=h, shadow=shadow, planes=planes))
    return jobs


def test_tiny_jobs_share_claims(frt, orc):
    jobs = _tiny_jobs()
    outs = frt.render_batch(jobs, "cuda", counters=True)
    singles = [frt.render(j, "cuda", counters=True) for j in jobs]
    torch.cuda.synchronize()
    hits = 0
    stats = []
    for k, (job, fr, one) in enumerate(zip(jobs, outs, singles)):
        g, s = to_numpy(fr), to_numpy(one)
        assert _same(g, s) == 1.0, k
        o = orc.render(job)
        cam = job["camera"]
        nd = neighbour_flags(o["status"].reshape(cam["height"], cam["width"])).ravel()
        st = compare(orc, job, g, o, nd)
        hits += st["oracle_hits"]
        # on images of a few pixels nearly every pixel has a neighbour of the
        # other class: the boundary set is bounded over the whole set
        assert_parity(st, max_boundary=1.0)
        stats.append(st)
    print("tiny jobs: %d, oracle hits %d" % (len(jobs), hits))
    assert hits > 200
    assert_aggregate_exclusions(stats, max_boundary=0.5, max_normal_boundary=0.05)


def test_batch_speedup_over_one_by_one(frt, batch_jobs):
    """Reports the throughput gain of one batched launch (and its graph
    replay) over the same 64 renders launched one by one."""
    frames = [frt.alloc_frame(j, "cuda") for j in batch_jobs]
    ws = frt.alloc_workspace(len(batch_jobs), "cuda")
    ws1 = frt.alloc_workspace(1, "cuda")

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        return s.elapsed_time(e) / reps

    t_single = timed(lambda: [frt.render(j, "cuda", out=f, workspace=ws1) for j, f in zip(batch_jobs, frames)])
    t_batch = timed(lambda: frt.render_batch(batch_jobs, "cuda", outs=frames, workspace=ws))
    t_graph = timed(lambda: frt.render_batch(batch_jobs, "cuda", outs=frames, workspace=ws, use_graph=True))
    frt.graph_reset()
    print("64 renders: one by one %.3f ms, batched %.3f ms (x%.2f), graph %.3f ms (x%.2f)"
          % (t_single, t_batch, t_single / t_batch, t_graph, t_single / t_graph))
    # the batched-launch target: at least twice the throughput of the same
    # renders launched one by one
    assert t_single >= 2.0 * t_batch
    assert t_single >= 2.0 * t_graph


@pytest.mark.parametrize("block,chunk", [(64, 64), (128, 256), (512, 1024), (256, 64)])
def test_every_ray_claimed_under_any_launch_shape(frt, block, chunk):
    """The queue hands every chunk out: each wave's first chunk by its index
    in the grid, the rest through eight counters that waves drain and then
    steal from.  Output planes prefilled with sentinels must be fully
    written for any chunk and block size, including grids of fewer blocks
    than counters (tiny renders), and must equal the default launch's
    output bit for bit."""
    jobs = _tiny_jobs()[:12] + [W.bulb_view(0.7, 0.2, width=333, height=101, shadow=True),
                                W.julia_view(width=200, height=120, shadow=True,
                                             planes=[W.plane([0.2, 1.0, 0.3], 0.05)])]
    ref = frt.render_batch(jobs, "cuda")
    torch.cuda.synchronize()
    variants = ("julia", "bulb_real", "bulb_int", "bulb8", "julia_deg")
    saved = {v: frt.autotune_get(v) for v in variants}
    try:
        for v in variants:
            b, c, w, o, r = saved[v]
            frt.autotune_set(v, block, chunk, w, o, r)
        outs = [frt.alloc_frame(j, "cuda") for j in jobs]
        for f in outs:
            f["depth"].fill_(float("nan"))
            f["normal"].fill_(float("nan"))
            f["colour"].fill_(float("nan"))
            f["status"].fill_(255)
        frt.render_batch(jobs, "cuda", outs=outs)
        # one render alone too (its own grid, often below eight blocks)
        single = frt.alloc_frame(jobs[3], "cuda")
        single["status"].fill_(255)
        single["depth"].fill_(float("nan"))
        frt.render(jobs[3], "cuda", out=single)
        torch.cuda.synchronize()
    finally:
        for v in variants:
            frt.autotune_set(v, *saved[v])
    for k, (f, g) in enumerate(zip(outs, ref)):
        assert not torch.isnan(f["depth"]).any() and not torch.isnan(f["colour"]).any(), k
        assert not (f["status"] == 255).any(), k
        for plane in ("depth", "normal", "colour", "status"):
            assert torch.equal(f[plane], g[plane]), (k, plane)
    assert not (single["status"] == 255).any() and not torch.isnan(single["depth"]).any()
    assert torch.equal(single["depth"], ref[3]["depth"])


def test_instrumented_build_counts_and_checks():
    """The instrumented build (trip counters and index checks compiled in)
    against the per-pixel counter planes of the same renders: the lanes that
    took a step path must equal the distance estimates, and the live lanes
    of the orbit loop the orbit bodies, exactly, for the primary and the
    shadow march of the eight 1080p views; and no index check may fail on
    those views, the degree batch, the 64-job batch or the differentiable
    set's adjoint.  The waves' time stamps must be in order.  Run in a child
    process, which loads libfrt_instr.so in place of libfrt.so."""
    import json
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(root, "paper_2102_01747_amd", "libfrt_instr.so")):
        pytest.skip("libfrt_instr.so not built")
    res = subprocess.run([sys.executable, "-m", "paper_2102_01747_amd.trip_counts", "--check"], cwd=root,
                         capture_output=True, text=True, timeout=240)
    print(res.stdout, res.stderr[-2000:])
    lines = [json.loads(l) for l in res.stdout.splitlines() if l.startswith("{")]
    stages = [l for l in lines if "stage" in l]
    failed = [l for l in lines if "failed_checks" in l]
    assert res.returncode == 0 and len(stages) == 2 and len(failed) == 1
    for st in stages:
        assert st["check"], st
        assert 0.5 < st["orbit_loop_lane_use"] <= 1.0
        # the wave stamps: every wave exited, and each found the queue dry
        # before (or as) it left; the exits lie in order
        assert st["waves"] >= 1024, st
        dry, ex = st["queue_dry_us"], st["exit_us"]
        assert 0.0 <= dry[0] <= dry[1] <= ex["last"], st
        assert 0.0 < ex["first"] <= ex["mean"] <= ex["last"] < 1e6, st
        assert 0.0 <= st["tail_idle_frac"] < 1.0, st
    assert all(not v for v in failed[0]["failed_checks"].values()), failed
