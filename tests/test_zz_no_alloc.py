"""The batch entry point that allocates nothing (frt_render_batch_noalloc)
against frt_render_batch: same kernels, so every output plane must be
identical bit for bit, on two calls in a row through the library's one
device scratch, the second with fewer and smaller renders; and repeated
calls leave the device's free memory unchanged."""
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


def _jobs_large():
    # every kernel variant, ragged sizes, planes, shadows and counters
    jobs = [W.with_size(j, 200 + 37 * k, 120 + 21 * k) for k, j in enumerate(W.julia_batch(n_jobs=6))]
    jobs += [W.bulb_view(0.4 + 0.9 * k, 0.2, width=176, height=99, shadow=True) for k in range(3)]
    jobs += [W.bulb_view(1.1, -0.3, width=64, height=64, power=5.0),
             W.bulb_view(2.0, 0.1, width=96, height=48, power=6.37, planes=[W.plane([0.0, 0.0, 1.0], 0.1)])]
    jobs += [W.with_size(j, 130, 70) for j in W.julia_degree_batch(n_jobs=3)]
    return jobs


def _jobs_small():
    return [W.julia_view(width=40, height=33, planes=[W.plane([0.3, 0.2, 1.0], 0.05)]),
            W.bulb_view(0.7, 0.25, width=48, height=27, shadow=True)]


def _compare(frt, jobs):
    ref = frt.render_batch(jobs, "cuda", counters=True)
    out = [frt.alloc_frame(j, "cuda", counters=True) for j in jobs]
    for f in out:                       # sentinels: every pixel must be written
        for v in f.values():
            v.fill_(-7 if v.dtype != torch.uint8 else 251)
    frt.render_batch_noalloc(jobs, out, "cuda")
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(ref, out)):
        for name in ("depth", "normal", "colour", "status", "counters"):
            x, y = a[name].cpu().numpy(), b[name].cpu().numpy()
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (k, name)
    return out


def test_noalloc_equals_batch_twice_then_smaller(frt):
    big, small = _jobs_large(), _jobs_small()
    print("noalloc: %d jobs, then %d jobs" % (len(big), len(small)), flush=True)
    _compare(frt, big)
    _compare(frt, small)
    # and back to the larger batch after the smaller one
    _compare(frt, big)


def test_noalloc_allocates_no_device_memory(frt):
    jobs = _jobs_small()
    out = [frt.alloc_frame(j, "cuda") for j in jobs]
    frt.render_batch_noalloc(jobs, out, "cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    alloc0 = torch.cuda.memory_allocated()
    for _ in range(20):
        frt.render_batch_noalloc(jobs, out, "cuda")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert torch.cuda.memory_allocated() == alloc0
    assert free1 == free0, (free0, free1)


def test_noalloc_rejects_too_many_jobs(frt):
    jobs = [W.julia_view(width=8, height=8)] * (frt.NOALLOC_MAX_JOBS + 1)
    out = [frt.alloc_frame(jobs[0], "cuda")] * len(jobs)
    with pytest.raises(frt.FrtError, match="FRT_NOALLOC_MAX_JOBS"):
        frt.render_batch_noalloc(jobs, out, "cuda")
