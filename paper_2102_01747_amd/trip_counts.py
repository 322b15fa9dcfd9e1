"""Trip statistics and index checks of the instrumented build.

    python -m paper_2102_01747_amd.trip_counts [--build] [--check]

Loads the instrumented build libfrt_instr.so (built with --build, or by
paper_2102_01747_amd._build.build(instrument=True): the same kernels with
the march kernels' trip counters and the kernels' index checks compiled in),
renders the eight 1920 x 1080 Mandelbulb views of the bench as one batch,
and prints one JSON line per march stage: wave-level trips round the outer
loop, orbit-loop iterations, step paths, refills and claims, and the lanes
they served.  With a kernel's SQ_INSTS_VALU from rocprofv3 these split its
VALU instructions between the orbit bodies and the per-trip work.  Each line
also gives the waves' real-time stamps in microseconds from the first
wave's start: when the queue was first and last found dry, the first, mean
and last exit, and the share of the waves' slots left empty before the last
exit (the end of the launch, where waves finish their last rays).  The
counters and checks change only what the kernels count, not what they
compute.

--check also renders with the per-pixel counter planes and requires that the
lanes the trip counters saw equal the planes' distance estimates and orbit
bodies; it then runs the degree batch, the 64-job Julia batch and the
adjoint of the differentiable set, and requires that no index check failed
in any of them (exit status 1 otherwise).
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NAMES = ("trips", "refills", "body_iterations", "step_paths", "claims", "live_lane_iterations", "step_lanes")
CHECKS = ("ray index", "pixel index", "job index", "list index")


def _checks(word):
    return [name for k, name in enumerate(CHECKS) if (int(word) >> k) & 1]


def wave_times(st):
    """Wave lifetimes from the real-time counter stamps (100 MHz ticks ->
    microseconds, from the earliest wave start): the mean, first and last
    exit, the first and last wave to find the queue dry, and the share of
    the waves' slots left idle before the last exit."""
    full = (1 << 64) - 1
    st = [int(v) for v in st]
    n = max(st[7], 1)
    t0 = full - st[1]
    us = lambda v: round((v - t0) / 100.0, 2)
    mean_exit = (st[6] / n - t0) / 100.0
    last = us(st[4])
    return {"waves": st[7], "start_spread_us": us(st[0]), "queue_dry_us": [us(full - st[3]), us(st[2])],
            "exit_us": {"first": us(full - st[5]), "mean": round(mean_exit, 2), "last": last},
            "tail_idle_frac": round(1.0 - mean_exit / last, 4) if last > 0 else 0.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--build", action="store_true", help="build libfrt_instr.so first")
    ap.add_argument("--check", action="store_true",
                    help="compare the trip counters with the counter planes and run more job sets under the "
                         "index checks (exit status 1 on any mismatch or failed check)")
    args = ap.parse_args()
    from paper_2102_01747_amd import _build

    if args.build:
        _build.build(instrument=True)
    import numpy as np
    import torch

    import paper_2102_01747_amd as frt
    import workloads as W

    if not os.path.exists(_build.INSTR_LIB):
        raise SystemExit("libfrt_instr.so is not built: run with --build")
    frt.LIB_PATH = _build.INSTR_LIB
    frt._lib = None
    frt.lib()
    dev = torch.device("cuda:0")
    jobs = W.bulb_views()
    frames = [frt.alloc_frame(j, dev, counters=args.check) for j in jobs]
    ws = frt.alloc_workspace(len(jobs), dev)
    for _ in range(2):
        frt.render_batch(jobs, dev, outs=frames, workspace=ws)
    torch.cuda.synchronize()
    raw = ws[512:776].cpu().numpy().view(np.uint64)
    rays = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    planes = None
    if args.check:
        # counter planes 1, 2: primary estimates and bodies; 6, 7: shadow ones
        planes = np.zeros(8, np.int64)
        for f in frames:
            planes += f["counters"].cpu().numpy().view(np.uint32).astype(np.int64).sum(axis=1)
    ok = True
    for stage, base in (("primary_march", 0), ("shadow_march", 16)):
        c = dict(zip(NAMES, (int(v) for v in raw[base:base + len(NAMES)])))
        c["stage"] = stage
        c["workload"] = "mandelbulb_n8_1920x1080_8views"
        c["rays"] = rays
        c["orbit_loop_lane_use"] = c["live_lane_iterations"] / (64.0 * c["body_iterations"]) if c["body_iterations"] else 0.0
        c["lanes_per_step_path"] = c["step_lanes"] / c["step_paths"] if c["step_paths"] else 0.0
        c["body_iterations_per_trip"] = c["body_iterations"] / c["trips"] if c["trips"] else 0.0
        c.update(wave_times(raw[base + len(NAMES):base + len(NAMES) + 8]))
        if planes is not None:
            est, bod = (planes[1], planes[2]) if base == 0 else (planes[6], planes[7])
            c["plane_estimates"], c["plane_bodies"] = int(est), int(bod)
            c["check"] = bool(c["step_lanes"] == est and c["live_lane_iterations"] == bod)
            ok &= c["check"]
        print(json.dumps(c), flush=True)
    failed = {"bench_views": _checks(raw[32])}
    if args.check:
        for name, js in (("degree_batch", W.julia_degree_batch()), ("julia_batch", W.julia_batch())):
            w2 = frt.alloc_workspace(len(js), dev)
            frt.render_batch(js, dev, workspace=w2)
            torch.cuda.synchronize()
            failed[name] = _checks(w2[768:776].cpu().numpy().view(np.uint64)[0])
        djobs, targets = W.diff_set()
        fr = frt.render_batch(djobs, dev)
        tf = frt.render_batch(targets, dev)
        gcs = [2.0 * (a["colour"] - b["colour"]) for a, b in zip(fr, tf)]
        w3 = frt.alloc_workspace(len(djobs), dev)
        frt.render_backward(djobs, fr, gcs, None, None, dev, workspace=w3)
        torch.cuda.synchronize()
        failed["diff_set_backward"] = _checks(w3[768:776].cpu().numpy().view(np.uint64)[0])
    print(json.dumps({"failed_checks": failed}), flush=True)
    ok &= all(not v for v in failed.values())
    if not ok:
        raise SystemExit(1)


if __name__ == "__main__":
    main()
