"""Trip statistics of the march kernels on the bench workload.

    python -m paper_2102_01747_amd.trip_counts [--build]

Loads the measurement build libfrt_trips.so (built with --build, or by
paper_2102_01747_amd._build.build(trip_counters=True)), renders the eight
1920 x 1080 Mandelbulb views of the bench as one batch, and prints one JSON
line per march stage: wave-level trips round the outer loop, orbit-loop
iterations, step paths, refills and claims, and the lanes they served.  With
a kernel's SQ_INSTS_VALU from rocprofv3 these split its VALU instructions
between the orbit bodies and the per-trip work.  The counters change only
what the kernels count, not what they compute.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NAMES = ("trips", "refills", "body_iterations", "step_paths", "claims", "live_lane_iterations", "step_lanes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--build", action="store_true", help="build libfrt_trips.so first")
    ap.add_argument("--check", action="store_true",
                    help="render with the per-pixel counter planes too and require that the lanes the trip "
                         "counters saw equal the planes' estimates and orbit bodies (exit status 1 otherwise)")
    args = ap.parse_args()
    from paper_2102_01747_amd import _build

    if args.build:
        _build.build(trip_counters=True)
    import numpy as np
    import torch

    import paper_2102_01747_amd as frt
    import workloads as W

    if not os.path.exists(_build.TRIPS_LIB):
        raise SystemExit("libfrt_trips.so is not built: run with --build")
    frt.LIB_PATH = _build.TRIPS_LIB
    frt._lib = None
    frt.lib()
    dev = torch.device("cuda:0")
    jobs = W.bulb_views()
    frames = [frt.alloc_frame(j, dev, counters=args.check) for j in jobs]
    ws = frt.alloc_workspace(len(jobs), dev)
    for _ in range(2):
        frt.render_batch(jobs, dev, outs=frames, workspace=ws)
    torch.cuda.synchronize()
    raw = ws[512:768].cpu().numpy().view(np.uint64)
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
        if planes is not None:
            est, bod = (planes[1], planes[2]) if base == 0 else (planes[6], planes[7])
            c["plane_estimates"], c["plane_bodies"] = int(est), int(bod)
            c["check"] = bool(c["step_lanes"] == est and c["live_lane_iterations"] == bod)
            ok &= c["check"]
        print(json.dumps(c), flush=True)
    if not ok:
        raise SystemExit(1)


if __name__ == "__main__":
    main()
