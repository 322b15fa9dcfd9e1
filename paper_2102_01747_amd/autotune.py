"""Autotuner for the persistent trace kernels.

For a list of jobs (rendered as one batch launch, or one launch per job),
searches the launch configuration of the kernel variant the jobs use --
block size, rays claimed per queue refill (chunk), resident waves per SIMD
the grid is sized for, orbit bodies per loop trip and the number of waiting
lanes that triggers shading/refill -- by coordinate descent from the current
setting, timing each candidate with HIP events on the current stream (median
of `reps` launches after one warm-up).  The best setting is installed with
frt_autotune_set and can be cached in a JSON file keyed by variant and a
workload tag.
"""
import json
import os
import statistics

import torch

from . import VARIANTS, alloc_frame, alloc_workspace, autotune_get, autotune_set, render, render_batch

SPACE = {
    "block": [64, 128, 256, 512],
    "chunk": [64, 128, 256, 512, 1024],
    "waves_per_simd": [2, 4, 6, 8, 0],
    "orbit_lanes": [1, 4, 8, 12, 16, 24, 32, 48],
    "rare_lanes": [2, 4, 8, 16, 24, 32, 48],
}
KEYS = ["block", "chunk", "waves_per_simd", "orbit_lanes", "rare_lanes"]


def variants_of(jobs):
    """Kernel variants the library traces these jobs with (one group each)."""
    out = []
    for j in jobs:
        fr = j["fractal"]
        if fr["kind"] == "julia":
            v = "julia" if float(fr.get("power", 2.0)) == 2.0 else "julia_deg"
        else:
            n = float(fr["power"])
            v = "bulb8" if n == 8.0 else ("bulb_int" if n.is_integer() and 2 <= n <= 64 else "bulb_real")
        if v not in out:
            out.append(v)
    return out


def variant_of(jobs):
    """The single variant of a one-variant job list."""
    vs = variants_of(jobs)
    if len(vs) != 1:
        raise ValueError("jobs use several kernel variants: %s" % vs)
    return vs[0]


def time_config(jobs, frames, ws, batch, reps=5, device="cuda"):
    stream = torch.cuda.current_stream(device)

    def launch():
        if batch:
            render_batch(jobs, device, outs=frames, workspace=ws)
        else:
            for j, f in zip(jobs, frames):
                render(j, device, out=f, workspace=ws)

    launch()
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        launch()
        e.record(stream)
        e.synchronize()
        times.append(s.elapsed_time(e))
    return statistics.median(times)


def tune(jobs, batch=True, reps=5, passes=2, device="cuda", log=None, variants=None):
    """Coordinate descent over SPACE for every variant the jobs use (or the
    given subset; each timed on the whole batch, the others held at their
    current setting); installs the best settings and returns them per
    variant with the time."""
    frames = [alloc_frame(j, device) for j in jobs]
    ws = alloc_workspace(len(jobs), device)
    results = []
    for var in variants_of(jobs):
        if variants is not None and var not in variants:
            continue
        cur = dict(zip(KEYS, autotune_get(var)))
        timed = {}

        def measure(cfg):
            key = tuple(cfg[k] for k in KEYS)
            if key not in timed:
                autotune_set(var, *key)
                timed[key] = time_config(jobs, frames, ws, batch, reps, device)
                if log:
                    log("  %s %s %.3f ms" % (var, dict(zip(KEYS, key)), timed[key]))
            return timed[key]

        best = measure(cur)
        for _ in range(passes):
            improved = False
            for k in KEYS:
                for v in SPACE[k]:
                    cand = dict(cur, **{k: v})
                    t = measure(cand)
                    if t < best * 0.995:
                        best, cur, improved = t, cand, True
            if not improved:
                break
        autotune_set(var, *[cur[k] for k in KEYS])
        results.append({"variant": var, "config": cur, "ms": best, "candidates": len(timed)})
    return results


TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def save_tuned(result, workload, path=TUNED_PATH):
    """Record a tune() result as the installed default of its kernel variant
    (the binding installs tuned.json when it loads the library)."""
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    entry = dict(result["config"])
    entry["workload"] = workload
    entry["ms"] = round(float(result["ms"]), 4)
    data[result["variant"]] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")


def main():
    """Tune the launch configuration on one of the reference workloads and
    record it in tuned.json: python -m paper_2102_01747_amd.autotune WORKLOAD
    with WORKLOAD one of bulb_views (8 x 1080p Mandelbulb, n = 8),
    julia_batch (64 uneven Julia renders), julia_degree_batch (32 Julia
    renders of degree 3-6), diff_set (16 x 512^2, Julia and Mandelbulb),
    stress (the 4K power sweep: real and integer powers)."""
    import argparse
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["bulb_views", "julia_batch", "julia_degree_batch", "diff_set", "stress"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--out", default=TUNED_PATH)
    ap.add_argument("--variants", nargs="*", default=None,
                    help="tune only these kernel variants (default: every variant the workload uses)")
    args = ap.parse_args()
    jobs = {"bulb_views": W.bulb_views, "julia_batch": W.julia_batch, "julia_degree_batch": W.julia_degree_batch,
            "diff_set": lambda: W.diff_set()[0], "stress": W.stress_sweep}[args.workload]()
    for res in tune(jobs, batch=True, reps=args.reps, passes=args.passes, log=lambda m: print(m, flush=True),
                    variants=args.variants):
        print(json.dumps(res), flush=True)
        save_tuned(res, args.workload, args.out)


if __name__ == "__main__":
    main()
