"""Benchmark: primary rays per second of the Mandelbulb sphere tracer on one MI355X.

Workload (one step): the eight 1920x1080 views of the power-8 Mandelbulb
(eye at radius 2.5, seeded azimuth/elevation, 10 orbit iterations, r > 2,
512 steps, eps = 5e-4 t, central-difference normals, one shadow ray per lit
hit), rendered in one persistent batch launch.  Inputs (camera and fractal
parameters) and output planes are resident in HBM before timing starts.

Prints one JSON line with the throughput, the roofline of the trace kernel
(algorithmic FP32 FLOP per launch over its HIP-event-measured duration, against
the 157.3 TFLOP/s FP32 vector peak) and the FP64 CPU oracle timed on a
bounded pixel sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "primary Mrays/s + % FP32 VALU peak; adjoint grads/s vs FD at rel err 1e-3"
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X: 256 CU x 2.4 GHz x 256 FLOP/clk/CU

# Algorithmic FLOP per unit (FMA = 2, add/mul = 1, elementary function = 1):
#   one orbit body: Julia z^2+c 24; Mandelbulb power map with its derivative 30
#   (20 arithmetic + 10 elementary functions), whichever kernel path runs it;
#   one distance evaluation outside the bodies: 16 (sample point 6, estimate
#   tail 6, step update and stop test 4).
FLOP_PER_BODY = {"julia": 24.0, "bulb": 30.0}
FLOP_PER_EVAL = 16.0


def algorithmic_flop(kind, counters):
    evals = counters[1].astype("float64").sum()
    bodies = counters[2].astype("float64").sum()
    return FLOP_PER_BODY[kind] * bodies + FLOP_PER_EVAL * evals, evals, bodies


def cpu_baseline(jobs, stride):
    import numpy as np

    import workloads as W
    from oracle import oracle as orc

    n = 0
    t0 = time.perf_counter()
    for v, job in enumerate(jobs):
        pix = W.stratified_pixels(job["camera"]["width"], job["camera"]["height"], stride, seed=100 + v)
        orc.render(job, pixels=pix)
        n += pix.size
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": orc.max_threads(), "kind": "oracle",
            "sample": "FP64 oracle on one pixel per %dx%d cell of each of the %d views (%d rays, %.1f s), "
                      "same shading and shadow rays" % (stride, stride, len(jobs), n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["batch", "single"], default="batch")
    ap.add_argument("--cpu-stride", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (to scale HBM byte counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured by rocprofv3 counters (JSON), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2102_01747_amd as frt
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4}), flush=True)
        return
    jobs = W.bulb_views()
    rays = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    frames = [frt.alloc_frame(j, dev) for j in jobs]
    ws = frt.alloc_workspace(len(jobs), dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        if args.mode == "batch":
            frt.render_batch(jobs, dev, outs=frames, workspace=ws)
        else:
            for j, f in zip(jobs, frames):
                frt.render(j, dev, out=f, workspace=ws)

    # algorithmic work of one step, from the per-pixel counters (untimed)
    cframes = [frt.alloc_frame(j, dev, counters=True) for j in jobs]
    frt.render_batch(jobs, dev, outs=cframes, workspace=ws)
    torch.cuda.synchronize()
    flop = 0.0
    for f in cframes:
        fl, _, _ = algorithmic_flop("bulb", f["counters"].cpu().numpy().view(np.uint32))
        flop += fl
    del cframes

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = wall * 1e3 / args.steps
    launch_ms = float(np.mean(ms))
    achieved = flop / (launch_ms * 1e-3) / 1e12

    traffic = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as fh:
                tr = json.load(fh)
            if tr.get("workload") == "mandelbulb_n8_1920x1080_8views" and tr.get("mode") == args.mode:
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None

    rec = {
        "metric": METRIC,
        "value": rays / (ms_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mandelbulb_n8_1920x1080_8views", "views": len(jobs), "width": 1920, "height": 1080,
                   "power": 8, "max_iter": 10, "max_steps": 512, "eps_rel": 5e-4, "normals": "central",
                   "shadow": True, "launch": args.mode, "primary_rays_per_step": rays},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "trace_kernel (persistent, Mandelbulb integer power)",
                     "flop_per_launch": flop, "launch_ms": launch_ms},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(jobs, args.cpu_stride)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
