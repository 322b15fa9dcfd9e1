"""Benchmark: primary rays per second of the Mandelbulb sphere tracer on one MI355X.

Workload (one step): the eight 1920x1080 views of the power-8 Mandelbulb
(eye at radius 2.5, seeded azimuth/elevation, 10 orbit iterations, r > 2,
512 steps, eps = 5e-4 t, central-difference normals, one shadow ray per lit
hit), rendered in one batch (primary-march, normal and shadow-march kernels,
each one launch over all eight views).  Inputs (camera and fractal
parameters) and output planes are resident in HBM before timing starts.

The launch configuration is the one the autotuner recorded for this kernel
variant (paper_2102_01747_amd/tuned.json; --tune searches again, untimed).  Prints one JSON line with
the throughput, the roofline of the dominant kernel (algorithmic FP32 FLOP
per launch over its duration measured with HIP events on its stream, against
the 157.3 TFLOP/s FP32 vector peak), the same figures for every stage, the
adjoint leg (gradients per second of the differentiable set, backward over
forward cost, and the finite-difference gradient it replaces), and the FP64
CPU oracle timed on a bounded pixel sample of the same workload on the host
cores.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "primary Mrays/s + % FP32 VALU peak; adjoint grads/s vs FD at rel err 1e-3"
WORKLOAD = "mandelbulb_n8_1920x1080_8views"
# --workload stress: the 4K power sweep (64 frames, n = 2 + 14 f / 63)
STRESS = "mandelbulb_sweep_n2_16_3840x2160_64frames"
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X: 256 CU x 2.4 GHz x 256 FLOP/clk/CU (packed FP32)
FP32_NONPACKED_PEAK_TFLOPS = 78.6   # the same without packed FP32, which this build does not emit

# Algorithmic FLOP per unit (FMA = 2, add/mul = 1, elementary function = 1):
#   one orbit body: Julia z^2+c 24; Mandelbulb power map with its derivative 30
#   (20 arithmetic + 10 elementary functions), whichever kernel path runs it;
#   one distance evaluation outside the bodies: 16 (sample point 6, estimate
#   tail 6, step update and stop test 4).
FLOP_PER_BODY = {"julia": 24.0, "bulb": 30.0}
# Bytes the primary march must write: float depth + status byte per ray, and
# float3 normal + float3 colour (zeros) per miss.
PRIMARY_BYTES_PER_RAY = 5
MISS_EXTRA_BYTES = 24
FLOP_PER_EVAL = 16.0
STAGES = ("primary_march", "normals", "shadow_march")


# sources of the forward kernels; the recorded HBM traffic is used only while
# they are unchanged since the counters were taken
KERNEL_SOURCES = ("frt_trace.hip", "frt_fractal.hpp", "frt_math.hpp", "frt_ray.hpp", "frt_job.hpp", "frt_normal.hpp",
                  "frt_gradient.hpp")


# sources of the adjoint kernels, for the recorded FP64 work per backward call
ADJOINT_SOURCES = ("frt_adjoint.hip", "frt_fractal.hpp", "frt_math.hpp", "frt_ray.hpp", "frt_job.hpp",
                   "frt_internal.hpp")
FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X FP64 vector


def kernel_sources_sha256(names=KERNEL_SOURCES):
    """SHA-256 of kernel code: the sources with comments and whitespace
    removed, so that an edit of a comment keeps the profiled figures (the
    sources hold no string literal with a comment marker), and the extra
    compile flags the build gives any of them."""
    import hashlib
    import re

    from paper_2102_01747_amd import _build

    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2102_01747_amd", "csrc", name)) as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
        if _build.SOURCE_FLAGS.get(name):
            h.update((" flags: " + " ".join(_build.SOURCE_FLAGS[name])).encode())
    return h.hexdigest()


def stage_flop(kind, counters):
    """Algorithmic FLOP of each stage from the per-pixel counter planes
    (1/2 primary evaluations/bodies, 4/5 normal taps, 6/7 shadow rays)."""
    c = counters.astype("float64")
    return [FLOP_PER_BODY[kind] * c[bo].sum() + FLOP_PER_EVAL * c[ev].sum() for ev, bo in ((1, 2), (4, 5), (6, 7))]


def cpu_baseline(jobs, target_s=20.0):
    """The FP64 oracle on the host cores over a stratified pixel sample of
    the same views: a stride-16 probe sets the rate, then the densest stride
    expected to finish in about `target_s` seconds is timed."""
    import workloads as W
    from oracle import oracle as orc

    def run(stride):
        n = 0
        t0 = time.perf_counter()
        for v, job in enumerate(jobs):
            pix = W.stratified_pixels(job["camera"]["width"], job["camera"]["height"], stride, seed=100 + v)
            orc.render(job, pixels=pix)
            n += pix.size
        return n, time.perf_counter() - t0

    n, dt = run(16)
    rate = n / dt
    total = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    stride = 16
    for s in (1, 2, 3, 4, 6, 8, 12):
        if total / (s * s) / rate <= target_s:
            stride = s
            break
    if stride != 16:
        n, dt = run(stride)
    cores = orc.max_threads()
    # one thread on the stride-16 sample (1/256 of the rays)
    n1, dt1 = 0, 0.0
    for v, job in enumerate(jobs):
        pix = W.stratified_pixels(job["camera"]["width"], job["camera"]["height"], 16, seed=300 + v)
        t0 = time.perf_counter()
        orc.render(job, pixels=pix, threads=1)
        dt1 += time.perf_counter() - t0
        n1 += pix.size
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle (OpenMP over rays) on one pixel per %dx%d cell of each of the %d views "
                      "(%d of %d rays, %.1f s), same normals and shadow rays" % (stride, stride, len(jobs), n, total, dt),
            "single_core": {"value": n1 / dt1 / 1e6, "unit": "Mrays/s",
                            "sample": "one thread, one pixel per 16x16 cell (%d rays, %.1f s)" % (n1, dt1)},
            "cpu_model": host_cpu_model()}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def timed_median(fn, reps, windows=5):
    """Per-call milliseconds of fn: one untimed call, then `windows` windows of
    `reps` back-to-back calls between HIP events on the current stream, and
    the median window (a host stall inside one short window would otherwise
    set the figure)."""
    import torch

    fn()
    torch.cuda.synchronize()
    per = []
    for _ in range(windows):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        per.append(s.elapsed_time(e) / reps)
    return sorted(per)[len(per) // 2]


TIMING = "median of 5 windows of back-to-back calls (HIP events on the current stream)"


def adjoint_leg(frt, dev, reps):
    """Differentiable set: 8 Julia + 8 Mandelbulb renders of 512x512 with a
    cut plane, loss = squared colour error to target renders at offset
    parameters.  Times the forward batch and the adjoint launch (HIP events
    on the current stream, the median of 5 windows), and the finite-difference gradient the adjoint
    replaces: central differences need 2 P renders per job (P parameters:
    c and plane for Julia, n and plane for the Mandelbulb), issued as 2 max(P)
    batch renders with one parameter of every job offset."""
    import torch

    import workloads as W
    from paper_2102_01747_amd.autograd import job_params, job_with_params

    jobs, targets = W.diff_set()
    frames = frt.render_batch(jobs, dev)
    tframes = frt.render_batch(targets, dev)
    torch.cuda.synchronize()
    gc = [2.0 * (f["colour"] - t["colour"]) for f, t in zip(frames, tframes)]
    ws_f = frt.alloc_workspace(len(jobs), dev)
    ws_b = frt.alloc_workspace(len(jobs), dev)
    grads = None

    def timed(fn):
        return timed_median(fn, reps)

    def backward():
        nonlocal grads
        grads = frt.render_backward(jobs, frames, gc, None, None, dev, workspace=ws_b, grads=grads)

    t_f = timed(lambda: frt.render_batch(jobs, dev, outs=frames, workspace=ws_f))
    t_b = timed(backward)
    slots = [[0, 1, 2, 3, 5, 6, 7, 8] if j["fractal"]["kind"] == "julia" else [4, 5, 6, 7, 8] for j in jobs]
    n_fd = 2 * max(len(sl) for sl in slots)
    pert = []
    for k in range(n_fd):
        batch = []
        for j, sl in zip(jobs, slots):
            row = job_params(j)
            row[sl[(k // 2) % len(sl)]] += 1e-5 if k % 2 == 0 else -1e-5
            batch.append(job_with_params(j, row))
        pert.append(batch)
    fd_frames = [frt.alloc_frame(j, dev) for j in jobs]

    def fd_all():
        for batch in pert:
            frt.render_batch(batch, dev, outs=fd_frames, workspace=ws_f)

    t_fd = timed(fd_all)
    n = len(jobs)
    # the adjoint kernels' FP64 work: hardware FP64 FLOP on active lanes per
    # backward call, from the PMC profile of the same sources, over this run's
    # backward time
    roof = None
    path = os.path.join(ROOT, "profiles", "adjoint_fp64.json")
    if os.path.exists(path):
        try:
            with open(path) as fh:
                pr = json.load(fh)
            if (pr.get("workload") == "julia8_mandelbulb8_512x512_cut_plane"
                    and pr.get("adjoint_sources_sha256") == kernel_sources_sha256(ADJOINT_SOURCES)):
                fl = float(pr["hw_fp64_flop_per_call"])
                ach = fl / (t_b * 1e-3) / 1e12
                roof = {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "flop_per_call": fl,
                        "flop_kind": "hardware FP64 on active lanes (SQ_INSTS_VALU_FLOPS_FP64 x 64 x VALUUtilization)",
                        "traffic": pr.get("bytes_per_call")}
        except (OSError, ValueError, KeyError):
            roof = None
    return {"workload": "julia8_mandelbulb8_512x512_cut_plane", "renders": n, "roofline": roof,
            "grads_per_s": n / ((t_f + t_b) * 1e-3), "forward_ms": t_f, "backward_ms": t_b,
            "backward_over_forward": t_b / t_f, "fd_renders_per_gradient": "2 x (8 Julia / 5 Mandelbulb parameters)",
            "fd_grads_per_s": n / (t_fd * 1e-3), "speedup_vs_fd": (t_fd) / (t_f + t_b),
            "rel_err_target": 1e-3, "timing": TIMING}


def batch_leg(frt, dev, reps):
    """The batched-launch target: the 64 uneven Julia renders of the batch
    workload (seeded c, cut plane, resolution, iterations and eps) launched
    one by one (frt_render, one stream, one workspace), as one batch
    (frt_render_batch) and as a replayed HIP graph of that batch; times from
    events on the current stream (the median of 5 windows), speedups over
    one by one."""
    import workloads as W

    jobs = W.julia_batch()
    frames = [frt.alloc_frame(j, dev) for j in jobs]
    ws = frt.alloc_workspace(len(jobs), dev)
    ws1 = frt.alloc_workspace(1, dev)

    def timed(fn):
        return timed_median(fn, reps)

    t_one = timed(lambda: [frt.render(j, dev, out=f, workspace=ws1) for j, f in zip(jobs, frames)])
    t_batch = timed(lambda: frt.render_batch(jobs, dev, outs=frames, workspace=ws))
    t_graph = timed(lambda: frt.render_batch(jobs, dev, outs=frames, workspace=ws, use_graph=True))
    frt.graph_reset()
    rays = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    return {"workload": "julia_batch_64_uneven", "renders": len(jobs), "rays": rays,
            "one_by_one_ms": t_one, "batched_ms": t_batch, "graph_ms": t_graph,
            "speedup": t_one / t_batch, "speedup_graph": t_one / t_graph,
            "batched_mrays_per_s": rays / (t_batch * 1e-3) / 1e6, "target_speedup": 2.0, "timing": TIMING}


def hardware_fp32(flop, launch_ms):
    """FP32 FLOP the dominant kernel issues on active lanes per launch (rocprofv3
    SQ_INSTS_VALU_FLOPS_FP32 x 64 x VALUUtilization, from the profile of the
    same sources and launch configuration), over this run's launch time."""
    if flop is None or launch_ms <= 0:
        return None
    tf = flop / (launch_ms * 1e-3) / 1e12
    return {"flop_per_launch": flop, "tflops": tf, "frac": tf / FP32_VECTOR_PEAK_TFLOPS,
            "frac_of_nonpacked": tf / FP32_NONPACKED_PEAK_TFLOPS}


def measured_ceilings(frt, dev, achieved):
    """Sustained FP32 FMA and transcendental issue rates of this device under
    the build's code generation (packed FP32 off), from the library's rate
    probes; the dominant kernel's algorithmic rate as a fraction of the
    measured FMA ceiling."""
    fma = frt.valu_rate("fma", 16384, dev) * 2 / 1e12          # TFLOP/s, FMA = 2
    trans = {op: frt.valu_rate(op, 4096, dev) / 1e12 for op in ("exp2", "log2", "rsq", "sin_rev")}
    return {"measured_fma_tflops": fma, "frac_of_measured_fma": achieved / fma,
            "measured_trans_tops": trans}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["batch", "single"], default="batch")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the vector-unit rate probes")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch leg")
    ap.add_argument("--tune", action="store_true",
                    help="re-run the autotuner on this workload before timing (default: the recorded tuned.json)")
    ap.add_argument("--workload", choices=["bulb_views", "stress"], default="bulb_views",
                    help="bulb_views: 8 x 1920x1080 Mandelbulb n = 8 (the benchmark); stress: the 4K power sweep")
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

    jobs = W.bulb_views() if args.workload == "bulb_views" else W.stress_sweep()
    wl_name = WORKLOAD if args.workload == "bulb_views" else STRESS
    rays = sum(j["camera"]["width"] * j["camera"]["height"] for j in jobs)
    frames = [frt.alloc_frame(j, dev) for j in jobs]
    ws = frt.alloc_workspace(len(jobs), dev)

    def step():
        if args.mode == "batch":
            frt.render_batch(jobs, dev, outs=frames, workspace=ws)
        else:
            for j, f in zip(jobs, frames):
                frt.render(j, dev, out=f, workspace=ws)

    from paper_2102_01747_amd import autotune

    if args.tune:
        autotune.tune(jobs, batch=(args.mode == "batch"), reps=3, passes=2, device=dev)
    variants = autotune.variants_of(jobs)
    launch_cfg = {v: dict(zip(autotune.KEYS, frt.autotune_get(v))) for v in variants}

    # algorithmic work of one step, from the per-pixel counters (untimed)
    cframes = [frt.alloc_frame(j, dev, counters=True) for j in jobs]
    frt.render_batch(jobs, dev, outs=cframes, workspace=ws)
    torch.cuda.synchronize()
    flops = np.zeros(3)
    misses = 0
    for f in cframes:
        flops += np.array(stage_flop("bulb", f["counters"].cpu().numpy().view(np.uint32)))
        misses += int(((f["status"] & 7) < 2).sum())
    del cframes
    # the primary march's algorithmic output: depth and status of every ray,
    # plus the zero normal and colour of every miss (hits get theirs from the
    # normal kernel); its reads are the job table only
    out_bytes = PRIMARY_BYTES_PER_RAY * rays + MISS_EXTRA_BYTES * misses

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps

    # per-kernel durations: HIP events recorded by the library on the launch
    # stream around each stage, over the same number of steps
    frt.set_stage_timing(True)
    per_stage = np.zeros(3)
    for _ in range(args.steps):
        if args.mode == "batch":
            step()
            per_stage += np.array(frt.stage_times())
        else:
            for j, f in zip(jobs, frames):
                frt.render(j, dev, out=f, workspace=ws)
                per_stage += np.array(frt.stage_times())
    frt.set_stage_timing(False)
    per_stage /= args.steps
    stages = {}
    for k, name in enumerate(STAGES):
        ach = flops[k] / (per_stage[k] * 1e-3) / 1e12 if per_stage[k] > 0 else 0.0
        stages[name] = {"ms": float(per_stage[k]), "flop": float(flops[k]), "achieved_tflops": ach,
                        "frac": ach / FP32_VECTOR_PEAK_TFLOPS}
    dom = max(STAGES, key=lambda n: stages[n]["ms"])
    achieved = stages[dom]["achieved_tflops"]

    traffic = None
    hw_flop = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as fh:
                tr = json.load(fh)
            if (tr.get("workload") == wl_name and tr.get("stage") == dom and len(variants) == 1
                    and tr.get("launch_config") == launch_cfg[variants[0]]
                    and tr.get("kernel_sources_sha256") == kernel_sources_sha256()):
                traffic = tr.get("bytes_per_launch")
                hw_flop = tr.get("hw_fp32_flop_per_launch")
        except (OSError, ValueError):
            traffic = None

    variant = "+".join(variants)
    if args.workload == "bulb_views":
        config = {"workload": WORKLOAD, "views": len(jobs), "width": 1920, "height": 1080, "power": 8,
                  "max_iter": 10, "max_steps": 512, "eps_rel": 5e-4, "normals": "central", "shadow": True,
                  "launch": args.mode, "primary_rays_per_step": rays}
    else:
        config = {"workload": STRESS, "frames": len(jobs), "width": 3840, "height": 2160, "power": "2 + 14 f / 63",
                  "max_iter": 15, "max_steps": 1024, "eps_rel": 2e-4, "normals": "central", "shadow": False,
                  "plane": "z <= 0.1", "launch": args.mode, "primary_rays_per_step": rays}
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
        "config": config,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": ("normal_kernel<%s>" if dom == "normals" else "march_kernel<%s>") % variant,
                     "stage": dom, "flop_per_launch": stages[dom]["flop"], "launch_ms": stages[dom]["ms"],
                     "peak_nonpacked_fp32": FP32_NONPACKED_PEAK_TFLOPS,
                     "frac_of_nonpacked": achieved / FP32_NONPACKED_PEAK_TFLOPS,
                     "algorithmic_bytes": float(out_bytes) if dom == "primary_march" else None,
                     "traffic_over_algorithmic": (traffic / out_bytes) if (traffic and dom == "primary_march")
                     else None},
        "stages": stages,
        "hardware_fp32": hardware_fp32(hw_flop, stages[dom]["ms"]),
        "whole_path_tflops": float(flops.sum() / (ms_step * 1e-3) / 1e12),
        "launch_config": launch_cfg,
    }
    if not args.no_ceilings:
        rec["roofline"].update(measured_ceilings(frt, dev, achieved))
    if not args.no_adjoint and args.workload == "bulb_views":
        rec["adjoint"] = adjoint_leg(frt, dev, max(3, args.steps // 4))
    if not args.no_batch and args.workload == "bulb_views":
        rec["batch"] = batch_leg(frt, dev, max(3, args.steps // 4))
    if not args.no_cpu_baseline and args.workload == "bulb_views":
        rec["cpu_baseline"] = cpu_baseline(jobs, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
