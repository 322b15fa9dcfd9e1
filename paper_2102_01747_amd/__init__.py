"""MI355X fractal sphere tracer -- Python binding of libfrt.so.

Argument marshalling only: every step of a render (ray generation, bounding
interval, cut face, march, refinement, normals, shading, shadow ray, adjoint)
runs in the HIP kernels of libfrt.so.  PyTorch supplies device memory and the
stream.  Jobs are the plain dictionaries of ``workloads.py``.

The library must have been built (``python -m paper_2102_01747_amd._build``
or ``__graft_entry__.build()``); importing the functions below without it
raises ``FrtError``.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# FRT_LIB_PATH selects another build of the same sources (the host-sanitised
# build of the CPU checks); by default the in-tree libfrt.so
LIB_PATH = os.environ.get("FRT_LIB_PATH") or os.path.join(_PKG, "libfrt.so")

FRT_OK, FRT_EINVAL, FRT_EHIP, FRT_ENOMEM, FRT_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS_MISS_BOUNDS, STATUS_MISS_TMAX, STATUS_HIT, STATUS_HIT_CUT, STATUS_HIT_EXHAUSTED = 0, 1, 2, 3, 4
FLAG_SHADOWED, FLAG_UNREFINED, FLAG_SHADOW_RAY = 8, 16, 64
NORMAL_MODES = {"tetra": 0, "central": 1, "analytic": 2}
SHADING_MODELS = {"lambert": 0, "phong": 1}
FLAG_REFLECT_HIT = 128
VARIANTS = {"julia": 0, "bulb_real": 1, "bulb_int": 2, "bulb8": 3, "julia_deg": 4}

f3 = ctypes.c_float * 3
f4 = ctypes.c_float * 4


class FrtError(RuntimeError):
    pass


class Camera(ctypes.Structure):
    _fields_ = [("eye", f3), ("target", f3), ("up", f3), ("fov_y_deg", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Fractal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c", f4), ("power", ctypes.c_float), ("max_iter", ctypes.c_int32),
                ("bailout2", ctypes.c_float), ("bound_radius", ctypes.c_float)]


class Plane(ctypes.Structure):
    _fields_ = [("n", f3), ("d", ctypes.c_float)]


class March(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("eps_abs", ctypes.c_float), ("eps_rel", ctypes.c_float),
                ("step_clamp", ctypes.c_float), ("t_max", ctypes.c_float), ("normal_mode", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("shadow", ctypes.c_int32), ("light_dir", f3), ("albedo", f3),
                ("k_ambient", ctypes.c_float), ("k_diffuse", ctypes.c_float), ("shading", ctypes.c_int32),
                ("k_specular", ctypes.c_float), ("shininess", ctypes.c_float), ("k_reflect", ctypes.c_float),
                ("trap_colour", ctypes.c_float * 12)]


class Frame(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("colour", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("counters", ctypes.c_void_p)]


class Object(ctypes.Structure):
    _fields_ = [("frac", Fractal), ("planes", Plane * 2), ("n_planes", ctypes.c_int32),
                ("rotation", ctypes.c_float * 9), ("translation", f3), ("scale", ctypes.c_float)]


class Job(ctypes.Structure):
    _fields_ = [("cam", Camera), ("frac", Fractal), ("planes", Plane * 2), ("n_planes", ctypes.c_int32),
                ("march", March), ("out", Frame)]


_lib = None


def lib():
    """The loaded libfrt.so; raises FrtError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FrtError("libfrt.so is not built (%s); run paper_2102_01747_amd._build.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER
        L.frt_workspace_bytes.argtypes = [i32]
        L.frt_workspace_bytes.restype = sz
        L.frt_render.argtypes = [P(Camera), P(Fractal), P(Plane), i32, P(March), Frame, vp, sz, vp]
        L.frt_render.restype = ctypes.c_int
        L.frt_render_batch.argtypes = [P(Job), i32, vp, sz, i32, vp]
        L.frt_render_batch.restype = ctypes.c_int
        L.frt_render_batch_noalloc.argtypes = [P(Job), i32, vp]
        L.frt_render_batch_noalloc.restype = ctypes.c_int
        L.frt_noalloc_scratch_bytes.argtypes = []
        L.frt_noalloc_scratch_bytes.restype = sz
        L.frt_render_backward.argtypes = [P(Job), i32, P(vp), P(vp), P(vp), P(vp), vp, vp, vp, vp, sz, vp]
        L.frt_render_backward.restype = ctypes.c_int
        L.frt_autotune_set.argtypes = [i32, i32, i32, i32, i32, i32]
        L.frt_autotune_set.restype = ctypes.c_int
        L.frt_autotune_get.argtypes = [i32, P(i32), P(i32), P(i32), P(i32), P(i32)]
        L.frt_autotune_get.restype = ctypes.c_int
        L.frt_graph_reset.argtypes = []
        L.frt_graph_reset.restype = ctypes.c_int
        L.frt_distance.argtypes = [P(Fractal), vp, ctypes.c_int64, vp, vp, vp]
        L.frt_distance.restype = ctypes.c_int
        L.frt_normal_at.argtypes = [P(Fractal), i32, vp, vp, ctypes.c_int64, vp, vp]
        L.frt_scene_workspace_bytes.argtypes = [i32]
        L.frt_scene_workspace_bytes.restype = ctypes.c_size_t
        L.frt_render_scene.argtypes = [P(Camera), P(Object), i32, P(March), Frame, vp, vp, vp, ctypes.c_size_t, vp]
        L.frt_render_scene.restype = ctypes.c_int
        L.frt_normal_at.restype = ctypes.c_int
        L.frt_math_eval.argtypes = [i32, vp, vp, vp, ctypes.c_int64, vp]
        L.frt_math_eval.restype = ctypes.c_int
        L.frt_valu_rate.argtypes = [i32, i32, P(ctypes.c_double), vp]
        L.frt_valu_rate.restype = ctypes.c_int
        L.frt_set_stage_timing.argtypes = [i32]
        L.frt_set_stage_timing.restype = ctypes.c_int
        L.frt_stage_times.argtypes = [P(ctypes.c_float)]
        L.frt_stage_times.restype = ctypes.c_int
        L.frt_status_string.argtypes = [ctypes.c_int]
        L.frt_status_string.restype = ctypes.c_char_p
        L.frt_last_error.argtypes = []
        L.frt_last_error.restype = ctypes.c_char_p
        _lib = L
        _install_tuned(L)
    return _lib


TUNED_PATH = os.path.join(_PKG, "tuned.json")


def _install_tuned(L):
    """Install the launch configurations the autotuner recorded on MI355X
    (tuned.json, one entry per kernel variant), if present."""
    if not os.path.exists(TUNED_PATH):
        return
    import json

    with open(TUNED_PATH) as fh:
        data = json.load(fh)
    for var, c in data.items():
        st = L.frt_autotune_set(VARIANTS[var], int(c["block"]), int(c["chunk"]), int(c["waves_per_simd"]),
                                int(c["orbit_lanes"]), int(c["rare_lanes"]))
        if st != FRT_OK:
            raise FrtError("tuned.json entry %s rejected: %s" % (var, L.frt_last_error().decode()))


def _check(status):
    if status != FRT_OK:
        L = lib()
        raise FrtError("%s: %s" % (L.frt_status_string(status).decode(), L.frt_last_error().decode()))


# --------------------------------------------------------------- marshalling
def make_camera(cam):
    return Camera(f3(*cam["eye"]), f3(*cam["target"]), f3(*cam["up"]), float(cam["fov_y_deg"]),
                  int(cam["width"]), int(cam["height"]))


def make_fractal(fr):
    kind = {"julia": 0, "bulb": 1}[fr["kind"]] if isinstance(fr["kind"], str) else int(fr["kind"])
    return Fractal(kind, f4(*fr.get("c", (0.0, 0.0, 0.0, 0.0))), float(fr.get("power", 2.0)), int(fr["max_iter"]),
                   float(fr["bailout2"]), float(fr.get("bound_radius", 0.0)))


def make_planes(planes):
    arr = (Plane * 2)()
    for k, pl in enumerate(planes):
        arr[k] = Plane(f3(*pl["n"]), float(pl["d"]))
    return arr, len(planes)


def make_march(m):
    mode = NORMAL_MODES[m["normal_mode"]] if isinstance(m["normal_mode"], str) else int(m["normal_mode"])
    return March(int(m["max_steps"]), float(m["eps_abs"]), float(m["eps_rel"]), float(m["step_clamp"]),
                 float(m["t_max"]), mode, int(m.get("refine_iters", 12)), int(bool(m["shadow"])),
                 f3(*m["light_dir"]), f3(*m["albedo"]), float(m["k_ambient"]), float(m["k_diffuse"]),
                 SHADING_MODELS[m.get("shading", "lambert")], float(m.get("k_specular", 0.0)),
                 float(m.get("shininess", 1.0)), float(m.get("k_reflect", 0.0)),
                 (ctypes.c_float * 12)(*[float(x) for row in m.get("trap_colour", [[0.0] * 3] * 4) for x in row]))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _device(device):
    d = torch.device(device)
    if d.type != "cuda":
        raise FrtError("the renderer runs on a GPU device, got %s" % d)
    if d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def alloc_frame(job, device="cuda", counters=False):
    """Output planes of one job (see include/frt.h for the layout)."""
    cam = job["camera"]
    P = int(cam["width"]) * int(cam["height"])
    dev = _device(device)
    fr = {"depth": torch.empty(P, device=dev, dtype=torch.float32),
          "normal": torch.empty(3, P, device=dev, dtype=torch.float32),
          "colour": torch.empty(3, P, device=dev, dtype=torch.float32),
          "status": torch.empty(P, device=dev, dtype=torch.uint8)}
    if counters:
        fr["counters"] = torch.empty(8, P, device=dev, dtype=torch.int32)   # read as uint32
    return fr


def make_frame(fr):
    return Frame(_ptr(fr["depth"]), _ptr(fr["normal"]), _ptr(fr["colour"]), _ptr(fr["status"]),
                 _ptr(fr.get("counters")))


def workspace_bytes(n_jobs):
    return int(lib().frt_workspace_bytes(int(n_jobs)))


def alloc_workspace(n_jobs, device="cuda"):
    ws = torch.empty(workspace_bytes(n_jobs) + 256, device=_device(device), dtype=torch.uint8)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + workspace_bytes(n_jobs)]


def make_job(job, frame):
    pl, npl = make_planes(job.get("planes", []))
    return Job(make_camera(job["camera"]), make_fractal(job["fractal"]), pl, npl, make_march(job["march"]),
               make_frame(frame))


def make_object(ob):
    pl, npl = make_planes(ob.get("planes", []))
    rot = [float(x) for x in (ob.get("rotation") or (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0))]
    return Object(make_fractal(ob["fractal"]), pl, npl, (ctypes.c_float * 9)(*rot),
                  f3(*ob.get("translation", (0.0, 0.0, 0.0))), float(ob.get("scale", 1.0)))


# ------------------------------------------------------------------- render
def render_scene(scene, device="cuda", counters=False, out=None, workspace=None, trap=False):
    """Render a scene (camera, list of objects, march) in one launch; returns
    the frame dict with an extra "object_id" plane (int32, -1 on a miss) and,
    with trap=True, the orbit-trap planes "trap" [4, P]."""
    L = lib()
    dev = _device(device)
    objs = scene["objects"]
    fr = out if out is not None else alloc_frame(scene, dev, counters)
    if "object_id" not in fr:
        fr["object_id"] = torch.empty(fr["depth"].numel(), device=dev, dtype=torch.int32)
    if trap and "trap" not in fr:
        fr["trap"] = torch.empty(4, fr["depth"].numel(), device=dev, dtype=torch.float32)
    n = len(objs)
    arr = (Object * max(n, 1))(*[make_object(o) for o in objs])
    nbytes = int(L.frt_scene_workspace_bytes(max(n, 1)))
    if workspace is None:
        ws = torch.empty(nbytes + 256, device=dev, dtype=torch.uint8)
        off = (-ws.data_ptr()) % 256
        workspace = ws[off:off + nbytes]
    cam, mc = make_camera(scene["camera"]), make_march(scene["march"])
    _check(L.frt_render_scene(ctypes.byref(cam), arr, n, ctypes.byref(mc), make_frame(fr), _ptr(fr["object_id"]),
                              _ptr(fr.get("trap")), _ptr(workspace), workspace.numel(), _stream(dev)))
    return fr


def render(job, device="cuda", counters=False, out=None, workspace=None):
    """Render one job asynchronously on the current stream; returns the
    frame dict (depth, normal, colour, status[, counters])."""
    L = lib()
    dev = _device(device)
    fr = out if out is not None else alloc_frame(job, dev, counters)
    ws = workspace if workspace is not None else alloc_workspace(1, dev)
    pl, npl = make_planes(job.get("planes", []))
    cam, frac, mc = make_camera(job["camera"]), make_fractal(job["fractal"]), make_march(job["march"])
    _check(L.frt_render(ctypes.byref(cam), ctypes.byref(frac), pl, npl, ctypes.byref(mc), make_frame(fr),
                        _ptr(ws), ws.numel(), _stream(dev)))
    return fr


def render_batch(jobs, device="cuda", counters=False, use_graph=False, outs=None, workspace=None):
    """Render many jobs in one persistent launch; returns a list of frames."""
    L = lib()
    dev = _device(device)
    frames = outs if outs is not None else [alloc_frame(j, dev, counters) for j in jobs]
    ws = workspace if workspace is not None else alloc_workspace(len(jobs), dev)
    arr = (Job * len(jobs))(*[make_job(j, f) for j, f in zip(jobs, frames)])
    _check(L.frt_render_batch(arr, len(jobs), _ptr(ws), ws.numel(), int(bool(use_graph)), _stream(dev)))
    return frames


NOALLOC_MAX_JOBS = 256   # FRT_NOALLOC_MAX_JOBS


def render_batch_noalloc(jobs, outs, device="cuda"):
    """render_batch into caller-allocated frames through the entry point
    that allocates nothing (its workspace is the library's own device
    scratch; calls that overlap on one GPU race)."""
    L = lib()
    dev = _device(device)
    arr = (Job * len(jobs))(*[make_job(j, f) for j, f in zip(jobs, outs)])
    _check(L.frt_render_batch_noalloc(arr, len(jobs), _stream(dev)))
    return outs


def noalloc_scratch_bytes():
    return int(lib().frt_noalloc_scratch_bytes())


def render_backward(jobs, frames, g_colour=None, g_depth=None, g_normal=None, device="cuda", workspace=None,
                    grads=None, per_pixel=False):
    """Adjoint of render_batch(jobs): per-job gradients of
    sum(g_colour * colour) + sum(g_depth * depth) + sum(g_normal * normal)
    with respect to the fractal parameters and the raw cut planes.

    frames: the forward frames (depth and status are read); g_colour,
    g_depth, g_normal: lists with one tensor (or None) per job, or None.
    Returns (grad_c [n, 4], grad_power [n], grad_plane [n, 2, 4]) on the
    device, asynchronously on the current stream; with per_pixel=True also
    a list of per-pixel contributions [13, P] per job (slots as in grad:
    c0-c3, power, plane 0 n xyz d, plane 1 n xyz d)."""
    L = lib()
    dev = _device(device)
    n = len(jobs)
    ws = workspace if workspace is not None else alloc_workspace(n, dev)
    if grads is None:
        grads = (torch.empty(n, 4, device=dev, dtype=torch.float32), torch.empty(n, device=dev, dtype=torch.float32),
                 torch.empty(n, 2, 4, device=dev, dtype=torch.float32))
    keep = []

    def table(gs, channels):
        if gs is None:
            return None
        arr = (ctypes.c_void_p * n)()
        for k, (g, j) in enumerate(zip(gs, jobs)):
            if g is None:
                continue
            P = int(j["camera"]["width"]) * int(j["camera"]["height"])
            if g.numel() != channels * P or g.dtype != torch.float32 or g.device != dev:
                raise FrtError("gradient of job %d must be float32 with %d elements on %s" % (k, channels * P, dev))
            g = g.contiguous()
            keep.append(g)
            arr[k] = g.data_ptr()
        return arr

    tc, td, tn = table(g_colour, 3), table(g_depth, 1), table(g_normal, 3)
    pix, tp = None, None
    if per_pixel:
        pix = [torch.empty(13, int(j["camera"]["width"]) * int(j["camera"]["height"]), device=dev,
                           dtype=torch.float32) for j in jobs]
        tp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in pix])
    arr = (Job * n)(*[make_job(j, f) for j, f in zip(jobs, frames)])
    _check(L.frt_render_backward(arr, n, tc, td, tn, tp, _ptr(grads[0]), _ptr(grads[1]), _ptr(grads[2]), _ptr(ws),
                                 ws.numel(), _stream(dev)))
    return (grads + (pix,)) if per_pixel else grads


def distance(fractal, points, device="cuda"):
    """Distance estimate and escape count at points [n, 3] (a CUDA float32
    tensor, or anything torch.as_tensor accepts)."""
    dev = _device(device)
    pts = torch.as_tensor(points, dtype=torch.float32, device=dev).reshape(-1, 3).contiguous()
    n = pts.shape[0]
    d = torch.empty(n, device=dev, dtype=torch.float32)
    it = torch.empty(n, device=dev, dtype=torch.int32)
    frac = make_fractal(fractal)
    _check(lib().frt_distance(ctypes.byref(frac), _ptr(pts), n, _ptr(d), _ptr(it), _stream(dev)))
    return d, it


def normal_at(fractal, points, mode, eps=None, device="cuda"):
    """Unit normals [n, 3] at points [n, 3] by the renderer's rule for `mode`
    ("tetra", "central" with tap scale eps [n]; "analytic"); zero where the
    gradient vanishes."""
    dev = _device(device)
    pts = torch.as_tensor(points, dtype=torch.float32, device=dev).reshape(-1, 3).contiguous()
    n = pts.shape[0]
    m = NORMAL_MODES[mode] if isinstance(mode, str) else int(mode)
    ep = None if eps is None else torch.as_tensor(eps, dtype=torch.float32, device=dev).reshape(-1).contiguous()
    if ep is not None and ep.numel() != n:
        raise ValueError("eps must hold one value per point")
    out = torch.empty(n, 3, device=dev, dtype=torch.float32)
    frac = make_fractal(fractal)
    _check(lib().frt_normal_at(ctypes.byref(frac), m, _ptr(pts), _ptr(ep) if ep is not None else None, n, _ptr(out),
                               _stream(dev)))
    return out


MATH_FUNCS = {"acos": 0, "atan2": 1, "sin_rev": 2, "cos_rev": 3, "log2": 4, "exp2": 5, "rsq": 6, "rcp": 7}


def math_eval(func, x, y=None, device="cuda"):
    """The library's fast float32 function `func` (see MATH_FUNCS) on x (and y)."""
    dev = _device(device)
    xs = torch.as_tensor(x, dtype=torch.float32, device=dev).contiguous()
    ys = torch.as_tensor(y, dtype=torch.float32, device=dev).contiguous() if y is not None else None
    out = torch.empty_like(xs)
    _check(lib().frt_math_eval(MATH_FUNCS[func], _ptr(xs), _ptr(ys), _ptr(out), xs.numel(), _stream(dev)))
    return out


RATE_OPS = {"fma": 0, "exp2": 1, "log2": 2, "rsq": 3, "rcp": 4, "sqrt": 5, "sin_rev": 6, "fma4_exp2": 7,
            "fadd": 8, "fmul": 9, "int_shift_add": 10}


def valu_rate(op, iters, device="cuda"):
    """Sustained device-wide rate, in lane operations per second, of the FP32
    vector operation `op` (see RATE_OPS; an FMA counts once)."""
    dev = _device(device)
    r = ctypes.c_double(0.0)
    _check(lib().frt_valu_rate(RATE_OPS[op], int(iters), ctypes.byref(r), _stream(dev)))
    return r.value


def autotune_set(variant, block, chunk, waves_per_simd=0, orbit_lanes=8, rare_lanes=16):
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().frt_autotune_set(v, int(block), int(chunk), int(waves_per_simd), int(orbit_lanes),
                                  int(rare_lanes)))


def autotune_get(variant):
    """(block, chunk, waves_per_simd, orbit_lanes, rare_lanes) of a kernel variant."""
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    vals = [ctypes.c_int32() for _ in range(5)]
    _check(lib().frt_autotune_get(v, *[ctypes.byref(x) for x in vals]))
    return tuple(x.value for x in vals)


def set_stage_timing(enable):
    _check(lib().frt_set_stage_timing(int(bool(enable))))


def stage_times():
    """(primary march, normals, shadow march) durations in ms of the last call."""
    ms = (ctypes.c_float * 3)()
    _check(lib().frt_stage_times(ms))
    return tuple(float(x) for x in ms)


def graph_reset():
    _check(lib().frt_graph_reset())
