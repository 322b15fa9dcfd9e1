"""ctypes binding of the FP64 CPU oracle (frt_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg use this module; the GPU library never does.
It accepts the plain job dictionaries produced by ``workloads.py`` (float32
values) and widens every parameter to double.

The rounding probes ``normal_perturbed`` and ``orbit_trap_perturbed`` perturb
every orbit body on purpose and only decide where a comparison tolerates
rounding: parity unpinned.  Every other function is pinned by the tests.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_HERE = os.path.dirname(os.path.abspath(__file__))

c_double3 = ctypes.c_double * 3
c_double4 = ctypes.c_double * 4

STATUS_MISS_BOUNDS = 0
STATUS_MISS_TMAX = 1
STATUS_HIT = 2
STATUS_HIT_CUT = 3
STATUS_HIT_EXHAUSTED = 4
FLAG_SHADOWED = 8
FLAG_UNREFINED = 16
FLAG_JUMP = 32          # oracle only: the root bracket closed on a jump of the estimate
FLAG_REFLECT_HIT = 128  # scenes with the closest-hit shading: the reflection ray hit an object

NORMAL_MODES = {"tetra": 0, "central": 1, "analytic": 2}
SHADING_MODELS = {"lambert": 0, "phong": 1}

# Jacobian column slots (see oracle_pixel_jacobian)
SLOT_C = slice(0, 4)
SLOT_POWER = 4
SLOT_PLANE = (slice(5, 9), slice(9, 13))


class Camera(ctypes.Structure):
    _fields_ = [("eye", c_double3), ("target", c_double3), ("up", c_double3),
                ("fov_y_deg", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Fractal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c", c_double4), ("power", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("bailout2", ctypes.c_double),
                ("bound_radius", ctypes.c_double)]


class Plane(ctypes.Structure):
    _fields_ = [("n", c_double3), ("d", ctypes.c_double)]


class March(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("eps_abs", ctypes.c_double), ("eps_rel", ctypes.c_double),
                ("step_clamp", ctypes.c_double), ("t_max", ctypes.c_double),
                ("normal_mode", ctypes.c_int32), ("shadow", ctypes.c_int32),
                ("light", c_double3), ("albedo", c_double3),
                ("k_ambient", ctypes.c_double), ("k_diffuse", ctypes.c_double),
                ("shading", ctypes.c_int32), ("k_specular", ctypes.c_double), ("shininess", ctypes.c_double),
                ("k_reflect", ctypes.c_double)]


_lib = None


def lib():
    """Load liboracle.so, building it first when it is absent."""
    global _lib
    if _lib is None:
        # FRT_ORACLE_LIB selects another build of the same source (the
        # sanitised build of the CPU checks)
        path = os.environ.get("FRT_ORACLE_LIB") or build_oracle.LIB
        if not os.path.exists(path):
            build_oracle.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.oracle_quat_square.argtypes = [dp, dp]
        L.oracle_quat_mul.argtypes = [dp, dp, dp]
        L.oracle_quat_pow.argtypes = [dp, ctypes.c_int32, dp]
        L.oracle_bulb_power.argtypes = [dp, ctypes.c_double, dp]
        L.oracle_escape_iters.argtypes = [P(Fractal), dp, ctypes.c_int32]
        L.oracle_escape_iters.restype = ctypes.c_int32
        L.oracle_de.argtypes = [P(Fractal), dp, ctypes.c_int64, dp, P(ctypes.c_int32), dp, dp]
        L.oracle_bound_radius.argtypes = [P(Fractal)]
        L.oracle_bound_radius.restype = ctypes.c_double
        L.oracle_camera_ray.argtypes = [P(Camera), ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.oracle_render.argtypes = [P(Camera), P(Fractal), P(Plane), ctypes.c_int32, P(March),
                                    P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int32,
                                    dp, dp, dp, P(ctypes.c_uint8), P(ctypes.c_int32), P(ctypes.c_int32),
                                    P(ctypes.c_int64), P(ctypes.c_int64), dp]
        L.oracle_render.restype = ctypes.c_int
        L.oracle_pixel_jacobian.argtypes = [P(Camera), P(Fractal), P(Plane), ctypes.c_int32, P(March),
                                            P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int32,
                                            dp, P(ctypes.c_int32)]
        L.oracle_pixel_jacobian.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int32
        L.oracle_trace_rays.argtypes = [P(Fractal), P(Plane), ctypes.c_int32, P(March), dp, dp, dp, ctypes.c_int64,
                                        ctypes.c_int32, P(ctypes.c_uint8), dp, dp, P(ctypes.c_int32),
                                        P(ctypes.c_int32), dp, dp, P(ctypes.c_int32), P(ctypes.c_int64),
                                        P(ctypes.c_int64)]
        L.oracle_trace_rays.restype = ctypes.c_int
        L.oracle_occluded.argtypes = [P(Fractal), P(Plane), ctypes.c_int32, P(March), dp, dp, dp, ctypes.c_int64,
                                      P(ctypes.c_uint8)]
        L.oracle_occluded.restype = ctypes.c_int
        L.oracle_trap.argtypes = [P(Fractal), dp, ctypes.c_int64, dp]
        L.oracle_trap_perturbed.argtypes = [P(Fractal), dp, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, dp]
        L.oracle_bracket_crossings.argtypes = [P(Camera), P(Fractal), P(Plane), ctypes.c_int32, P(March),
                                               P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int32, dp, dp,
                                               P(ctypes.c_int32)]
        L.oracle_bracket_crossings.restype = ctypes.c_int
        L.oracle_escape_margin.argtypes = [P(Fractal), dp, ctypes.c_int64, dp, P(ctypes.c_int32)]
        L.oracle_normal_perturbed.argtypes = [P(Fractal), dp, dp, dp, ctypes.c_int64, ctypes.c_int32,
                                              ctypes.c_double, ctypes.c_uint64, dp]
        L.oracle_normal_at.argtypes = [P(Fractal), dp, dp, dp, ctypes.c_int64, ctypes.c_int32, dp]
        L.oracle_probe_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double]
        L.oracle_probe_noise.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_camera(cam):
    return Camera(c_double3(*cam["eye"]), c_double3(*cam["target"]), c_double3(*cam["up"]),
                  float(cam["fov_y_deg"]), int(cam["width"]), int(cam["height"]))


def make_fractal(fr):
    kind = {"julia": 0, "bulb": 1}[fr["kind"]]
    c = list(fr.get("c", (0.0, 0.0, 0.0, 0.0)))
    power = float(fr.get("power", 2.0 if kind == 0 else 8.0))
    if kind == 0 and (power != int(power) or not 2 <= power <= 16):
        raise ValueError("Julia degree must be an integer in [2, 16], got %r" % power)
    return Fractal(kind, c_double4(*c), power, int(fr["max_iter"]), float(fr["bailout2"]),
                   float(fr.get("bound_radius", 0.0)))


def make_planes(planes):
    arr = (Plane * 2)()
    for k, pl in enumerate(planes):
        arr[k] = Plane(c_double3(*pl["n"]), float(pl["d"]))
    return arr, len(planes)


def make_march(m):
    mode = NORMAL_MODES[m["normal_mode"]]
    return March(int(m["max_steps"]), float(m["eps_abs"]), float(m["eps_rel"]), float(m["step_clamp"]),
                 float(m["t_max"]), mode, int(bool(m["shadow"])), c_double3(*m["light_dir"]),
                 c_double3(*m["albedo"]), float(m["k_ambient"]), float(m["k_diffuse"]),
                 SHADING_MODELS[m.get("shading", "lambert")], float(m.get("k_specular", 0.0)),
                 float(m.get("shininess", 1.0)), float(m.get("k_reflect", 0.0)))


def max_threads():
    return int(lib().oracle_max_threads())


def render(job, pixels=None, threads=0):
    """Render a job (all pixels, or the listed linear indices j*W+i).

    Returns a dict of numpy arrays: depth [n], normal [3,n], colour [3,n],
    status [n] (uint8), steps [n], hit_iters [n], de_evals [n],
    orbit_bodies [n], raw_t [n].
    """
    if job["march"].get("shading", "lambert") != "lambert":
        raise ValueError("the closest-hit shading model is defined for scenes (render_scene)")
    L = lib()
    cam, fr, mc = make_camera(job["camera"]), make_fractal(job["fractal"]), make_march(job["march"])
    pl, npl = make_planes(job.get("planes", []))
    if pixels is None:
        n = int(cam.width) * int(cam.height)
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.size
    out = {
        "depth": np.empty(n), "normal": np.empty((3, n)), "colour": np.empty((3, n)),
        "status": np.empty(n, np.uint8), "steps": np.empty(n, np.int32), "hit_iters": np.empty(n, np.int32),
        "de_evals": np.empty(n, np.int64), "orbit_bodies": np.empty(n, np.int64), "raw_t": np.empty(n),
    }
    rc = L.oracle_render(ctypes.byref(cam), ctypes.byref(fr), pl, npl, ctypes.byref(mc),
                         _ptr(pix, ctypes.c_int64), n, int(threads),
                         _ptr(out["depth"], ctypes.c_double), _ptr(out["normal"], ctypes.c_double),
                         _ptr(out["colour"], ctypes.c_double), _ptr(out["status"], ctypes.c_uint8),
                         _ptr(out["steps"], ctypes.c_int32), _ptr(out["hit_iters"], ctypes.c_int32),
                         _ptr(out["de_evals"], ctypes.c_int64), _ptr(out["orbit_bodies"], ctypes.c_int64),
                         _ptr(out["raw_t"], ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle_render failed")
    return out


def pixel_jacobian(job, pixels, threads=0):
    """Per-pixel Jacobian [n, 7, 13] (rows depth, normal xyz, colour rgb;
    columns c0-c3, power, plane0 n xyz d, plane1 n xyz d) and the escape
    counts at the hit point and every normal tap [n, 7]."""
    L = lib()
    cam, fr, mc = make_camera(job["camera"]), make_fractal(job["fractal"]), make_march(job["march"])
    pl, npl = make_planes(job.get("planes", []))
    pix = np.ascontiguousarray(pixels, dtype=np.int64)
    n = pix.size
    jac = np.zeros((n, 7, 13))
    taps = np.zeros((n, 7), np.int32)
    rc = L.oracle_pixel_jacobian(ctypes.byref(cam), ctypes.byref(fr), pl, npl, ctypes.byref(mc),
                                 _ptr(pix, ctypes.c_int64), n, int(threads),
                                 _ptr(jac, ctypes.c_double), _ptr(taps, ctypes.c_int32))
    if rc == -2:
        raise NotImplementedError("the Jacobian of analytic normals needs second derivatives")
    if rc != 0:
        raise RuntimeError("oracle_pixel_jacobian failed")
    return jac, taps


def bracket_crossings(job, pixels, samples=256):
    """Final march bracket (lt, t) of listed pixels and the number of sign
    changes of d - eps over `samples` + 1 uniform points of it (-1, -1, 0
    where the ray did not end on a refinable surface hit)."""
    L = lib()
    cam, fr, mc = make_camera(job["camera"]), make_fractal(job["fractal"]), make_march(job["march"])
    pl, npl = make_planes(job.get("planes", []))
    pix = np.ascontiguousarray(pixels, dtype=np.int64)
    n = pix.size
    lt, t = np.empty(n), np.empty(n)
    cr = np.empty(n, np.int32)
    rc = L.oracle_bracket_crossings(ctypes.byref(cam), ctypes.byref(fr), pl, npl, ctypes.byref(mc),
                                    _ptr(pix, ctypes.c_int64), n, int(samples), _ptr(lt, ctypes.c_double),
                                    _ptr(t, ctypes.c_double), _ptr(cr, ctypes.c_int32))
    if rc != 0:
        raise RuntimeError("oracle_bracket_crossings failed")
    return lt, t, cr


def de(fractal, points):
    """Distance estimate at points [n,3]: (d, escape count, final |z|^2,
    running derivative: dz2 for Julia, dr for the Mandelbulb)."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    d, it, m2, dv = np.empty(n), np.empty(n, np.int32), np.empty(n), np.empty(n)
    L.oracle_de(ctypes.byref(fr), _ptr(pts, ctypes.c_double), n, _ptr(d, ctypes.c_double),
                _ptr(it, ctypes.c_int32), _ptr(m2, ctypes.c_double), _ptr(dv, ctypes.c_double))
    return d, it, m2, dv


def escape_iters(fractal, points, max_iter):
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(pts.shape[0], np.int32)
    L = lib()
    for i in range(pts.shape[0]):
        out[i] = L.oracle_escape_iters(ctypes.byref(fr), _ptr(pts[i], ctypes.c_double), int(max_iter))
    return out


def bound_radius(fractal):
    return float(lib().oracle_bound_radius(ctypes.byref(make_fractal(fractal))))


def quat_square(z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(4)
    lib().oracle_quat_square(_ptr(z, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def quat_mul(x, y):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty(4)
    lib().oracle_quat_mul(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def quat_pow(z, p):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(4)
    lib().oracle_quat_pow(_ptr(z, ctypes.c_double), int(p), _ptr(out, ctypes.c_double))
    return out


def bulb_power(w, n):
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty(3)
    lib().oracle_bulb_power(_ptr(w, ctypes.c_double), float(n), _ptr(out, ctypes.c_double))
    return out


def camera_rays(camera, pixels):
    """Origins and unit directions [n,3] for linear pixel indices."""
    L = lib()
    cam = make_camera(camera)
    pix = np.asarray(pixels, dtype=np.int64).ravel()
    o = np.empty((pix.size, 3))
    d = np.empty((pix.size, 3))
    for k, lin in enumerate(pix):
        oo, dd = np.empty(3), np.empty(3)
        L.oracle_camera_ray(ctypes.byref(cam), int(lin % cam.width), int(lin // cam.width),
                            _ptr(oo, ctypes.c_double), _ptr(dd, ctypes.c_double))
        o[k], d[k] = oo, dd
    return o, d


def normal_at(fractal, points, dirs, eps, mode):
    """Normal estimate (tetra or central taps) at points [n,3] with per-point eps."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    drs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    ep = np.ascontiguousarray(np.broadcast_to(eps, (pts.shape[0],)), dtype=np.float64)
    out = np.empty_like(pts)
    m = NORMAL_MODES[mode] if isinstance(mode, str) else int(mode)
    L.oracle_normal_at(ctypes.byref(fr), _ptr(pts, ctypes.c_double), _ptr(drs, ctypes.c_double),
                       _ptr(ep, ctypes.c_double), pts.shape[0], m, _ptr(out, ctypes.c_double))
    return out


def escape_margin(fractal, points):
    """Smallest relative distance of |z_k|^2 to the bailout over the orbit at
    each point [n,3], and whether the orbit escaped."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    m = np.empty(pts.shape[0])
    e = np.empty(pts.shape[0], np.int32)
    L.oracle_escape_margin(ctypes.byref(fr), _ptr(pts, ctypes.c_double), pts.shape[0], _ptr(m, ctypes.c_double),
                           _ptr(e, ctypes.c_int32))
    return m, e.astype(bool)


TETRA_TAPS = np.array([[1, -1, -1], [-1, -1, 1], [-1, 1, -1], [1, 1, 1]], dtype=np.float64)
CENTRAL_TAPS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)


def tap_points(points, eps, mode):
    """Normal-tap positions [n, taps, 3] around points [n,3] for per-point eps."""
    m = NORMAL_MODES[mode] if isinstance(mode, str) else int(mode)
    if m == 2:      # the analytic normal evaluates the estimate at the point itself
        return np.array(points, dtype=np.float64)[:, None, :]
    taps, h = (TETRA_TAPS, 0.5773 * np.asarray(eps)) if m == 0 else (CENTRAL_TAPS, np.asarray(eps))
    return np.asarray(points)[:, None, :] + np.asarray(h).reshape(-1, 1, 1) * taps[None]


def normal_perturbed(fractal, points, dirs, eps, mode, rel, seed):
    """Normal at points with every orbit body perturbed by a relative
    uniform(-rel, rel) factor per component (seeded): a rounding probe."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    drs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    ep = np.ascontiguousarray(np.broadcast_to(eps, (pts.shape[0],)), dtype=np.float64)
    out = np.empty_like(pts)
    m = NORMAL_MODES[mode] if isinstance(mode, str) else int(mode)
    L.oracle_normal_perturbed(ctypes.byref(fr), _ptr(pts, ctypes.c_double), _ptr(drs, ctypes.c_double),
                              _ptr(ep, ctypes.c_double), pts.shape[0], m, float(rel), int(seed),
                              _ptr(out, ctypes.c_double))
    return out


# ---------------------------------------------------------------- scenes
def trace_rays(fractal, planes, march, origins, dirs, samples=0, eps0=None):
    """Primary part (march, refinement, normal; no shading) of explicit rays
    in the fractal's own frame and units; eps0 [n] optionally sets each
    ray's eps_abs (and start).  Returns status, depth, normal
    [n, 3], steps, hit_iters, raw_t, lt (last-but-one sample), crossings
    (sign changes of d - eps over the final bracket, if samples > 0)."""
    L = lib()
    fr, mc = make_fractal(fractal), make_march(march)
    pl, npl = make_planes(planes)
    o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    e0 = None if eps0 is None else np.ascontiguousarray(np.broadcast_to(eps0, (n,)), dtype=np.float64)
    out = {"status": np.empty(n, np.uint8), "depth": np.empty(n), "normal": np.empty((n, 3)),
           "steps": np.empty(n, np.int32), "hit_iters": np.empty(n, np.int32), "raw_t": np.empty(n),
           "lt": np.empty(n), "crossings": np.zeros(n, np.int32), "de_evals": np.empty(n, np.int64),
           "orbit_bodies": np.empty(n, np.int64)}
    rc = L.oracle_trace_rays(ctypes.byref(fr), pl, npl, ctypes.byref(mc), _ptr(o, ctypes.c_double),
                             _ptr(d, ctypes.c_double), _ptr(e0, ctypes.c_double), n, int(samples),
                             _ptr(out["status"], ctypes.c_uint8),
                             _ptr(out["depth"], ctypes.c_double), _ptr(out["normal"], ctypes.c_double),
                             _ptr(out["steps"], ctypes.c_int32), _ptr(out["hit_iters"], ctypes.c_int32),
                             _ptr(out["raw_t"], ctypes.c_double), _ptr(out["lt"], ctypes.c_double),
                             _ptr(out["crossings"], ctypes.c_int32), _ptr(out["de_evals"], ctypes.c_int64),
                             _ptr(out["orbit_bodies"], ctypes.c_int64))
    if rc != 0:
        raise RuntimeError("oracle_trace_rays failed")
    return out


def occluded(fractal, planes, march, q, light, eps):
    """Shadow test of explicit rays in the fractal's frame: bool [n]."""
    L = lib()
    fr, mc = make_fractal(fractal), make_march(march)
    pl, npl = make_planes(planes)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    lt = np.ascontiguousarray(light, dtype=np.float64).reshape(-1, 3)
    ep = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1)
    hit = np.zeros(q.shape[0], np.uint8)
    rc = L.oracle_occluded(ctypes.byref(fr), pl, npl, ctypes.byref(mc), _ptr(q, ctypes.c_double),
                           _ptr(lt, ctypes.c_double), _ptr(ep, ctypes.c_double), q.shape[0],
                           _ptr(hit, ctypes.c_uint8))
    if rc != 0:
        raise RuntimeError("oracle_occluded failed")
    return hit.astype(bool)


def object_frame(ob):
    """(R, T, s) of a scene object: x_obj = R^T (x - T) / s."""
    R = np.array(ob.get("rotation") or (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0), dtype=np.float64).reshape(3, 3)
    T = np.array(ob.get("translation", (0.0, 0.0, 0.0)), dtype=np.float64)
    return R, T, float(ob.get("scale", 1.0))


def object_march(march, s):
    """The march settings in an object's units: eps_abs, step_clamp and
    t_max divided by its scale (eps_rel and the rest unchanged)."""
    m = dict(march)
    m["eps_abs"] = float(march["eps_abs"]) / s
    m["step_clamp"] = float(march["step_clamp"]) / s
    m["t_max"] = float(march["t_max"]) / s
    return m


def render_scene(scene, pixels=None, samples=0):
    """A scene of several fractal objects (Sec. 3): every primary ray is
    traced through each object in its own frame and the closest hit kept
    (ties to the lower index); the hit is shaded in world space and its
    shadow ray is blocked by a hit on any object.  Returns the render() dict
    plus object_id (-1 on a miss), lt and crossings of the object hit."""
    cam, mc = scene["camera"], scene["march"]
    W, H = int(cam["width"]), int(cam["height"])
    pix = np.arange(W * H) if pixels is None else np.asarray(pixels, np.int64)
    o, d = camera_rays(cam, pix)
    n = pix.size
    best = np.full(n, -1, np.int64)
    best_t = np.full(n, np.inf)
    entered = np.zeros(n, bool)
    status = np.zeros(n, np.uint8)
    nrm = np.zeros((n, 3))
    keep = {k: np.zeros(n, dt) for k, dt in (("steps", np.int32), ("hit_iters", np.int32), ("raw_t", np.float64),
                                               ("lt", np.float64), ("crossings", np.int32),
                                               ("de_evals", np.int64), ("orbit_bodies", np.int64))}
    for k, ob in enumerate(scene["objects"]):
        R, T, s = object_frame(ob)
        r = trace_rays(ob["fractal"], ob.get("planes", []), object_march(mc, s), (o - T) @ R / s, d @ R, samples)
        cls = r["status"] & 7
        entered |= cls != STATUS_MISS_BOUNDS
        tw = r["depth"] * s
        better = (cls >= STATUS_HIT) & (tw < best_t)
        best[better] = k
        best_t[better] = tw[better]
        status[better] = r["status"][better]
        nrm[better] = r["normal"][better] @ R.T
        for key in ("steps", "hit_iters", "crossings", "de_evals", "orbit_bodies"):
            keep[key][better] = r[key][better]
        keep["raw_t"][better] = r["raw_t"][better] * s
        keep["lt"][better] = np.where(r["lt"][better] >= 0.0, r["lt"][better] * s, -1.0)
    hit = best >= 0
    nl = np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm = np.where(nl > 0, nrm / np.where(nl > 0, nl, 1.0), nrm)
    status[~hit] = np.where(entered[~hit], STATUS_MISS_TMAX, STATUS_MISS_BOUNDS)
    depth = np.where(hit, best_t, -1.0)
    Ld = np.array(mc["light_dir"], dtype=np.float64)
    Ld /= np.linalg.norm(Ld)
    ndl = nrm @ Ld
    vis = np.ones(n)
    if mc["shadow"]:
        lit = np.nonzero(hit & (ndl > 0.0))[0]
        eps_s = mc["eps_abs"] + mc["eps_rel"] * depth[lit]
        q = o[lit] + depth[lit, None] * d[lit] + 4.0 * eps_s[:, None] * nrm[lit]
        shadowed = np.zeros(lit.size, bool)
        for ob in scene["objects"]:
            R, T, s = object_frame(ob)
            todo = ~shadowed
            if not todo.any():
                break
            idx = np.nonzero(todo)[0]
            hit_k = occluded(ob["fractal"], ob.get("planes", []), object_march(mc, s), (q[idx] - T) @ R / s,
                             np.broadcast_to(Ld @ R, (idx.size, 3)), eps_s[idx] / s)
            shadowed[idx[hit_k]] = True
        vis[lit[shadowed]] = 0.0
        status[lit[shadowed]] |= FLAG_SHADOWED
    h = np.nonzero(hit)[0]
    colour = np.zeros((3, n))
    trap = np.zeros((4, n))
    colour[:, h], trap[:, h], rhit = shade_hits(scene, best[h], o[h] + depth[h, None] * d[h], d[h], nrm[h],
                                                vis[h], mc["eps_abs"] + mc["eps_rel"] * depth[h])
    status[h[rhit]] |= FLAG_REFLECT_HIT
    colour = np.where(hit[None, :], colour, 0.0)
    out = {"depth": depth, "normal": np.where(hit[None, :], nrm.T, 0.0), "colour": colour, "status": status,
           "object_id": best, "trap": trap}
    out.update(keep)
    return out


def shade_hits(scene, object_ids, points, dirs, normals, vis, eps_s):
    """Colour of scene hits (R11, R23, R24): object index [n], world hit
    points [n, 3], unit ray directions [n, 3], unit normals [n, 3],
    shadow-ray visibility [n] (0 or 1) and eps(t*) [n].  The albedo follows
    the orbit trap of the hit point in its object's frame when a palette is
    given (closest-hit shading only); Lambert's term, then with the
    closest-hit shading the white highlight (shadowed with the diffuse term)
    and the reflection bounce.  Returns colour [3, n], the traps [4, n] and
    the reflected-hit flags [n] (all False under Lambert shading)."""
    mc = scene["march"]
    n = np.asarray(object_ids).size
    pts = np.asarray(points, np.float64).reshape(n, 3)
    d = np.asarray(dirs, np.float64).reshape(n, 3)
    nrm = np.asarray(normals, np.float64).reshape(n, 3)
    vis = np.asarray(vis, np.float64)
    trap = np.zeros((4, n))
    for k, ob in enumerate(scene["objects"]):
        m = np.nonzero(np.asarray(object_ids) == k)[0]
        if m.size:
            R, T, s = object_frame(ob)
            trap[:, m] = orbit_trap(ob["fractal"], (pts[m] - T) @ R / s).T
    Ld = np.array(mc["light_dir"], dtype=np.float64)
    Ld /= np.linalg.norm(Ld)
    ndl = nrm @ Ld
    phong = mc.get("shading", "lambert") == "phong"
    albedo = np.array(mc["albedo"], dtype=np.float64)
    pal = np.array(mc.get("trap_colour", [[0.0] * 3] * 4), dtype=np.float64) if phong else np.zeros((4, 3))
    alb = trap_albedo(albedo, pal, trap)                           # [3, n]
    colour = alb * (mc["k_ambient"] + mc["k_diffuse"] * np.maximum(0.0, ndl) * vis)[None, :]
    rhit = np.zeros(n, bool)
    if phong:
        # R23: white Phong highlight (shadowed with the diffuse term), then one
        # reflection bounce weighted by Schlick's Fresnel term with f0 = albedo
        colour = colour + float(mc["k_specular"]) * _phong_spec(nrm, Ld, -d, ndl, float(mc["shininess"]))[None, :] * vis
        term, rhit = reflection_term(scene, pts, d, nrm, eps_s, alb)
        colour = colour + term
    return colour, trap, rhit


def reflection_term(scene, points, dirs, normals, eps_s, albedo):
    """The reflection bounce of the closest-hit shading (R23) for hits at
    world points [n, 3] seen along unit dirs [n, 3], with unit normals
    [n, 3], thresholds eps(t*) [n] and albedos [3, n]: the ray leaves
    p* + 4 eps N along dir - 2 (dir . N) N against every object (threshold
    eps(t*) + eps_rel s at distance s), and its first hit is shaded with
    Lambert and the highlight (no shadow ray, 0 on a miss), weighted by
    k_r and Schlick's F = albedo + (1 - albedo)(1 - max(0, -dir . N))^5.
    Returns the term [3, n] and the reflected hit flags [n]."""
    mc = scene["march"]
    Ld = np.array(mc["light_dir"], dtype=np.float64)
    Ld /= np.linalg.norm(Ld)
    albedo0 = np.array(mc["albedo"], dtype=np.float64)
    pal = np.array(mc.get("trap_colour", [[0.0] * 3] * 4), dtype=np.float64)
    d = np.asarray(dirs, np.float64)
    nrm = np.asarray(normals, np.float64)
    n = d.shape[0]
    dn = np.einsum("ij,ij->i", d, nrm)
    rd = d - 2.0 * dn[:, None] * nrm
    q = np.asarray(points, np.float64) + 4.0 * np.asarray(eps_s, np.float64)[:, None] * nrm
    rt = np.full(n, np.inf)
    rn = np.zeros((n, 3))
    rtrap = np.zeros((4, n))
    for ob in scene["objects"]:
        R, T, s = object_frame(ob)
        qo, rdo = (q - T) @ R / s, rd @ R
        r = trace_rays(ob["fractal"], ob.get("planes", []), object_march(mc, s), qo, rdo, eps0=eps_s / s)
        tw = r["depth"] * s
        better = ((r["status"] & 7) >= STATUS_HIT) & (tw < rt)
        rt[better] = tw[better]
        rn[better] = r["normal"][better] @ R.T
        if better.any():
            bi = np.nonzero(better)[0]
            rtrap[:, bi] = orbit_trap(ob["fractal"], qo[bi] + r["depth"][bi, None] * rdo[bi]).T
    rhit = np.isfinite(rt)
    rl = np.linalg.norm(rn, axis=1, keepdims=True)
    rn = np.where(rl > 0, rn / np.where(rl > 0, rl, 1.0), rn)
    rndl = rn @ Ld
    ralb = trap_albedo(albedo0, pal, rtrap)
    c_r = ralb * (mc["k_ambient"] + mc["k_diffuse"] * np.maximum(0.0, rndl))[None, :]
    c_r = c_r + float(mc["k_specular"]) * _phong_spec(rn, Ld, -rd, rndl, float(mc["shininess"]))[None, :]
    c_r = np.where(rhit[None, :], c_r, 0.0)
    cos_i = np.maximum(0.0, -dn)
    ah = np.asarray(albedo, np.float64)
    F = ah + (1.0 - ah) * ((1.0 - cos_i) ** 5)[None, :]
    return float(mc["k_reflect"]) * F * c_r, rhit


def trap_albedo(albedo, palette, trap):
    """Albedo of hits [3, n] coloured by their orbit traps [4, n] (R24): per
    channel albedo_c + sum_k palette[k][c] T_k, clamped to [0, 1]."""
    return np.clip(np.asarray(albedo, np.float64)[:, None] + np.asarray(palette, np.float64).T @ trap, 0.0, 1.0)


def _phong_spec(nrm, L, V, ndl, shininess):
    """max(0, R.V)^shininess with R = 2 (N.L) N - L the mirrored light
    direction, zero where the light is behind the surface."""
    Rl = 2.0 * ndl[:, None] * nrm - L[None, :]
    return np.where(ndl > 0.0, np.maximum(0.0, np.einsum("ij,ij->i", Rl, V)) ** shininess, 0.0)


def shade_lambert(march, normals, shadowed):
    """Lambert colour (R11) of hits with the given unit normals [n, 3] and
    shadow outcomes [n] (bool): albedo (k_a + k_d max(0, N.L) V), as the
    render computes it, for shading a normal evaluated at another point.
    Returns [3, n]."""
    L = np.array(march["light_dir"], dtype=np.float64)
    L /= np.linalg.norm(L)
    ndl = np.asarray(normals, np.float64) @ L
    vis = np.where(np.asarray(shadowed, bool), 0.0, 1.0)
    lam = march["k_ambient"] + march["k_diffuse"] * np.maximum(0.0, ndl) * vis
    return np.array(march["albedo"], dtype=np.float64)[:, None] * lam[None, :]


def probe_noise(seed, point, body, comp, rel):
    """The rounding probes' multiplicative factor for one (seed, point, body,
    component): uniform on [1 - rel, 1 + rel]."""
    return lib().oracle_probe_noise(int(seed), int(point), int(body), int(comp), float(rel))


def orbit_trap_perturbed(fractal, points, rel, seed):
    """The orbit trap with every power perturbed by a relative
    uniform(-rel, rel) factor per component (seeded): a rounding probe."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty((pts.shape[0], 4))
    L.oracle_trap_perturbed(ctypes.byref(fr), _ptr(pts, ctypes.c_double), pts.shape[0], float(rel), int(seed),
                            _ptr(out, ctypes.c_double))
    return out


def orbit_trap(fractal, points):
    """Orbit trap at points [n, 3] (R24): [n, 4] minima over the orbit of
    |x|, |y|, |z| and the squared norm."""
    L = lib()
    fr = make_fractal(fractal)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty((pts.shape[0], 4))
    L.oracle_trap(ctypes.byref(fr), _ptr(pts, ctypes.c_double), pts.shape[0], _ptr(out, ctypes.c_double))
    return out
