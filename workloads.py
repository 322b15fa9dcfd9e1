"""Seeded synthetic workloads for the fractal sphere tracer.

This module holds input generation only -- camera placement, fractal
parameters, cut planes and march settings -- and none of the rendering
arithmetic.  Every float is rounded to float32 when it is drawn, so the GPU
library and the FP64 oracle read bit-identical parameter values.

The paper (arXiv 2102.01747) renders interactive scenes and publishes no
workload sizes, so the sizes below are the benchmark definitions this project
measures on: a quaternion Julia view at 256x256, an eight-view 1080p
Mandelbulb, a 64-job batch of uneven Julia renders, a 16-render
differentiable set and a 4K power sweep.  Seeds use numpy's PCG64
(``numpy.random.default_rng``) and the draw order is the order written here.
"""
import math

import numpy as np


def f32(x):
    return float(np.float32(x))


def f32v(v):
    return [f32(x) for x in v]


_S3 = 1.0 / math.sqrt(3.0)
LIGHT_DIR = f32v([_S3, _S3, _S3])          # normalize(1, 1, 1)
ALBEDO = [1.0, 1.0, 1.0]
K_AMBIENT = f32(0.1)
K_DIFFUSE = f32(0.9)
JULIA_C1 = f32v([-0.2, 0.6, 0.2, 0.2])     # quaternion constant of the Julia view
JULIA_C3 = f32v([-0.45, 0.1, 0.4, 0.2])   # constant of the cubic (degree-3) Julia views


def camera(eye, width, height, fov_y_deg=45.0, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    return {"eye": f32v(eye), "target": f32v(target), "up": f32v(up), "fov_y_deg": f32(fov_y_deg),
            "width": int(width), "height": int(height)}


def orbit_eye(radius, azimuth, elevation):
    """Eye on a sphere around the origin: R (cos e sin a, sin e, cos e cos a)."""
    return [radius * math.cos(elevation) * math.sin(azimuth), radius * math.sin(elevation),
            radius * math.cos(elevation) * math.cos(azimuth)]


def march(max_steps, eps_abs=0.0, eps_rel=0.0, normal_mode="tetra", shadow=False, step_clamp=0.2,
          t_max=7000.0, refine_iters=12, shading="lambert", k_specular=0.0, shininess=1.0, k_reflect=0.0):
    return {"max_steps": int(max_steps), "eps_abs": f32(eps_abs), "eps_rel": f32(eps_rel),
            "step_clamp": f32(step_clamp), "t_max": f32(t_max), "normal_mode": normal_mode,
            "refine_iters": int(refine_iters), "shadow": bool(shadow), "light_dir": list(LIGHT_DIR),
            "albedo": list(ALBEDO), "k_ambient": K_AMBIENT, "k_diffuse": K_DIFFUSE, "shading": shading,
            "k_specular": f32(k_specular), "shininess": f32(shininess), "k_reflect": f32(k_reflect)}


# The closest-hit shading of the paper's shaders (Phong highlight, one
# reflection bounce with Schlick's Fresnel term; reflection weight 0.1 as in
# the Julia closest-hit listing), with a coloured albedo so that the Fresnel
# term's f0 differs per channel.
PHONG = {"shading": "phong", "k_specular": 0.5, "shininess": 40.0, "k_reflect": 0.1}
PHONG_ALBEDO = f32v([0.9, 0.6, 0.3])
# Orbit-trap colouring of the closest-hit shading (the colour parameters of
# the Mandelbulb distance listing, read by the shader): per unit of the trap
# components (min |x|, min |y|, min |z|, min |w|^2) the change of the albedo
# (r, g, b); the builder's palette, since the paper's colouring is not given.
TRAP_COLOUR = [f32v([-0.6, 0.2, 0.5]), f32v([0.3, -0.5, 0.2]), f32v([0.2, 0.3, -0.6]), f32v([-0.2, -0.2, -0.1])]


def phong(mc, trap_colour=False):
    """A march dict switched to the closest-hit shading (with the orbit-trap
    palette when trap_colour is set)."""
    out = dict(mc)
    out.update({k: (f32(v) if isinstance(v, float) else v) for k, v in PHONG.items()})
    out["albedo"] = list(PHONG_ALBEDO)
    if trap_colour:
        out["trap_colour"] = [list(r) for r in TRAP_COLOUR]
    return out


def job_scene(jb):
    """A single render as a one-object scene with the identity placement."""
    return scene(jb["camera"], [scene_object(jb["fractal"], jb.get("planes", ()))], jb["march"])


def julia(c, max_iter, bailout2=256.0, bound_radius=0.0, degree=2):
    """Quaternion Julia z^p + c; `degree` is the integer p (stored as power)."""
    return {"kind": "julia", "c": f32v(c), "power": float(int(degree)), "max_iter": int(max_iter),
            "bailout2": f32(bailout2), "bound_radius": f32(bound_radius)}


def bulb(power, max_iter, bailout2=4.0, bound_radius=0.0):
    return {"kind": "bulb", "c": [0.0, 0.0, 0.0, 0.0], "power": f32(power), "max_iter": int(max_iter),
            "bailout2": f32(bailout2), "bound_radius": f32(bound_radius)}


def plane(n, d):
    return {"n": f32v(n), "d": f32(d)}


def job(cam, frac, mc, planes=()):
    return {"camera": cam, "fractal": frac, "planes": [dict(p) for p in planes], "march": mc}


# ---------------------------------------------------------------------------
# Julia view: c = (-0.2, 0.6, 0.2, 0.2), slice w=0, 256x256, eye (0,0,3),
# 45 deg, 11 orbit iterations, |z|^2 > 256, 256 steps, eps 1e-3, tetrahedral
# normals, Lambert shading.
# ---------------------------------------------------------------------------
def julia_view(c=JULIA_C1, width=256, height=256, max_iter=11, max_steps=256, eps_abs=1e-3, planes=(),
               eye=(0.0, 0.0, 3.0), shadow=False, normal_mode="tetra", degree=2):
    return job(camera(eye, width, height), julia(c, max_iter, degree=degree),
               march(max_steps, eps_abs=eps_abs, normal_mode=normal_mode, shadow=shadow), planes)


# ---------------------------------------------------------------------------
# Mandelbulb p^8 + c, 1920x1080, eye orbiting at radius 2.5 at 8 seeded
# angles (seed 2; per view: azimuth U[0, 2pi), elevation U[-pi/6, pi/6]),
# 10 orbit iterations, r > 2, 512 steps, eps = 5e-4 t, central normals, one
# shadow ray per lit hit.
# ---------------------------------------------------------------------------
def bulb_view(azimuth, elevation, width=1920, height=1080, power=8.0, max_iter=10, max_steps=512,
              eps_rel=5e-4, shadow=True, planes=(), radius=2.5, normal_mode="central"):
    return job(camera(orbit_eye(radius, azimuth, elevation), width, height), bulb(power, max_iter),
               march(max_steps, eps_rel=eps_rel, normal_mode=normal_mode, shadow=shadow), planes)


def bulb_views(seed=2, n_views=8, width=1920, height=1080, **kw):
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_views):
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = rng.uniform(-math.pi / 6.0, math.pi / 6.0)
        jobs.append(bulb_view(az, el, width=width, height=height, **kw))
    return jobs


# ---------------------------------------------------------------------------
# Batch of 64 quaternion Julia renders (seed 3; per job in this order):
# c ~ U[-0.8, 0.8]^4; cut plane through the origin with normal
# normalize(N(0, I3)); W and H drawn independently from {128,256,512,1024};
# iterations uniform in 8..24; eps_abs ~ U[1e-4, 1e-3].  Camera and step
# budget as in the Julia view.
# ---------------------------------------------------------------------------
def julia_batch(seed=3, n_jobs=64, sizes=(128, 256, 512, 1024), max_steps=256):
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_jobs):
        c = rng.uniform(-0.8, 0.8, size=4)
        nrm = rng.normal(size=3)
        nrm = nrm / np.linalg.norm(nrm)
        w = int(rng.choice(sizes))
        h = int(rng.choice(sizes))
        iters = int(rng.integers(8, 25))
        eps = rng.uniform(1e-4, 1e-3)
        jobs.append(julia_view(c=c, width=w, height=h, max_iter=iters, max_steps=max_steps, eps_abs=eps,
                               planes=[plane(nrm, 0.0)]))
    return jobs


# ---------------------------------------------------------------------------
# Batch of 32 quaternion Julia renders of higher degree (seed 6; per job in
# this order): degree p uniform in {3, 4, 5, 6}; c ~ U[-0.8, 0.8]^4; cut
# plane through the origin with normal normalize(N(0, I3)); W and H drawn
# independently from {256, 512, 1024}; iterations uniform in 8..16;
# eps_abs ~ U[1e-4, 1e-3].  Camera and step budget as in the Julia view.
# ---------------------------------------------------------------------------
def julia_degree_batch(seed=6, n_jobs=32, degrees=(3, 4, 5, 6), sizes=(256, 512, 1024), max_steps=256):
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_jobs):
        p = int(rng.choice(degrees))
        c = rng.uniform(-0.8, 0.8, size=4)
        nrm = rng.normal(size=3)
        nrm = nrm / np.linalg.norm(nrm)
        w = int(rng.choice(sizes))
        h = int(rng.choice(sizes))
        iters = int(rng.integers(8, 17))
        eps = rng.uniform(1e-4, 1e-3)
        jobs.append(julia_view(c=c, width=w, height=h, max_iter=iters, max_steps=max_steps, eps_abs=eps,
                               planes=[plane(nrm, 0.0)], degree=p))
    return jobs


# ---------------------------------------------------------------------------
# Differentiable set (seed 4): 8 Julia renders (c0 = Julia-view c +
# N(0, 0.05^2)^4, Julia-view camera, seeded plane through the origin) and 8
# Mandelbulb renders (n = 8, seeded orbit camera, seeded plane through the
# origin), all 512x512.  Targets: c* = c0 + U[-0.02, 0.02]^4,
# n* = 8 + U[-0.1, 0.1], plane normal* = normal + N(0, 0.02^2)^3.
# ---------------------------------------------------------------------------
def diff_set(seed=4, n_julia=8, n_bulb=8, width=512, height=512):
    rng = np.random.default_rng(seed)
    jobs, targets = [], []
    for _ in range(n_julia):
        c0 = np.array(JULIA_C1) + rng.normal(0.0, 0.05, size=4)
        nrm = rng.normal(size=3)
        nrm = nrm / np.linalg.norm(nrm)
        ct = c0 + rng.uniform(-0.02, 0.02, size=4)
        nt = nrm + rng.normal(0.0, 0.02, size=3)
        jobs.append(julia_view(c=c0, width=width, height=height, planes=[plane(nrm, 0.0)]))
        targets.append(julia_view(c=ct, width=width, height=height, planes=[plane(nt, 0.0)]))
    for _ in range(n_bulb):
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = rng.uniform(-math.pi / 6.0, math.pi / 6.0)
        nrm = rng.normal(size=3)
        nrm = nrm / np.linalg.norm(nrm)
        n_t = 8.0 + rng.uniform(-0.1, 0.1)
        nt = nrm + rng.normal(0.0, 0.02, size=3)
        jobs.append(bulb_view(az, el, width=width, height=height, shadow=False, planes=[plane(nrm, 0.0)]))
        targets.append(bulb_view(az, el, width=width, height=height, power=n_t, shadow=False,
                                 planes=[plane(nt, 0.0)]))
    return jobs, targets


# ---------------------------------------------------------------------------
# Stress sweep: frame f of 64 has n = 2 + 14 f / 63, 3840x2160, eye at radius
# 2.5, azimuth 2 pi f / 64, elevation 0.3 rad, 15 orbit iterations, 1024
# steps, eps = 2e-4 t, cut plane z <= 0.1, central normals, no shadow.
# ---------------------------------------------------------------------------
def stress_frame(f, n_frames=64, width=3840, height=2160):
    n = 2.0 + 14.0 * f / 63.0
    return bulb_view(2.0 * math.pi * f / n_frames, 0.3, width=width, height=height, power=n, max_iter=15,
                     max_steps=1024, eps_rel=2e-4, shadow=False, planes=[plane((0.0, 0.0, 1.0), 0.1)])


def stress_sweep(n_frames=64, width=3840, height=2160):
    return [stress_frame(f, n_frames, width, height) for f in range(n_frames)]


def with_size(jb, width, height):
    """Copy of a job at another resolution (same camera pose and parameters)."""
    out = {k: (dict(v) if isinstance(v, dict) else [dict(p) for p in v]) for k, v in jb.items()}
    out["camera"]["width"] = int(width)
    out["camera"]["height"] = int(height)
    return out


# ---------------------------------------------------------------------------
# Iteration-count animation (Fig. 2 animates the n = 8 Mandelbulb by the
# number of orbit iterations): frame k of n_frames uses max_iter = k + 1,
# everything else as one Mandelbulb view (azimuth 0.7, elevation 0.25).
# ---------------------------------------------------------------------------
def iteration_animation(n_frames=10, width=480, height=270, shadow=True):
    return [bulb_view(0.7, 0.25, width=width, height=height, max_iter=k + 1, shadow=shadow)
            for k in range(n_frames)]


# ---------------------------------------------------------------------------
# Scenes of several procedural objects (Sec. 3, Fig. 4), each placed by a
# rotation R (object to world), a translation T and a uniform scale s.
# ---------------------------------------------------------------------------
def rotation(axis, angle):
    """Rotation by `angle` radians about a unit `axis`, row-major, float32."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    R = np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)
    return f32v(R.ravel())


def scene_object(fractal, planes=(), rot=None, translation=(0.0, 0.0, 0.0), scale=1.0):
    return {"fractal": fractal, "planes": [dict(p) for p in planes],
            "rotation": list(rot) if rot is not None else f32v(np.eye(3).ravel()),
            "translation": f32v(translation), "scale": f32(scale)}


def scene(cam, objects, mc):
    return {"camera": cam, "objects": objects, "march": mc}


# Julia (the Julia view's c, cut plane) and n = 8 Mandelbulb side by side,
# each rotated and scaled, eye (0, 1, 4.5), 45 deg, eps = 5e-4 t, central
# normals, shadow rays.
def julia_bulb_scene(width=320, height=200, shadow=True, normal_mode="central", max_steps=512):
    objs = [scene_object(julia(JULIA_C1, 11), planes=[plane([0.3, 0.2, 1.0], 0.05)],
                         rot=rotation([0.0, 1.0, 0.0], 0.6), translation=(-1.35, 0.0, 0.0), scale=0.9),
            scene_object(bulb(8.0, 10), rot=rotation([1.0, 0.0, 0.2], 0.4), translation=(1.3, 0.1, -0.3),
                         scale=1.1)]
    return scene(camera((0.0, 1.0, 4.5), width, height),
                 objs, march(max_steps, eps_rel=5e-4, normal_mode=normal_mode, shadow=shadow, t_max=20.0))


# Three objects that overlap on screen and in depth and shadow one another:
# a small cubic Julia in front, a real-power (n = 6.37) Mandelbulb behind it
# and a large degree-2 Julia further back, lit from the upper front.
def overlap_scene(width=256, height=192, shadow=True, normal_mode="tetra", max_steps=512):
    objs = [scene_object(julia(JULIA_C3, 9, degree=3), rot=rotation([0.3, 1.0, 0.0], 1.1),
                         translation=(0.35, 0.3, 1.2), scale=0.45),
            scene_object(bulb(6.37, 10), rot=rotation([0.0, 0.0, 1.0], 0.3), translation=(-0.2, 0.0, 0.0),
                         scale=0.9),
            scene_object(julia([-0.5, 0.3, 0.1, 0.0], 11), planes=[plane([0.0, 0.0, 1.0], 0.2)],
                         rot=rotation([1.0, 0.0, 0.0], -0.5), translation=(0.3, -0.4, -2.0), scale=1.6)]
    return scene(camera((0.0, 0.4, 4.0), width, height),
                 objs, march(max_steps, eps_rel=5e-4, normal_mode=normal_mode, shadow=shadow, t_max=20.0))


def stratified_pixels(width, height, stride, seed=0):
    """One pixel per stride x stride cell (seeded position inside the cell)."""
    rng = np.random.default_rng(seed)
    ys = np.arange(0, height, stride)
    xs = np.arange(0, width, stride)
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    oy = rng.integers(0, stride, size=gy.shape)
    ox = rng.integers(0, stride, size=gx.shape)
    py = np.minimum(gy + oy, height - 1)
    px = np.minimum(gx + ox, width - 1)
    return (py * width + px).ravel().astype(np.int64)
