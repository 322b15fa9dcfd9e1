"""FP64 finite differences of the oracle render for the gradient tests.

A parameter slot is perturbed by +-h and +-h/4; a pixel is stable for that
slot when its status and its escape counts at the hit point and at every
normal tap are unchanged by all four perturbations, and its difference
quotient has converged (the h and h/4 quotients agree to 1e-4 of the pixel's
scale).  Chaotic pixels have large higher derivatives, so the convergence
condition removes the few where truncation error dominates.  Slots: c0-c3,
power, plane 0 (raw n xyz, d), plane 1.
"""
import copy

import numpy as np


def perturb(job, slot, h):
    j = copy.deepcopy(job)
    if slot < 4:
        j["fractal"]["c"] = list(j["fractal"]["c"])
        j["fractal"]["c"][slot] += h
    elif slot == 4:
        j["fractal"]["power"] += h
    else:
        k, e = (slot - 5) // 4, (slot - 5) % 4
        if e < 3:
            j["planes"][k]["n"] = list(j["planes"][k]["n"])
            j["planes"][k]["n"][e] += h
        else:
            j["planes"][k]["d"] += h
    return j


def rows(out):
    """Per-pixel outputs as rows: depth, normal xyz, colour rgb."""
    return np.concatenate([out["depth"][None], out["normal"], out["colour"]], 0)


def finite_differences(orc, job, pix, slots, base_status, base_taps, scale, h=1e-6):
    """Central differences [7, n] per slot at step h/4, and the per-slot
    stability masks [n] (see the module docstring).  scale [7, n, 13]: the
    magnitude of each pixel's derivatives used by the convergence test."""
    fd, stable = {}, {}
    for s in slots:
        outs, ok = {}, np.ones(pix.size, bool)
        for hh in (h, -h, h / 4, -h / 4):
            jp = perturb(job, s, hh)
            o = orc.render(jp, pix)
            _, tp = orc.pixel_jacobian(jp, pix)
            ok &= (o["status"] == base_status) & np.all(tp == base_taps, 1)
            outs[hh] = rows(o)
        fd1 = (outs[h] - outs[-h]) / (2 * h)
        fd2 = (outs[h / 4] - outs[-h / 4]) / (h / 2)
        ok &= np.all(np.abs(fd1 - fd2) <= 1e-4 * scale[:, :, s], 0)
        fd[s], stable[s] = fd2, ok
    return fd, stable
