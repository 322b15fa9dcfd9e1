"""Pin of the oracle's forward-mode (dual-number) Jacobian against central
finite differences of the oracle's own FP64 render.

A pixel takes part when its branch structure is unchanged by the
perturbation (status, escape counts at the hit point and at every normal
tap) and its finite-difference quotient has converged (steps h and h/4
agree); chaotic pixels have large higher derivatives, so the second
condition removes the few where truncation error dominates.
"""
import copy

import numpy as np
import pytest

import workloads as W


def _perturb(job, slot, h):
    j = copy.deepcopy(job)
    if slot < 4:
        j["fractal"]["c"][slot] += h
    elif slot == 4:
        j["fractal"]["power"] += h
    else:
        k, e = (slot - 5) // 4, (slot - 5) % 4
        if e < 3:
            j["planes"][k]["n"][e] += h
        else:
            j["planes"][k]["d"] += h
    return j


def _rows(out):
    return np.concatenate([out["depth"][None], out["normal"], out["colour"]], 0)


CASES = {
    "julia_cut": (lambda: W.julia_view(width=48, height=48, planes=[W.plane([0.3, 0.2, 1.0], 0.05)]),
                  [0, 1, 2, 3, 5, 6, 7, 8]),
    "julia_two_planes": (lambda: W.julia_view(width=40, height=40, planes=[W.plane([0.3, 0.2, 1.0], 0.05),
                                                                           W.plane([-1.0, 0.4, 0.2], 0.3)]),
                         [0, 3, 9, 10, 11, 12]),
    "bulb_cut_shadow": (lambda: W.bulb_view(0.7, 0.2, width=40, height=40, shadow=True,
                                            planes=[W.plane([0.2, 1.0, 0.1], 0.1)]), [4, 5, 6, 7, 8]),
    "bulb_real_power": (lambda: W.bulb_view(2.1, -0.3, width=40, height=40, power=6.37, shadow=False),
                        [4]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pixel_jacobian_matches_finite_differences(orc, case):
    make, slots = CASES[case]
    jb = make()
    base = orc.render(jb)
    cls = base["status"] & 7
    smooth = (base["status"] & (orc.FLAG_UNREFINED | orc.FLAG_JUMP)) == 0
    pix = np.nonzero(np.isin(cls, [orc.STATUS_HIT, orc.STATUS_HIT_CUT]) & smooth)[0]
    assert pix.size > 200
    J, taps = orc.pixel_jacobian(jb, pix)
    h = 1e-6
    used = 0
    for s in slots:
        outs, stable = {}, np.ones(pix.size, bool)
        for hh in (h, -h, h / 4, -h / 4):
            jp = _perturb(jb, s, hh)
            o = orc.render(jp, pix)
            _, tp = orc.pixel_jacobian(jp, pix)
            stable &= (o["status"] == base["status"][pix]) & np.all(tp == taps, 1)
            outs[hh] = _rows(o)
        fd1 = (outs[h] - outs[-h]) / (2 * h)
        fd2 = (outs[h / 4] - outs[-h / 4]) / (h / 2)
        ad = J[:, :, s].T
        scale = 1.0 + np.abs(ad)
        converged = np.all(np.abs(fd1 - fd2) <= 1e-4 * scale, 0)
        ok = stable & converged
        assert ok.mean() > 0.97, (s, stable.mean(), converged.mean())
        err = np.abs(fd2 - ad)[:, ok] / scale[:, ok]
        assert err.max() < 2e-4, (s, err.max())
        used += ok.sum()
    assert used > 0
