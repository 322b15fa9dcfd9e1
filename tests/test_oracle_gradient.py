"""Pin of the oracle's forward-mode (dual-number) Jacobian against central
finite differences of the oracle's own FP64 render.

A pixel takes part when its branch structure is unchanged by the
perturbation (status, escape counts at the hit point and at every normal
tap) and its finite-difference quotient has converged (steps h and h/4
agree); chaotic pixels have large higher derivatives, so the second
condition removes the few where truncation error dominates.
"""
import numpy as np
import pytest

import workloads as W
from gradcheck import finite_differences


CASES = {
    "julia_cut": (lambda: W.julia_view(width=48, height=48, planes=[W.plane([0.3, 0.2, 1.0], 0.05)]),
                  [0, 1, 2, 3, 5, 6, 7, 8]),
    # a wedge: each plane is the entry plane of about half the cut face
    "julia_two_planes": (lambda: W.julia_view(width=40, height=40, planes=[W.plane([0.6, 0.0, 0.8], 0.0),
                                                                           W.plane([-0.6, 0.0, 0.8], 0.0)]),
                         [0, 3, 5, 8, 9, 10, 11, 12]),
    "julia_cubic_cut": (lambda: W.julia_view(width=44, height=44, degree=3, c=[-0.45, 0.1, 0.4, 0.2],
                                             planes=[W.plane([-0.2, 0.3, 1.0], 0.1)]),
                        [0, 1, 2, 3, 5, 6, 7, 8]),
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
    scale = 1.0 + np.abs(J.transpose(1, 0, 2))            # [7, n, 13]
    fd, stable = finite_differences(orc, jb, pix, slots, base["status"][pix], taps, scale)
    used = 0
    for s in slots:
        ad = J[:, :, s].T
        sc = 1.0 + np.abs(ad)
        ok = stable[s]
        assert ok.mean() > 0.97, (s, ok.mean())
        assert np.abs(J[:, :, s]).max() > 0, s     # the slot is exercised
        err = np.abs(fd[s] - ad)[:, ok] / sc[:, ok]
        assert err.max() < 2e-4, (s, err.max())
        used += ok.sum()
    assert used > 0
