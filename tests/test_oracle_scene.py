"""Pins of the oracle's scene composition (several fractal objects placed by
similarity maps, closest hit, shadows across objects) and of the
iteration-count animation, against definitions that do not go through the
scene code: single-object renders, a transformed camera, and per-object
minima.  No GPU needed."""
import copy

import numpy as np
import pytest

import workloads as W


def _single(orc, sc, k):
    """Scene with object k alone."""
    one = copy.deepcopy(sc)
    one["objects"] = [one["objects"][k]]
    return orc.render_scene(one)


@pytest.mark.parametrize("which", ["julia_cut_shadow", "bulb_shadow"])
def test_identity_object_equals_single_render(orc, which):
    if which == "julia_cut_shadow":
        jb = W.julia_view(width=72, height=60, planes=[W.plane([0.3, 0.2, 1.0], 0.05)], shadow=True)
    else:
        jb = W.bulb_view(0.4, 0.2, width=72, height=60, shadow=True)
    sc = W.scene(jb["camera"], [W.scene_object(jb["fractal"], jb["planes"])], jb["march"])
    a, b = orc.render(jb), orc.render_scene(sc)
    assert np.array_equal(a["status"], b["status"])
    assert np.array_equal(a["depth"], b["depth"])
    assert np.abs(a["normal"] - b["normal"]).max() < 1e-15
    assert np.abs(a["colour"] - b["colour"]).max() < 1e-15
    hit = b["object_id"] == 0
    assert np.array_equal(hit, (a["status"] & 7) >= 2)
    assert np.array_equal(a["steps"][hit], b["steps"][hit])


@pytest.mark.parametrize("rot", ["signed_cycle", "general"])
@pytest.mark.parametrize("kind", ["julia", "bulb"])
def test_similarity_equivariance(orc, kind, rot):
    """An object placed by (R, T, s) and seen from camera C renders like the
    untransformed object seen from the camera mapped into its frame, with
    eps_abs, step_clamp and t_max divided by s and the light rotated by R^T:
    depth scales by s, normals rotate by R, colours and classes agree.
    "signed_cycle": R a signed cyclic permutation (det +1, R != R^T), s = 2
    and dyadic T, so every map is exact and the two renders agree to
    rounding.  "general": a float32 rotation, whose transpose is its inverse
    only to ~2e-7; the hit points then move by that much, and the normals by
    what the surface's curvature makes of it."""
    if kind == "julia":
        fr, planes = W.julia(W.JULIA_C1, 11), [W.plane([0.3, 0.2, 1.0], 0.05)]
        mc = W.march(256, eps_abs=1e-3, eps_rel=2e-4, shadow=True, t_max=30.0)
    else:
        fr, planes = W.bulb(8.0, 10), []
        mc = W.march(512, eps_rel=5e-4, normal_mode="central", shadow=True, t_max=30.0)
    if rot == "signed_cycle":
        R9, T, s = [0.0, 0.0, 1.0, -1.0, 0.0, 0.0, 0.0, -1.0, 0.0], [0.5, -0.25, 0.75], 2.0
    else:
        R9, T, s = W.rotation([0.3, 1.0, -0.4], 0.9), [0.4, -0.3, 0.7], 1.7
    cam = W.camera((0.5, 1.25, 5.0), 64, 48, target=T)
    sc = W.scene(cam, [W.scene_object(fr, planes, R9, T, s)], mc)
    R = np.array(R9, dtype=np.float64).reshape(3, 3)
    Tv = np.array(T, dtype=np.float64)
    to_obj = lambda x: (np.asarray(x, dtype=np.float64) - Tv) @ R / s
    jb = {"camera": {"eye": list(to_obj(cam["eye"])), "target": list(to_obj(cam["target"])),
                     "up": list(np.asarray(cam["up"], dtype=np.float64) @ R), "fov_y_deg": cam["fov_y_deg"],
                     "width": cam["width"], "height": cam["height"]},
          "fractal": fr, "planes": planes, "march": dict(mc)}
    for key in ("eps_abs", "step_clamp", "t_max"):
        jb["march"][key] = mc[key] / s
    jb["march"]["light_dir"] = list(np.asarray(mc["light_dir"], dtype=np.float64) @ R)
    a, b = orc.render(jb), orc.render_scene(sc)
    hit = (a["status"] & 7) >= 2
    assert hit.sum() > 300
    assert np.array_equal(a["status"] & 7, b["status"] & 7)
    same_shadow = (a["status"] & 8) == (b["status"] & 8)
    assert same_shadow.mean() > 0.999
    keep = hit & same_shadow
    rn = R @ a["normal"][:, hit]
    dn = np.linalg.norm(b["normal"][:, hit] - rn, axis=0)
    if rot == "signed_cycle":
        np.testing.assert_allclose(b["depth"][hit], s * a["depth"][hit], rtol=1e-12)
        assert dn.max() < 1e-8
        np.testing.assert_allclose(b["colour"][:, keep], a["colour"][:, keep], atol=1e-9)
    else:
        assert np.abs(R @ R.T - np.eye(3)).max() < 3e-7
        np.testing.assert_allclose(b["depth"][hit], s * a["depth"][hit], rtol=1e-6)
        assert np.median(dn) < 1e-5 and np.percentile(dn, 99) < 2e-4


@pytest.mark.parametrize("name", ["julia_bulb", "overlap"])
def test_closest_hit_is_the_minimum_over_objects(orc, name):
    """Without shadows, every pixel shows the object with the smallest
    single-object depth, with that object's depth, normal and colour."""
    sc = W.julia_bulb_scene(width=96, height=60, shadow=False) if name == "julia_bulb" else \
        W.overlap_scene(width=96, height=72, shadow=False)
    out = orc.render_scene(sc)
    singles = [_single(orc, sc, k) for k in range(len(sc["objects"]))]
    D = np.stack([np.where(s_["depth"] >= 0, s_["depth"], np.inf) for s_ in singles])
    ref_id = np.where(np.isinf(D.min(0)), -1, D.argmin(0))
    assert np.array_equal(out["object_id"], ref_id)
    for k, s_ in enumerate(singles):
        m = out["object_id"] == k
        assert np.array_equal(out["depth"][m], s_["depth"][m])
        assert np.array_equal(out["status"][m], s_["status"][m])
        assert np.abs(out["colour"][:, m] - s_["colour"][:, m]).max(initial=0.0) < 1e-15
    if name == "overlap":     # objects really occlude one another
        assert (np.isfinite(D).sum(0) >= 2).sum() > 500


def test_shadows_fall_across_objects(orc):
    """In the overlap scene some pixels of each rear object are shadowed
    only because another object blocks the light: shadowed in the scene, lit
    when the object is rendered alone."""
    sc = W.overlap_scene(width=128, height=96)
    out = orc.render_scene(sc)
    cross = 0
    for k in range(len(sc["objects"])):
        alone = _single(orc, sc, k)
        m = out["object_id"] == k
        cross += int(np.sum(m & ((out["status"] & 8) != 0) & ((alone["status"] & 8) == 0)))
        # a pixel shadowed alone stays shadowed in the scene
        assert not np.any(m & ((alone["status"] & 8) != 0) & ((out["status"] & 8) == 0))
    assert cross > 50, cross


def test_iteration_animation_frames(orc):
    """Fig. 2's animation by iteration count: frame k uses k + 1 orbit
    bodies and nothing else changes; the frames differ (the estimate, and
    with it the surface, depends on the budget) and every frame hits."""
    frames = W.iteration_animation(n_frames=6, width=64, height=36, shadow=False)
    assert [f["fractal"]["max_iter"] for f in frames] == [1, 2, 3, 4, 5, 6]
    for f in frames[1:]:
        g = copy.deepcopy(f)
        g["fractal"]["max_iter"] = 1
        assert g == frames[0]
    outs = [orc.render(f) for f in frames]
    assert all(((o["status"] & 7) >= 2).sum() > 500 for o in outs)
    assert all(not np.array_equal(a["depth"], b["depth"]) for a, b in zip(outs, outs[1:]))
