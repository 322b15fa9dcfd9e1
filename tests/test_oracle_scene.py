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


# ------------------------------------------------ closest-hit shading (R23)
def _ball(translation, scale):
    fr = W.julia([0, 0, 0, 0], 11, bound_radius=1.5)
    return W.scene_object(fr, translation=translation, scale=scale)


def _rho(eps):
    from scipy.optimize import brentq
    import math
    return brentq(lambda r: 0.5 * r * math.log(r) - eps, 1.0, 2.0, xtol=1e-15)


def _phong_closed(N, L, V, albedo, mc):
    """Phong colour [3, n]; albedo [3] or per point [3, n]."""
    ndl = N @ L
    Rl = 2.0 * ndl[:, None] * N - L
    spec = np.where(ndl > 0, np.maximum(0.0, np.einsum("ij,ij->i", Rl, V)) ** mc["shininess"], 0.0)
    alb = albedo if albedo.ndim == 2 else albedo[:, None]
    return alb * (mc["k_ambient"] + mc["k_diffuse"] * np.maximum(0, ndl))[None, :] + \
        mc["k_specular"] * spec[None, :]


def _trap_c0(p, max_iter, bailout2):
    """Orbit trap of a c = 0 degree-2 Julia point in closed form: z_k =
    zeta^(2^k) in span{1, v_hat} with zeta = x + i |v| (R24's minima of |x|,
    |y|, |z| and |z|^2 over the start point and every body run)."""
    v = p[1:]
    vn = np.linalg.norm(v)
    tr = [abs(p[0]), abs(p[1]), abs(p[2]), p @ p]
    z = complex(p[0], vn)
    for _ in range(max_iter):
        z = z * z
        comp = [abs(z.real), abs(z.imag * v[0] / vn), abs(z.imag * v[1] / vn), abs(z) ** 2]
        tr = [min(a, b) for a, b in zip(tr, comp)]
        if abs(z) ** 2 > bailout2:
            break
    return np.array(tr)


def _trap_albedo(albedo, pal, traps):
    return np.clip(albedo[:, None] + np.asarray(pal, np.float64).T @ traps, 0.0, 1.0)


def test_trap_colouring_on_the_c0_ball_is_closed_form(orc):
    """The closest-hit shading with the trap palette on one c = 0 ball: each
    hit's albedo is albedo + palette . T, clamped, with the trap T of the
    hit point in closed form (complex powers), and the colour is the Phong
    term of the radial normal with that albedo."""
    mc = W.phong(W.march(256, eps_abs=1e-3, normal_mode="analytic"), trap_colour=True)
    sc = W.scene(W.camera((0.3, 0.8, 3.0), 80, 80), [_ball((0.0, 0.0, 0.0), 1.0)], mc)
    out = orc.render_scene(sc)
    hit = np.nonzero(out["object_id"] == 0)[0]
    assert hit.size > 1000
    o, d = orc.camera_rays(sc["camera"], hit)
    p = o + out["depth"][hit, None] * d
    fr = sc["objects"][0]["fractal"]
    _, T0, s0 = orc.object_frame(sc["objects"][0])
    traps = np.array([_trap_c0((q - T0) / s0, fr["max_iter"], fr["bailout2"]) for q in p]).T
    alb = _trap_albedo(np.array(mc["albedo"], dtype=np.float64), mc["trap_colour"], traps)
    assert np.ptp(alb, axis=1).min() > 0.05        # the palette does colour the ball
    N = p / np.linalg.norm(p, axis=1, keepdims=True)
    L = np.array(mc["light_dir"], dtype=np.float64)
    L /= np.linalg.norm(L)
    ref = _phong_closed(N, L, -d, alb, mc)
    assert np.abs(out["colour"][:, hit] - ref).max() < 1e-6


def test_phong_on_the_c0_ball_is_closed_form(orc):
    """One c = 0 ball (convex: no reflection ray comes back to it): colour is
    the Phong term of the radial normal, no pixel reports a reflection hit."""
    mc = W.phong(W.march(256, eps_abs=1e-3, normal_mode="analytic"))
    sc = W.scene(W.camera((0.3, 0.8, 3.0), 96, 96), [_ball((0.0, 0.0, 0.0), 1.0)], mc)
    out = orc.render_scene(sc)
    hit = np.nonzero(out["object_id"] == 0)[0]
    assert hit.size > 1000
    assert not np.any(out["status"] & orc.FLAG_REFLECT_HIT)
    o, d = orc.camera_rays(sc["camera"], hit)
    p = o + out["depth"][hit, None] * d
    N = p / np.linalg.norm(p, axis=1, keepdims=True)
    L = np.array(mc["light_dir"], dtype=np.float64)
    L /= np.linalg.norm(L)
    ref = _phong_closed(N, L, -d, np.array(mc["albedo"], dtype=np.float64), mc)
    assert np.abs(out["colour"][:, hit] - ref).max() < 1e-6


@pytest.mark.parametrize("trap_colour", [False, True])
def test_reflection_between_two_balls_is_closed_form(orc, trap_colour):
    """Two c = 0 balls (radius s rho_eps): where a reflection ray from ball A
    meets ball B (ray-sphere intersection in closed form), the colour is
    A's Phong term plus 0.1 Schlick(f0 = albedo) times B's Phong term at the
    intersection; elsewhere the reflection adds nothing.  With the trap
    palette, A's albedo (also Fresnel's f0) and B's albedo at the
    reflected hit are coloured by the closed-form traps of the two points."""
    mc = W.phong(W.march(256, eps_abs=1e-3, t_max=20.0, normal_mode="analytic"), trap_colour=trap_colour)
    A, B = (-0.7, 0.0, 0.0), (0.75, 0.1, -0.3)
    sA, sB = 0.6, 0.5
    sc = W.scene(W.camera((0.0, 0.3, 3.0), 128, 96), [_ball(A, sA), _ball(B, sB)], mc)
    out = orc.render_scene(sc)
    pix = np.nonzero(out["object_id"] == 0)[0]
    o, d = orc.camera_rays(sc["camera"], pix)
    t = out["depth"][pix]
    Av, Bv = np.array(A, dtype=np.float64), np.array(B, dtype=np.float64)
    p = o + t[:, None] * d
    N = (p - Av) / np.linalg.norm(p - Av, axis=1, keepdims=True)
    L = np.array(mc["light_dir"], dtype=np.float64)
    L /= np.linalg.norm(L)
    albedo = np.array(mc["albedo"], dtype=np.float64)
    pal = mc.get("trap_colour", [[0.0] * 3] * 4)
    fr = sc["objects"][0]["fractal"]
    # traps in each object's own frame (its float32 placement: the trap is
    # sensitive to the point at the 1e-7 level)
    _, TA, sAf = orc.object_frame(sc["objects"][0])
    _, TB, sBf = orc.object_frame(sc["objects"][1])
    albA = _trap_albedo(albedo, pal, np.array([_trap_c0((q - TA) / sAf, fr["max_iter"], fr["bailout2"])
                                                for q in p]).T)
    base = _phong_closed(N, L, -d, albA, mc)
    # reflected ray against B's eps-level sphere (world radius sB rho(eps_B))
    eps_s = mc["eps_abs"] + 0.0 * t
    dn = np.einsum("ij,ij->i", d, N)
    rd = d - 2 * dn[:, None] * N
    q = p + 4 * eps_s[:, None] * N
    # in B's frame the level set sits where 0.5 r ln r = eps_s / sB (eps_rel = 0)
    rB = np.array([sB * _rho(e / sB) for e in eps_s])
    oc = q - Bv
    bq = np.einsum("ij,ij->i", oc, rd)
    disc = bq ** 2 - (np.einsum("ij,ij->i", oc, oc) - rB ** 2)
    meets = disc > 0
    th = np.where(meets, -bq - np.sqrt(np.maximum(disc, 0)), np.inf)
    meets &= th > 0
    clear = np.abs(disc) > 1e-3                        # away from B's silhouette
    assert np.sum(meets & clear) > 30
    hp = q + np.where(meets, th, 0.0)[:, None] * rd
    NB = (hp - Bv) / np.linalg.norm(hp - Bv, axis=1, keepdims=True)
    if trap_colour:
        # a trap component at the reflected hit can move by 4e-4 when the
        # point moves by 1e-7 (here: the radial normal against the oracle's
        # analytic one), so the closed-form trap is taken at the oracle's own
        # reflected hit, checked first against the closed-form intersection
        Rb, Tb, sb = orc.object_frame(sc["objects"][1])
        nrm = out["normal"][:, pix].T
        dno = np.einsum("ij,ij->i", d, nrm)
        rdo = d - 2 * dno[:, None] * nrm
        qo = p + 4 * eps_s[:, None] * nrm
        r = orc.trace_rays(sc["objects"][1]["fractal"], [], orc.object_march(mc, sb), (qo - Tb) @ Rb / sb, rdo @ Rb,
                           eps0=eps_s / sb)
        hpo = qo + (r["depth"] * sb)[:, None] * rdo
        both = meets & clear & ((r["status"] & 7) >= 2)
        assert np.abs(hpo[both] - hp[both]).max() < 1e-6
        hp = np.where(both[:, None], hpo, hp)
    albB = _trap_albedo(albedo, pal, np.array([_trap_c0((q - TB) / sBf, fr["max_iter"], fr["bailout2"])
                                                for q in hp]).T)
    c_r = _phong_closed(np.where(meets[:, None], NB, 0.0), L, -rd, albB, mc)
    F = albA + (1 - albA) * ((1 - np.maximum(0, -dn)) ** 5)[None, :]
    ref = base + np.where(meets[None, :], mc["k_reflect"] * F * c_r, 0.0)
    flag = (out["status"][pix] & orc.FLAG_REFLECT_HIT) != 0
    assert np.array_equal(flag[clear], meets[clear])
    assert np.abs(out["colour"][:, pix][:, clear] - ref[:, clear]).max() < 1e-5


def test_orbit_trap_of_c0_julia_is_closed_form(orc):
    """c = 0, degree 2: z_k = z^(2^k) stays in the complex plane span{1, v};
    its components are Re(zeta^(2^k)) and Im(zeta^(2^k)) v_hat with
    zeta = x + i|v|, so the trap follows from complex powers."""
    rng = np.random.default_rng(90)
    pts = rng.normal(size=(300, 3))
    pts *= (rng.uniform(0.7, 1.3, size=300) / np.linalg.norm(pts, axis=1))[:, None]
    fr = W.julia([0, 0, 0, 0], 6)
    got = orc.orbit_trap(fr, pts)
    for p, g in zip(pts, got):
        v = p[1:]
        vn = np.linalg.norm(v)
        zeta = complex(p[0], vn)
        tr = [abs(p[0]), abs(p[1]), abs(p[2]), p @ p]
        z = zeta
        for _ in range(6):
            z = z * z
            comp = [abs(z.real), abs(z.imag * v[0] / vn), abs(z.imag * v[1] / vn), abs(z) ** 2]
            tr = [min(a, b) for a, b in zip(tr, comp)]
            if abs(z) ** 2 > 256.0:
                break
        np.testing.assert_allclose(g, tr, rtol=1e-9, atol=1e-12)
