"""GPU-vs-oracle comparison rules shared by the GPU tests and the benchmark.

Every rule below is decided by the FP64 oracle alone (nothing the GPU
reports moves a pixel out of a comparison), and every exclusion is counted,
reported and bounded by the tests.

Hit/miss agreement is measured over every compared pixel.  Depth, class and
normal are compared where both sides hit and the pixel is not in the
boundary set B, the pixels whose outcome the oracle shows to be decided by
rounding rather than by the method:
  - an 8-neighbour has a different oracle hit/miss or cut-face outcome;
  - the oracle ran out of steps, or its root bracket closed on a jump of
    the estimate (no smooth root there);
  - the ray grazes the surface (|N . dir| < 0.05).
Depth tolerance: 2 eps(t*).  Several depths are correct where the march may
legitimately stop at another crossing of the eps-region: float32 and FP64
sample the ray at slightly different points, and near thin layers of the
estimate one side steps over a crossing the other stops at.  A depth that
differs by more than 2 eps is therefore accepted when the oracle confirms it
is a root: d - eps, evaluated by the oracle in FP64, changes sign within
2 eps of the GPU's depth (inside the ray's interval).  Such pixels are
counted (depth_other_root) and bounded.  Where the oracle's own final march
bracket holds more than one crossing (counted on 257 samples) a depth inside
that bracket is accepted as before (depth_multi_root).

Normal tolerance: 1e-3 rad, measured against the oracle's normal evaluated
at the GPU's own hit point (which separates the normal estimate from the
depth error); the angle to the oracle's normal at its own hit point is
reported and bounded as well.  A normal is ill-conditioned at float32
resolution when
  - a tap's orbit comes within 1e-4 (relative) of the bailout (its escape
    count, where the estimate jumps, is decided by rounding); or
  - the FP64 normal moves by more than 2e-4 rad under float32-sized changes
    of its inputs: the power z^p of every orbit body perturbed by a random
    relative 2 p 2^-24 (the rounding budget of a p-th power in float32), over
    four seeds; or the point moved by one float32 ulp of its largest
    coordinate along each axis (the GPU forms its hit point in float32).
The 1e-3 bar applies to the well-conditioned normals; the ill-conditioned
ones are counted (normal_boundary_frac, bounded per test) and compared
against a tolerance scaled by their measured sensitivity,
max(1e-3, 10 x sensitivity), with the angle quantiles reported.

Colour (2e-3) is compared, like the normal, against the oracle's shading of
its normal at the GPU's hit point, where the shadow outcome agrees and the
normal is well conditioned; the colour against the oracle's own hit point is
reported and held to 99% agreement.  In scenes with the closest-hit shading
that shading includes the trap colouring and the reflection bounce from the
GPU's hit point.  The reflected ray amplifies the normal's error, so a
pixel's colour is compared only where tilting the oracle's normal by
REFLECT_TILT (four directions) moves the shaded colour by less than 1e-3 and
keeps the reflected hit or miss; the excluded share (reflect_ill_frac) is
bounded per test.
"""
import numpy as np

CLS_MASK = 7
HIT_CLASSES = (2, 3, 4)


def to_numpy(frame):
    out = {}
    for k, v in frame.items():
        out[k] = v.detach().cpu().numpy() if hasattr(v, "detach") else np.asarray(v)
    return out


def angle(a, b):
    """Angle between rows of a and b, each normalised in float64 first; the
    atan2 form stays accurate for nearly parallel vectors, where arccos of a
    dot product of float32-normalised vectors is not."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.einsum("...i,...i->...", a, b))


def neighbour_flags(status_img):
    """Per pixel: does any 8-neighbour differ in hit/miss or in cut-face-ness?"""
    cls = status_img & CLS_MASK
    hit = cls >= 2
    cut = cls == 3
    H, W = cls.shape
    diff = np.zeros((H, W), bool)
    hp = np.pad(hit, 1, mode="edge")
    cp = np.pad(cut, 1, mode="edge")
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            sh = hp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
            sc = cp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
            diff |= (sh != hit) | (sc != cut)
    return diff


def neighbourhood_pixels(pixels, width, height):
    """The 3x3 neighbourhoods (clamped) of sampled pixels, shape [n, 9]."""
    py, px = np.divmod(np.asarray(pixels, np.int64), width)
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            out.append(np.clip(py + dy, 0, height - 1) * width + np.clip(px + dx, 0, width - 1))
    return np.stack(out, 1)


def sampled_compare(orc, job, frame, pixels):
    """Compare a GPU frame (dict of torch tensors or numpy arrays) with the
    oracle on sampled pixels; the boundary rule uses the oracle's 3x3
    neighbourhood of every sample."""
    cam = job["camera"]
    W_, H = cam["width"], cam["height"]
    nb = neighbourhood_pixels(pixels, W_, H)
    o_nb = orc.render(job, pixels=nb.ravel())
    st_nb = o_nb["status"].reshape(nb.shape)
    hit_nb, cut_nb = (st_nb & CLS_MASK) >= 2, (st_nb & CLS_MASK) == 3
    nd = np.any(hit_nb != hit_nb[:, 4:5], 1) | np.any(cut_nb != cut_nb[:, 4:5], 1)
    o = {k: (v[..., 4::9] if v.ndim == 1 else v[:, 4::9]) for k, v in o_nb.items()}
    gs = {}
    for k, v in frame.items():
        if v is None:
            continue
        if hasattr(v, "detach"):
            import torch
            idx = torch.as_tensor(pixels, device=v.device)
            gs[k] = (v[idx] if v.dim() == 1 else v[:, idx]).cpu().numpy()
        else:
            gs[k] = v[pixels] if v.ndim == 1 else v[:, pixels]
    if "counters" in gs:
        gs["counters"] = gs["counters"].view(np.uint32) if gs["counters"].dtype == np.int32 else gs["counters"]
    return compare(orc, job, gs, o, nd, pixels=pixels)


def normal_sensitivity(orc, fr, mc, pts, dirs, eps, seeds=4, margin=1e-4):
    """Per point: (sensitivity, low_margin).  sensitivity is the largest angle
    by which the FP64 normal moves under float32-sized changes of its inputs
    (the rounding probe of every orbit body's power over `seeds` draws, and a
    shift of the point by 2^-23 max|p_k| along each axis); low_margin marks a
    tap whose orbit comes within `margin` (relative) of the bailout."""
    n = len(pts)
    if n == 0:
        return np.zeros(0), np.zeros(0, bool)
    pts = np.asarray(pts, np.float64)
    eps = np.broadcast_to(np.asarray(eps, np.float64), (n,))
    tp = orc.tap_points(pts, eps, mc["normal_mode"])
    mg, _ = orc.escape_margin(fr, tp.reshape(-1, 3))
    low = mg.reshape(n, tp.shape[1]).min(1) < margin
    p = fr["power"]          # Mandelbulb n, or the Julia degree
    ref = orc.normal_at(fr, pts, dirs, eps, mc["normal_mode"])
    sens = np.zeros(n)
    for s in range(seeds):
        pert = orc.normal_perturbed(fr, pts, dirs, eps, mc["normal_mode"], 2.0 * p * 2.0 ** -24, 1000 + s)
        sens = np.maximum(sens, angle(pert, ref))
    delta = 2.0 ** -23 * np.abs(pts).max(1)
    for ax in range(3):
        for sg in (-1.0, 1.0):
            q = pts.copy()
            q[:, ax] += sg * delta
            sens = np.maximum(sens, angle(orc.normal_at(fr, q, dirs, eps, mc["normal_mode"]), ref))
    return sens, low


def normal_ill_conditioned(orc, fr, mc, pts, dirs, eps, tol=2e-4, margin=1e-4):
    """Per point: is the FP64 normal estimate ill-conditioned at float32
    resolution (see the module docstring)?"""
    sens, low = normal_sensitivity(orc, fr, mc, pts, dirs, eps, margin=margin)
    return (sens > tol) | low


def trap_ill_conditioned(orc, fr, pts, seeds=4, tol=1e-4, margin=1e-4):
    """Per point: is the FP64 orbit trap ill-conditioned at float32
    resolution?  When a trap component moves by more than tol under the
    rounding probe of every body's power (relative 2 p 2^-24, `seeds`
    draws) or under a shift of the point by 2^-23 max|p_k| along each axis,
    or an orbit body comes within `margin` (relative) of the bailout."""
    pts = np.asarray(pts, np.float64)
    if len(pts) == 0:
        return np.zeros(0, bool)
    ref = orc.orbit_trap(fr, pts)
    rel = 2.0 * fr["power"] * 2.0 ** -24
    ill = np.zeros(len(pts), bool)
    for sd in range(seeds):
        ill |= np.any(np.abs(orc.orbit_trap_perturbed(fr, pts, rel, 2000 + sd) - ref) > tol, axis=1)
    delta = 2.0 ** -23 * np.abs(pts).max(1)
    for ax in range(3):
        for sg in (-1.0, 1.0):
            q = pts.copy()
            q[:, ax] += sg * delta
            ill |= np.any(np.abs(orc.orbit_trap(fr, q) - ref) > tol, axis=1)
    mg, _ = orc.escape_margin(fr, pts)
    return ill | (mg < margin)


def ray_interval(orc, job, orig, dirs):
    """The oracle's search interval [lo, hi] of each ray: [eps_abs, t_max]
    cut by the bounding sphere and the kept half-spaces (empty: lo > hi)."""
    fr, mc = job["fractal"], job["march"]
    R = max(orc.bound_radius(fr), float(fr.get("bound_radius", 0.0)))
    b = np.einsum("ij,ij->i", orig, dirs)
    disc = b * b - (np.einsum("ij,ij->i", orig, orig) - R * R)
    sq = np.sqrt(np.maximum(disc, 0.0))
    lo = np.maximum(mc["eps_abs"], -b - sq)
    hi = np.where(disc >= 0.0, np.minimum(mc["t_max"], -b + sq), -np.inf)
    for pl in job.get("planes", []):
        nh = np.asarray(pl["n"], np.float64)
        nh = nh / np.linalg.norm(nh)
        den = dirs @ nh
        num = pl["d"] - orig @ nh
        with np.errstate(divide="ignore", invalid="ignore"):
            tk = num / den
        hi = np.where(den > 0.0, np.minimum(hi, tk), hi)
        lo = np.where(den < 0.0, np.maximum(lo, tk), lo)
        hi = np.where((den == 0.0) & (num < 0.0), -np.inf, hi)
    return lo, hi


def oracle_root_near(orc, job, orig, dirs, t, halfwidth, samples=32):
    """Per ray: does g(s) = d(o + s dir) - eps(s), evaluated by the oracle,
    change sign on [t - halfwidth, t + halfwidth] within the ray's interval
    (samples + 1 uniform points)?"""
    if len(t) == 0:
        return np.zeros(0, bool)
    fr, mc = job["fractal"], job["march"]
    lo, hi = ray_interval(orc, job, orig, dirs)
    s = np.asarray(t, np.float64)[:, None] + np.linspace(-1.0, 1.0, samples + 1)[None] * halfwidth[:, None]
    inside = (s >= lo[:, None]) & (s <= hi[:, None])
    pts = orig[:, None, :] + s[..., None] * dirs[:, None, :]
    d = orc.de(fr, pts.reshape(-1, 3))[0].reshape(s.shape)
    g = d - (mc["eps_abs"] + mc["eps_rel"] * s)
    neg = np.any(inside & (g < 0.0), 1)
    pos = np.any(inside & (g >= 0.0), 1)
    return neg & pos


def boundary_set(o, neigh_diff, dirs):
    """The boundary set B of the module docstring (per compared pixel),
    from the oracle's render o alone."""
    os_ = o["status"].astype(np.int64)
    oc = os_ & CLS_MASK
    B = neigh_diff.copy()
    B |= (oc == 4) | ((os_ & 32) != 0)
    B |= (oc >= 2) & (np.abs(np.einsum("ij,ij->i", o["normal"].T, dirs)) < 0.05)
    return B


def adjoint_mask(orc, job, g, o, pixels=None, neigh_diff=None):
    """Pixels where the adjoint's per-pixel contribution is compared (the
    whole image, or the listed pixels with their neighbour flags): both
    sides report the same smooth hit class (refined surface hit or cut
    face) at the same root (depths within 2 eps), the pixel is outside B,
    a surface hit's normal is well conditioned at float32 resolution and
    every normal tap's orbit escapes, and the oracle's final march bracket
    holds a single crossing of d - eps.  Elsewhere the two sides may
    legitimately differentiate different branches: a bracket with several
    crossings holds roots closer together than 2 eps (typically two smooth
    roots on either side of a jump of the estimate, where the escape count
    changes), so the depth test cannot tell which one each side polished,
    and the derivatives at the two differ by far more than the 1e-3 bar."""
    cam, mc, fr = job["camera"], job["march"], job["fractal"]
    H, W = cam["height"], cam["width"]
    if pixels is None:
        pixels = np.arange(H * W)
        neigh_diff = neighbour_flags(o["status"].reshape(H, W)).ravel()
    gs, os_ = g["status"].astype(np.int64), o["status"].astype(np.int64)
    gc, oc = gs & CLS_MASK, os_ & CLS_MASK
    _, dirs = orc.camera_rays(cam, pixels)
    B = boundary_set(o, neigh_diff, dirs)
    smooth = ((gs & 16) == 0) & ((os_ & (16 | 32)) == 0) & np.isin(gc, (2, 3)) & (gc == oc)
    shade_same = (gs & 8) == (os_ & 8)
    eps_o = mc["eps_abs"] + mc["eps_rel"] * np.maximum(o["depth"], 0.0)
    same_root = np.abs(g["depth"].astype(np.float64) - o["depth"]) <= 2.0 * eps_o
    M = smooth & shade_same & same_root & ~B
    surf = np.nonzero(M & (gc == 2))[0]
    if surf.size:
        orig, d = orc.camera_rays(cam, pixels[surf])
        ts = g["depth"][surf].astype(np.float64)
        pts = orig + ts[:, None] * d
        eps = mc["eps_abs"] + mc["eps_rel"] * ts
        bad = normal_ill_conditioned(orc, fr, mc, pts, d, eps)
        # the parameter derivative of an estimate whose orbit never escapes
        # runs through the whole interior orbit: there it changes beyond the
        # 1e-3 bar between the float32 hit point and the oracle's
        tp = orc.tap_points(pts, eps, mc["normal_mode"])
        _, esc = orc.escape_margin(fr, tp.reshape(-1, 3))
        bad |= ~esc.reshape(surf.size, tp.shape[1]).all(1)
        _, _, crossings = orc.bracket_crossings(job, pixels[surf])
        bad |= crossings > 1
        M[surf[bad]] = False
    return M


def sampled_adjoint_mask(orc, job, frame, pixels):
    """adjoint_mask on sampled pixels of a GPU frame (torch tensors or numpy
    planes of the whole image), with the oracle's 3x3 neighbourhoods for the
    boundary rule.  Returns (mask, GPU planes at the pixels, oracle render
    of the pixels)."""
    cam = job["camera"]
    nb = neighbourhood_pixels(pixels, cam["width"], cam["height"])
    o_nb = orc.render(job, pixels=nb.ravel())
    st_nb = o_nb["status"].reshape(nb.shape)
    hit_nb, cut_nb = (st_nb & CLS_MASK) >= 2, (st_nb & CLS_MASK) == 3
    nd = np.any(hit_nb != hit_nb[:, 4:5], 1) | np.any(cut_nb != cut_nb[:, 4:5], 1)
    o = {k: (v[..., 4::9] if v.ndim == 1 else v[:, 4::9]) for k, v in o_nb.items()}
    gs = {}
    for k in ("depth", "status", "normal", "colour"):
        v = frame[k]
        if hasattr(v, "detach"):
            import torch
            idx = torch.as_tensor(pixels, device=v.device)
            gs[k] = (v[idx] if v.dim() == 1 else v[:, idx]).cpu().numpy()
        else:
            gs[k] = v[pixels] if v.ndim == 1 else v[:, pixels]
    return adjoint_mask(orc, job, gs, o, pixels=np.asarray(pixels), neigh_diff=nd), gs, o


def jacobian_sensitivity(orc, job, pix, J0, slots, shift=2e-7):
    """Per pixel: the largest relative change of the oracle's Jacobian
    (columns `slots`, relative to 1e-3 + |J|) when the camera is shifted by
    `shift` along each axis.  The GPU forms its hit point in float32 (depth
    and ray direction rounded at ~1e-7), and on fine fractal detail the
    derivatives of the normal change measurably over that distance; where
    this sensitivity is large the two sides differentiate at legitimately
    different points."""
    import copy
    sens = np.zeros(pix.size)
    ref = J0[:, :, slots]
    for ax in range(3):
        for sg in (-1.0, 1.0):
            jb = copy.deepcopy(job)
            eye = list(jb["camera"]["eye"])
            eye[ax] = float(np.float64(eye[ax]) + sg * shift)
            jb["camera"]["eye"] = eye
            J1, _ = orc.pixel_jacobian(jb, pix)
            rel = np.abs(J1[:, :, slots] - ref) / (1e-3 + np.abs(ref))
            sens = np.maximum(sens, rel.max(axis=(1, 2)))
    return sens


def _normal_stats(stats, ang, sens, ill):
    """Normal figures of a comparison: the 1e-3 bar on the well-conditioned
    normals, the sensitivity-scaled bar on all of them, and quantiles of the
    angle on the excluded set."""
    wc = ~ill
    n = ang.size
    stats["normal_boundary_frac"] = float(ill.mean()) if n else 0.0
    stats["normal_ok"] = float(np.mean(ang[wc] <= 1e-3)) if wc.any() else 1.0
    stats["normal_ang_p99"] = float(np.percentile(ang[wc], 99)) if wc.any() else 0.0
    stats["normal_ang_max"] = float(np.max(ang[wc])) if wc.any() else 0.0
    stats["normal_ok_conditioned"] = float(np.mean(ang <= np.maximum(1e-3, 10.0 * sens))) if n else 1.0
    if ill.any():
        q = np.percentile(ang[ill], [50, 99, 100])
        stats["normal_excluded_ang_p50"], stats["normal_excluded_ang_p99"], stats["normal_excluded_ang_max"] = map(float, q)
    else:
        stats["normal_excluded_ang_p50"] = stats["normal_excluded_ang_p99"] = stats["normal_excluded_ang_max"] = 0.0


def compare(orc, job, g, o, neigh_diff, pixels=None):
    """g: GPU frame (numpy, restricted to `pixels` if given); o: oracle render
    of the same pixels; neigh_diff: neighbour flags of those pixels."""
    cam, mc, fr = job["camera"], job["march"], job["fractal"]
    n = o["depth"].size
    if pixels is None:
        pixels = np.arange(n)
    gs, os_ = g["status"].astype(np.int64), o["status"].astype(np.int64)
    gc, oc = gs & CLS_MASK, os_ & CLS_MASK
    ghit, ohit = gc >= 2, oc >= 2
    stats = {"pixels": int(n), "hit_agree": float(np.mean(ghit == ohit)), "gpu_hits": int(ghit.sum()),
             "oracle_hits": int(ohit.sum())}
    orig, dirs = orc.camera_rays(cam, pixels)
    B = boundary_set(o, neigh_diff, dirs)
    on = o["normal"].T
    both = ghit & ohit & ~B
    stats["boundary_frac"] = float(B.mean())
    stats["compared"] = int(both.sum())
    stats["class_agree"] = float(np.mean(gc[both] == oc[both])) if both.any() else 1.0
    ts = o["depth"][both]
    eps = mc["eps_abs"] + mc["eps_rel"] * ts
    derr = np.abs(g["depth"][both] - ts)
    ok = derr <= 2 * eps
    other = np.zeros(ok.shape, bool)
    # a final bracket with several crossings of d - eps holds several correct
    # depths: there the GPU's depth must lie in the oracle's bracket
    stats["depth_multi_root"] = 0
    stats["depth_other_root"] = 0
    if both.any() and not ok.all():
        sel = np.nonzero(~ok)[0]
        lt, tt, cr = orc.bracket_crossings(job, pixels[both][sel])
        tg = g["depth"][both][sel].astype(np.float64)
        e2 = 2 * eps[sel]
        valid = (cr > 1) & (tg >= lt - e2) & (tg <= tt + e2)
        ok[sel[valid]] = True
        other[sel[valid]] = True
        stats["depth_multi_root"] = int(valid.sum())
        # another crossing of the eps-region that the oracle confirms as a root
        sel = np.nonzero(~ok)[0]
        if sel.size:
            pi = np.nonzero(both)[0][sel]
            tg = g["depth"][pi].astype(np.float64)
            eg = mc["eps_abs"] + mc["eps_rel"] * tg
            root = (gc[pi] == 2) & oracle_root_near(orc, job, orig[pi], dirs[pi], tg, 2.0 * eg)
            ok[sel[root]] = True
            other[sel[root]] = True
            stats["depth_other_root"] = int(root.sum())
    stats["depth_ok"] = float(np.mean(ok)) if both.any() else 1.0
    stats["depth_other_frac"] = float(stats["depth_other_root"] / both.sum()) if both.any() else 0.0
    stats["depth_err_max_over_eps"] = float(np.max(np.where(other, 0.0, derr) / eps)) if both.any() else 0.0
    # normal: oracle normal at the GPU's hit point (cut faces: the plane normal on both sides)
    gn = g["normal"].T[both]
    idx = np.nonzero(both)[0]
    p_g = orig[idx] + g["depth"][idx, None].astype(np.float64) * dirs[idx]
    eps_g = mc["eps_abs"] + mc["eps_rel"] * g["depth"][idx].astype(np.float64)
    n_at = orc.normal_at(fr, p_g, dirs[idx], eps_g, mc["normal_mode"])
    cut = gc[idx] == 3
    n_at[cut] = on[idx][cut]
    ang = angle(gn, n_at)
    ang_own = angle(gn, on[idx])
    sens, low = normal_sensitivity(orc, fr, mc, p_g, dirs[idx], eps_g)
    ill = (sens > 2e-4) | low
    ill[cut] = False
    sens[cut] = 0.0
    _normal_stats(stats, ang, sens, ill)
    # against the oracle's normal at its own hit point, where both sides found
    # the same root and the normal is well conditioned
    same = ~ill & ~other
    stats["normal_ok_vs_oracle_point"] = float(np.mean(ang_own[same] <= 1e-3)) if same.any() else 1.0
    stats["normal_bad_vs_oracle_point"] = int(np.sum(ang_own[same] > 1e-3))
    wc = ~ill
    # colour where the shadow outcome agrees and the normal is well
    # conditioned: against the oracle's shading of its normal at the GPU's
    # hit point (which separates the colour from the depth error, as for the
    # normal; error bounded by k_d |dN|), and, reported, against the oracle's
    # colour at its own hit point
    sv = wc & ((gs[idx] & 8) == (os_[idx] & 8))
    pv = idx[sv]
    if pv.size:
        ref = orc.shade_lambert(mc, n_at[sv], (os_[pv] & 8) != 0)
        cerr = np.abs(g["colour"][:, pv] - ref).max(0)
        cown = np.abs(g["colour"][:, pv] - o["colour"][:, pv]).max(0)
        same = ~other[sv]
        stats["colour_ok"] = float(np.mean(cerr <= 2e-3))
        stats["colour_err_max"] = float(cerr.max())
        stats["colour_ok_vs_oracle_point"] = float(np.mean(cown[same] <= 2e-3)) if same.any() else 1.0
    else:
        stats["colour_ok"], stats["colour_err_max"], stats["colour_ok_vs_oracle_point"] = 1.0, 0.0, 1.0
    stats["shadow_agree"] = float(np.mean((gs[both] & 8) == (os_[both] & 8))) if both.any() else 1.0
    # misses carry the miss encoding
    gm = ~ghit
    stats["miss_encoding_ok"] = bool(np.all(g["depth"][gm] == -1.0) and np.all(g["normal"][:, gm] == 0.0)
                                     and np.all(g["colour"][:, gm] == 0.0))
    return stats


def assert_parity(stats, hit_agree=0.999, depth_ok=1.0, normal_ok=0.999, class_agree=1.0, max_boundary=0.10,
                  max_normal_boundary=0.05, max_depth_other=0.002, normal_conditioned=0.995):
    """The bars of a comparison, with ceilings on every exclusion: the
    boundary set B (max_boundary of the compared pixels), the ill-conditioned
    normals (max_normal_boundary of the compared hits) and the depths
    accepted as another confirmed root (max_depth_other)."""
    msg = str(stats)
    assert stats["hit_agree"] >= hit_agree, msg
    assert stats["depth_ok"] >= depth_ok, msg
    assert stats["class_agree"] >= class_agree, msg
    assert stats["normal_ok"] >= normal_ok, msg
    assert stats["colour_ok"] >= normal_ok, msg
    assert stats["miss_encoding_ok"], msg
    assert stats["boundary_frac"] <= max_boundary, msg
    assert stats["normal_boundary_frac"] <= max_normal_boundary, msg
    # depths accepted as another root the oracle confirms: at most
    # max_depth_other of the compared hits (and at least one pixel allowed)
    assert stats.get("depth_other_root", 0) <= max(1, max_depth_other * stats["compared"]), msg
    assert stats["normal_ok_conditioned"] >= normal_conditioned, msg
    assert stats.get("colour_ok_vs_oracle_point", 1.0) >= 0.99, msg
    # the normal against the oracle's normal at its own hit point: at most
    # 1% of the well-conditioned normals (and never more than one pixel on
    # tiny images) beyond 1e-3 rad
    bad = stats.get("normal_bad_vs_oracle_point", 0)
    assert stats.get("normal_ok_vs_oracle_point", 1.0) >= 0.99 or bad <= 1, msg


def assert_aggregate_exclusions(stats_list, max_boundary, max_normal_boundary):
    """Ceilings on the exclusions summed over several comparisons (a batch
    whose single renders may be small or mostly chaotic): the boundary set
    over all compared pixels and the ill-conditioned normals over all
    compared hits."""
    pix = sum(st["pixels"] for st in stats_list)
    comp = sum(st["compared"] for st in stats_list)
    B = sum(st["boundary_frac"] * st["pixels"] for st in stats_list) / max(pix, 1)
    nB = sum(st["normal_boundary_frac"] * st["compared"] for st in stats_list) / max(comp, 1)
    print("aggregate over %d comparisons: boundary %.4f of %d pixels, ill-conditioned normals %.4f of %d hits"
          % (len(stats_list), B, pix, nB, comp))
    assert B <= max_boundary, (B, max_boundary)
    assert nB <= max_normal_boundary, (nB, max_normal_boundary)
    return B, nB


# ----------------------------------------------------------------- scenes
def id_neighbour_flags(id_img, status_img):
    """Per pixel: does any 8-neighbour show another object (or a miss), or
    differ in cut-face-ness?"""
    cut = (status_img & CLS_MASK) == 3
    H, W = id_img.shape
    diff = np.zeros((H, W), bool)
    ip = np.pad(id_img, 1, mode="edge")
    cp = np.pad(cut, 1, mode="edge")
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            diff |= (ip[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] != id_img)
            diff |= (cp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] != cut)
    return diff


# Normal tilt of the reflection-conditioning probe (rad): the bound on the
# FP64 normal's change under float32-sized input changes that separates the
# well-conditioned normals from the ill-conditioned ones.
REFLECT_TILT = 2e-4


def tilted_normals(nrm, tilt):
    """The unit normals [n, 3] tilted by `tilt` rad toward +-a and +-b, two
    unit vectors orthogonal to each normal and to each other."""
    nrm = np.asarray(nrm, np.float64)
    helper_axis = np.where(np.abs(nrm[:, :1]) < 0.9, [[1.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]])
    a = np.cross(nrm, helper_axis)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nrm, a)
    out = []
    for ax in (a, b):
        for sg in (1.0, -1.0):
            v = np.cos(tilt) * nrm + sg * np.sin(tilt) * ax
            out.append(v / np.linalg.norm(v, axis=1, keepdims=True))
    return out


def compare_scene(orc, sc, g, o, neigh_diff):
    """Scene parity (full image): object ids over every pixel; class, depth,
    normal and colour as in compare() on the pixels where both sides hit
    the same object and that lie outside B (with the object id in the
    neighbour rule), the normal rule evaluated in the object's own frame at
    the GPU's hit point and rotated back."""
    cam, mc = sc["camera"], sc["march"]
    n = o["depth"].size
    gid = g["object_id"].astype(np.int64)
    oid = o["object_id"].astype(np.int64)
    gs, os_ = g["status"].astype(np.int64), o["status"].astype(np.int64)
    gc, oc = gs & CLS_MASK, os_ & CLS_MASK
    stats = {"pixels": int(n), "id_agree": float(np.mean(gid == oid)),
             "hit_agree": float(np.mean((gid >= 0) == (oid >= 0))),
             "gpu_hits": int((gid >= 0).sum()), "oracle_hits": int((oid >= 0).sum())}
    orig, dirs = orc.camera_rays(cam, np.arange(n))
    B = boundary_set(o, neigh_diff, dirs)
    both = (gid == oid) & (gid >= 0) & ~B
    stats["boundary_frac"] = float(B.mean())
    stats["compared"] = int(both.sum())
    stats["class_agree"] = float(np.mean(gc[both] == oc[both])) if both.any() else 1.0
    idx = np.nonzero(both)[0]
    gd = g["depth"][idx].astype(np.float64)
    ts = o["depth"][idx]
    eps = mc["eps_abs"] + mc["eps_rel"] * ts
    derr = np.abs(gd - ts)
    ok = derr <= 2 * eps
    multi = np.zeros(ok.shape, bool)
    for k, ob in enumerate(sc["objects"]):
        sel = np.nonzero(~ok & (gid[idx] == k))[0]
        if sel.size == 0:
            continue
        R, T, s = orc.object_frame(ob)
        pi = idx[sel]
        r = orc.trace_rays(ob["fractal"], ob.get("planes", []), orc.object_march(mc, s), (orig[pi] - T) @ R / s,
                           dirs[pi] @ R, samples=256)
        lt, tt = r["lt"] * s, r["raw_t"] * s
        e2 = 2 * eps[sel]
        valid = (r["crossings"] > 1) & (lt >= 0) & (gd[sel] >= lt - e2) & (gd[sel] <= tt + e2)
        ok[sel[valid]] = True
        multi[sel[valid]] = True
    stats["depth_multi_root"] = int(multi.sum())
    # another crossing that the oracle confirms as a root, in the object's frame
    other = 0
    for k, ob in enumerate(sc["objects"]):
        sel = np.nonzero(~ok & (gid[idx] == k) & (gc[idx] == 2))[0]
        if sel.size == 0:
            continue
        R, T, s = orc.object_frame(ob)
        pi = idx[sel]
        objjob = {"fractal": ob["fractal"], "planes": ob.get("planes", []), "march": orc.object_march(mc, s)}
        eg = mc["eps_abs"] + mc["eps_rel"] * gd[sel]
        root = oracle_root_near(orc, objjob, (orig[pi] - T) @ R / s, dirs[pi] @ R, gd[sel] / s, 2.0 * eg / s)
        ok[sel[root]] = True
        multi[sel[root]] = True
        other += int(root.sum())
    stats["depth_other_root"] = other
    stats["depth_other_frac"] = float(other / idx.size) if idx.size else 0.0
    stats["depth_ok"] = float(np.mean(ok)) if idx.size else 1.0
    stats["depth_err_max_over_eps"] = float(np.max(np.where(multi, 0.0, derr) / eps)) if idx.size else 0.0
    # normals in each object's frame at the GPU's hit point
    n_at = np.zeros((idx.size, 3))
    ill = np.zeros(idx.size, bool)
    sens = np.zeros(idx.size)
    cut = gc[idx] == 3
    on = o["normal"].T
    for k, ob in enumerate(sc["objects"]):
        sel = np.nonzero((gid[idx] == k) & ~cut)[0]
        if sel.size == 0:
            continue
        R, T, s = orc.object_frame(ob)
        pi = idx[sel]
        p_w = orig[pi] + gd[sel, None] * dirs[pi]
        p_o = (p_w - T) @ R / s
        d_o = dirs[pi] @ R
        e_o = (mc["eps_abs"] + mc["eps_rel"] * gd[sel]) / s
        n_at[sel] = orc.normal_at(ob["fractal"], p_o, d_o, e_o, mc["normal_mode"]) @ R.T
        se, lo = normal_sensitivity(orc, ob["fractal"], mc, p_o, d_o, e_o)
        sens[sel] = se
        ill[sel] = (se > 2e-4) | lo
    n_at[cut] = on[idx][cut]
    gn = g["normal"].T[idx]
    ang = angle(gn, n_at) if idx.size else np.zeros(0)
    _normal_stats(stats, ang, sens, ill)
    wc = ~ill
    # with trap colouring the albedo follows the orbit trap of the hit point:
    # colour is compared where that trap is well conditioned too
    pal = np.asarray(mc.get("trap_colour", [[0.0] * 3] * 4), np.float64)
    if mc.get("shading", "lambert") == "phong" and np.any(pal != 0.0):
        tri = np.zeros(idx.size, bool)
        for k, ob in enumerate(sc["objects"]):
            sel = np.nonzero(gid[idx] == k)[0]
            if sel.size == 0:
                continue
            R, T, s = orc.object_frame(ob)
            pi = idx[sel]
            tri[sel] = trap_ill_conditioned(orc, ob["fractal"], (orig[pi] + gd[sel, None] * dirs[pi] - T) @ R / s)
        stats["trap_boundary_frac"] = float(tri.mean()) if idx.size else 0.0
        wc = wc & ~tri
    # colour where the shadow outcome agrees and normal (and trap) are well
    # conditioned: against the oracle's shading at the GPU's hit point (its
    # normal and trap there, and with the closest-hit shading the reflection
    # bounce from there), which separates the colour from the depth error as
    # for the normal, on the pixels whose reflected ray hits or misses on
    # both sides; the colour against the oracle's own hit point is reported
    # and held to 99% agreement
    sv = wc & ((gs[idx] & 8) == (os_[idx] & 8))
    pv = idx[sv]
    if pv.size:
        p_w = orig[pv] + gd[sv, None] * dirs[pv]
        eps_g = mc["eps_abs"] + mc["eps_rel"] * gd[sv]
        vis = np.where((os_[pv] & 8) != 0, 0.0, 1.0)
        ref, _, rhit = orc.shade_hits(sc, gid[pv], p_w, dirs[pv], n_at[sv], vis, eps_g)
        rsame = rhit == ((gs[pv] & 128) != 0)
        stats["reflect_agree_at_gpu_point"] = float(rsame.mean())
        if mc.get("shading", "lambert") == "phong" and float(mc.get("k_reflect", 0.0)) > 0.0:
            # the reflected ray amplifies the normal's error: its share is
            # compared where tilting the normal by REFLECT_TILT moves the
            # colour by less than 1e-3 and keeps the reflected hit/miss
            rill = np.zeros(pv.size, bool)
            for nv in tilted_normals(n_at[sv], REFLECT_TILT):
                c2, _, rh2 = orc.shade_hits(sc, gid[pv], p_w, dirs[pv], nv, vis, eps_g)
                rill |= (np.abs(c2 - ref).max(0) > 1e-3) | (rh2 != rhit)
            stats["reflect_ill_frac"] = float(rill.mean())
            rsame &= ~rill
        cerr = np.abs(g["colour"][:, pv] - ref).max(0)[rsame]
        stats["colour_compared"] = int(rsame.sum())
        stats["colour_ok"] = float(np.mean(cerr <= 2e-3)) if cerr.size else 1.0
        stats["colour_err_max"] = float(cerr.max()) if cerr.size else 0.0
        own = (gs[pv] & 128) == (os_[pv] & 128)
        cown = np.abs(g["colour"][:, pv] - o["colour"][:, pv]).max(0)[own]
        stats["colour_ok_vs_oracle_point"] = float(np.mean(cown <= 2e-3)) if cown.size else 1.0
    else:
        stats["colour_compared"] = 0
        stats["colour_ok"], stats["colour_err_max"], stats["colour_ok_vs_oracle_point"] = 1.0, 0.0, 1.0
        stats["reflect_agree_at_gpu_point"] = 1.0
    stats["shadow_agree"] = float(np.mean((gs[both] & 8) == (os_[both] & 8))) if both.any() else 1.0
    stats["reflect_agree"] = float(np.mean((gs[both] & 128) == (os_[both] & 128))) if both.any() else 1.0
    gm = gid < 0
    stats["miss_encoding_ok"] = bool(np.all(g["depth"][gm] == -1.0) and np.all(g["normal"][:, gm] == 0.0)
                                     and np.all(g["colour"][:, gm] == 0.0))
    return stats


def assert_scene_parity(stats, id_agree=0.999, normal_ok=0.999, colour_ok=None, reflect_agree=0.995,
                        max_boundary=0.10, max_normal_boundary=0.05, max_depth_other=0.002,
                        normal_conditioned=0.995, max_trap_boundary=0.2, max_reflect_ill=0.1):
    msg = str(stats)
    assert stats.get("reflect_ill_frac", 0.0) <= max_reflect_ill, msg
    assert stats.get("reflect_agree_at_gpu_point", 1.0) >= reflect_agree, msg
    assert stats["boundary_frac"] <= max_boundary, msg
    assert stats["normal_boundary_frac"] <= max_normal_boundary, msg
    assert stats["depth_other_root"] <= max(1, max_depth_other * stats["compared"]), msg
    assert stats["normal_ok_conditioned"] >= normal_conditioned, msg
    assert stats.get("trap_boundary_frac", 0.0) <= max_trap_boundary, msg
    assert stats["reflect_agree"] >= reflect_agree, msg
    assert stats["id_agree"] >= id_agree, msg
    assert stats["hit_agree"] >= id_agree, msg
    assert stats["depth_ok"] >= 1.0, msg
    assert stats["class_agree"] >= 1.0, msg
    assert stats["normal_ok"] >= normal_ok, msg
    assert stats["colour_ok"] >= (normal_ok if colour_ok is None else colour_ok), msg
    assert stats.get("colour_ok_vs_oracle_point", 1.0) >= 0.99, msg
    assert stats["miss_encoding_ok"], msg
