"""Oracle pins for the residual estimator (Sec. 3-5 of the paper).

Each check is fixed by something other than the oracle's own formulas: an
exact zero, a closed form, an independent float64 quadrature, the difference
of two independently rendered frames, or agreement between different
strategy subsets (each subset is an unbiased estimator of the same residual
only if every technique's pdf is right)."""
import math

import numpy as np
import pytest

from paper_2406_16302_amd import scenes

T = 8  # oracle threads


def batched(fn, seeds):
    xs = np.array([fn(s) for s in seeds])
    return xs.mean(0), xs.std(0, ddof=1) / math.sqrt(len(seeds))


def zscores(a, sa, b, sb):
    sig = np.sqrt(sa ** 2 + sb ** 2)
    m = sig > 0
    return (a - b)[m] / sig[m], m


# --- exact zeros ------------------------------------------------------------

def test_identity_motion_edit_is_exactly_zero(oracle_lib):
    w = scenes.cornell_motion(width=16, height=16, depth=5)
    o = oracle_lib.OracleScene(w.scene)
    r = o.render_residual(4, 5, 3, pose_new=oracle_lib.IDENTITY, threads=T)
    assert r["stats"]["paths"] > 1000
    assert np.count_nonzero(r["image"]) == 0
    assert r["stats"]["accepted"] == r["stats"]["paths"]


def test_identity_material_edit_is_exactly_zero(oracle_lib):
    w = scenes.cornell_material(width=16, height=16, depth=5)
    o = oracle_lib.OracleScene(w.scene)
    same = w.scene.materials[4]
    r = o.render_residual(4, 5, 3, material_mode=True, new_mat=same, mask=0x07, two_way=False, threads=T)
    assert r["stats"]["paths"] > 1000
    assert np.count_nonzero(r["image"]) == 0


# --- closed form --------------------------------------------------------------

def test_white_furnace_material_edit_closed_form(oracle_lib):
    """Convex Lambertian sphere in a closed non-reflective L_e = 1 enclosure:
    the sphere's outgoing radiance is its albedo, so a 0.5 -> 0.8 edit adds
    exactly 0.3 to fully covered pixels and nothing elsewhere."""
    w = scenes.furnace(width=24, height=24)
    sc = w.scene
    o = oracle_lib.OracleScene(sc)
    R, se = batched(lambda s: oracle_lib.residual_for(w, o, spp=8, depth=3, seed=s, threads=T)["image"],
                    range(100, 116))
    # inscribed radius of the icosphere and pixel-corner coverage (independent geometry)
    obj = sc.tri_object == 1
    tri = sc.positions[sc.indices[obj]].astype(np.float64)
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = np.abs((nrm * tri[:, 0]).sum(1)).min()
    eye = sc.camera[:3].astype(np.float64)
    dist = np.linalg.norm(eye)
    half = math.asin(r_in / dist)
    th = math.tan(math.radians(sc.camera[9]) / 2)
    W, H = sc.width, sc.height
    covered = np.zeros((H, W), bool)
    empty = np.zeros((H, W), bool)
    r_out = np.linalg.norm(sc.positions[np.unique(sc.indices[obj])], axis=1).max()
    half_out = math.asin(r_out / dist)
    for py in range(H):
        for px in range(W):
            angs = []
            for cy in (0, 1):
                for cx in (0, 1):
                    sx = (2 * (px + cx) / W - 1) * th
                    sy = (1 - 2 * (py + cy) / H) * th
                    angs.append(math.atan(math.hypot(sx, sy)))
            covered[py, px] = max(angs) < half
            empty[py, px] = min(angs) > half_out
    assert covered.sum() > 50 and empty.sum() > 50
    z = (R[covered] - 0.3) / np.maximum(se[covered], 1e-12)
    assert (np.abs(z) < 3.5).mean() > 0.98
    m = R[covered].mean()
    assert abs(m - 0.3) < 3 * np.sqrt((se[covered] ** 2).sum()) / covered.sum() + 1e-9
    assert np.count_nonzero(R[empty]) == 0


# --- generation densities equal the MIS strategy terms --------------------------

@pytest.mark.parametrize("depth", [3, 5])
def test_generation_pdf_equals_mis_term(oracle_lib, depth):
    cases = [(scenes.cornell_motion(width=16, height=16, depth=depth), (1, 2, 3, 5, 6, 7)),
             (scenes.ghost_plane(open_object=True), (4, 5, 6)),
             (scenes.cornell_material(width=16, height=16, depth=depth), (1, 2, 3))]  # GGX object
    for w, techs in cases:
        o = oracle_lib.OracleScene(w.scene)
        if w.edit.kind == scenes.EDIT_MATERIAL:
            r = o.render_residual(4, depth, 7, material_mode=True, new_mat=w.edit.new_material, mask=0x07,
                                  two_way=False, records=True)
        else:
            r = o.render_residual(4, depth, 7, pose_new=w.edit.old_to_new, records=True)
        rec = r["records"]
        assert (rec["p_gen"] <= rec["mis_tech"] * (1 + 1e-5)).all()
        for t in techs:
            s = rec[(rec["tech"] == t) & (rec["n_starts"] == 1)]
            if t == 3 and depth < 5:
                continue
            assert len(s) > 10, (w.name, t)
            rel = np.abs(s["p_gen"] / s["mis_tech"] - 1)
            assert np.quantile(rel, 0.99) < 1e-5 and rel.max() < 1e-3, (w.name, t, rel.max())


# --- technique subsets estimate the same residual --------------------------------

def test_technique_subsets_agree(oracle_lib):
    d = 5
    w = scenes.cornell_motion(width=8, height=8, depth=d)
    o = oracle_lib.OracleScene(w.scene)

    def est(mask, base, spp=48, B=16):
        return batched(lambda s: o.render_residual(spp, d, s, pose_new=w.edit.old_to_new, mask=mask,
                                                   threads=T)["image"], range(base, base + B))

    ref, rse = est(0x7F, 1000)
    for k, mask in enumerate([0x41, 0x42, 0x44, 0x48, 0x50, 0x60, 0x40]):
        R, se = est(mask, 2000 + 100 * k)
        z, _ = zscores(R, se, ref, rse)
        assert (np.abs(z) < 3).mean() > 0.97, hex(mask)
        zm = (R.mean() - ref.mean()) / (np.sqrt((se ** 2).sum() + (rse ** 2).sum()) / R.size)
        assert abs(zm) < 3.5, (hex(mask), zm)


def test_mapping_is_an_involution_with_symmetric_rejection(oracle_lib):
    for d in (3, 5):
        w = scenes.cornell_motion(width=16, height=16, depth=d)
        o = oracle_lib.OracleScene(w.scene)
        c = oracle_lib.map_check(o, w.edit.old_to_new, 4, d, 3)
        assert c["checked"] > 1000
        assert c["accept_mismatch"] == 0 and c["roundtrip_mismatch"] == 0
    w = scenes.ghost_plane()
    c = oracle_lib.map_check(oracle_lib.OracleScene(w.scene), w.edit.old_to_new, 16, 4, 3)
    assert c["checked"] > 1000 and c["accept_mismatch"] == 0 and c["roundtrip_mismatch"] == 0


# --- unbiasedness against the difference of two independent frames -------------

@pytest.mark.parametrize("kind", ["motion", "material", "motion_no_mapping", "motion_unequal_counts",
                                  "material_unequal_counts", "motion_balance"])
def test_residual_converges_to_frame_difference(oracle_lib, kind):
    """motion_no_mapping: the path-mapping ablation (every pair rejected,
    each frame's dynamic paths with weight 1) is also unbiased.
    *_unequal_counts: techniques with different sample counts, combined by
    the balance heuristic over those counts, stay unbiased.
    motion_balance: accepted pairs weighted by the balance heuristic over the
    strategies of both directions instead of c = 1/2."""
    counts = [512, 128, 256, 384, 128, 256, 64, 0] if kind.endswith("unequal_counts") else None
    if kind.startswith("motion"):
        w = scenes.cornell_motion(width=8, height=8, depth=4)
        frame_kw = dict(pose_new=w.edit.old_to_new)
        res_kw = dict(pose_new=w.edit.old_to_new, no_mapping=kind.endswith("no_mapping"), tech_spp=counts,
                      balance=kind.endswith("balance"))
    else:
        w = scenes.cornell_material(width=8, height=8, depth=4)
        frame_kw = dict(new_mat=w.edit.new_material)
        res_kw = dict(new_mat=w.edit.new_material, material_mode=True, mask=0x07, two_way=False, tech_spp=counts)
    d = w.depth
    o = oracle_lib.OracleScene(w.scene)
    D, dse = batched(lambda s: o.render_frame(2, 4096, d, s, threads=T, **frame_kw)[0]
                     - o.render_frame(1, 4096, d, s + 777, threads=T, **frame_kw)[0], range(10, 34))
    R, se = batched(lambda s: o.render_residual(256, d, s, threads=T, **res_kw)["image"], range(500, 524))
    if kind == "motion_no_mapping":
        st = o.render_residual(16, d, 1, threads=T, **res_kw)["stats"]
        assert st["paths"] > 0 and st["accepted"] == 0 and st["unmapped"] == st["paths"]
    z, _ = zscores(R, se, D, dse)
    # the three channels of a pixel share their paths, so values beyond 3
    # sigma come in threes: allow one such pixel of the 64
    assert (np.abs(z) < 3).mean() > 0.98 - (0.01 if counts else 0.0)
    assert np.abs(z).max() < 5.5
    zm = (R.mean() - D.mean()) / (np.sqrt((se ** 2).sum() + (dse ** 2).sum()) / R.size)
    assert abs(zm) < 3.5


# --- depth-2 paths against a deterministic quadrature ------------------------------

def _np_hit(tris, o, d, tmin=1e-7, tmax=None):
    v0, e1, e2 = tris[:, 0], tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]
    p = np.cross(d[:, None, :], e2[None])
    det = (e1[None] * p).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o[:, None, :] - v0[None]
        u = (s * p).sum(-1) * inv
        q = np.cross(s, e1[None])
        v = (d[:, None, :] * q).sum(-1) * inv
        t = (e2[None] * q).sum(-1) * inv
    ok = (det != 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > tmin)
    if tmax is not None:
        ok &= t < tmax[:, None]
    return np.where(ok, t, np.inf)


def _quadrature_frame(sc, pose, nsub, nl):
    """E x L paths of a Lambertian scene with one quad light, by midpoint rules
    over sub-pixels and light points (float64, exact visibility)."""
    pos = sc.positions.astype(np.float64)
    tris = pos[sc.indices]
    obj = sc.tri_object == 1
    R = np.array(pose, np.float64).reshape(3, 4)
    tris = tris.copy()
    tris[obj] = tris[obj] @ R[:, :3].T + R[:, 3]
    mats = sc.materials
    emit = mats[sc.tri_material, 0] == 2
    nrm = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    lt = tris[emit]
    lo, hi = lt.reshape(-1, 3).min(0), lt.reshape(-1, 3).max(0)
    ly = lo[1]
    lnorm = nrm[emit][0]
    Le = mats[sc.tri_material[emit][0], 5:8]
    g = (np.arange(nl) + 0.5) / nl
    LX, LZ = np.meshgrid(lo[0] + g * (hi[0] - lo[0]), lo[2] + g * (hi[2] - lo[2]), indexing="ij")
    lpts = np.stack([LX.ravel(), np.full(LX.size, ly), LZ.ravel()], 1)
    dA = (hi[0] - lo[0]) * (hi[2] - lo[2]) / lpts.shape[0]
    eye = sc.camera[:3].astype(np.float64)
    tgt = sc.camera[3:6].astype(np.float64)
    up = sc.camera[6:9].astype(np.float64)
    fwd = (tgt - eye) / np.linalg.norm(tgt - eye)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    cup = np.cross(right, fwd)
    th = math.tan(math.radians(sc.camera[9]) / 2)
    W, H = sc.width, sc.height
    s = (np.arange(nsub) + 0.5) / nsub
    img = np.zeros((H, W, 3))
    for py in range(H):
        # film points: pixel column, sub-row, sub-column -> (W, nsub, nsub)
        px = np.arange(W)[:, None, None] + s[None, None, :]
        sy = py + s[None, :, None]
        fx = (2 * px / W - 1) * th * (W / H) + 0 * sy
        fy = (1 - 2 * sy / H) * th + 0 * px
        dirs = fwd + fx[..., None] * right + fy[..., None] * cup
        dirs = dirs.reshape(-1, 3)
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        o = np.repeat(eye[None], len(dirs), 0)
        t = _np_hit(tris, o, dirs)
        ti = t.argmin(1)
        tt = t[np.arange(len(t)), ti]
        rad = np.zeros((len(dirs), 3))
        hit = np.isfinite(tt)
        xp = o + dirs * tt[:, None]
        with np.errstate(invalid="ignore"):
            nf = nrm[ti] * np.sign(((eye - xp) * nrm[ti]).sum(1))[:, None]
        lit = hit & emit[ti]
        rad[lit] = Le * (((eye - xp[lit]) * nrm[ti[lit]]).sum(1) > 0)[:, None]
        surf = np.nonzero(hit & ~emit[ti])[0]
        occ = tris[~emit]
        for c0 in range(0, len(surf), 256):
            ks = surf[c0:c0 + 256]
            to = lpts[None] - xp[ks][:, None]                     # (n, L, 3)
            r2 = (to ** 2).sum(-1)
            wl = to / np.sqrt(r2)[..., None]
            cx = (wl * nf[ks][:, None]).sum(-1)
            cl = -(wl @ lnorm)
            so = (xp[ks] + 1e-7 * nf[ks])[:, None].repeat(len(lpts), 1).reshape(-1, 3)
            tv = _np_hit(occ, so, to.reshape(-1, 3), tmax=np.full(len(so), 1 - 1e-6))
            vis = ~np.isfinite(tv.min(1)).reshape(len(ks), -1)
            g = np.where((cx > 0) & (cl > 0) & vis, cx * cl / r2, 0.0).sum(1) * dA
            albedo = mats[sc.tri_material[ti[ks]], 1:4]
            rad[ks] = albedo / math.pi * Le[None] * g[:, None]
        img[py] = rad.reshape(W, nsub * nsub, 3).mean(1)
    return img


def test_depth2_residual_matches_quadrature(oracle_lib):
    w = scenes.cornell_motion(width=8, height=8, depth=2)
    sc = w.scene
    o = oracle_lib.OracleScene(sc)
    R, se = batched(lambda s: o.render_residual(256, 2, s, pose_new=w.edit.old_to_new, threads=T)["image"],
                    range(40, 56))
    q2f = _quadrature_frame(sc, w.edit.old_to_new, 8, 8)
    q1f = _quadrature_frame(sc, oracle_lib.IDENTITY, 8, 8)
    q2c = _quadrature_frame(sc, w.edit.old_to_new, 4, 4)
    q1c = _quadrature_frame(sc, oracle_lib.IDENTITY, 4, 4)
    q_f, q_c = q2f - q1f, q2c - q1c
    qerr = np.abs(q_f - q_c)
    dev = np.abs(R - q_f)
    assert (dev <= 3 * se + qerr + 1e-7).mean() > 0.95
    tot_sig = np.sqrt((se ** 2).sum()) + qerr.sum()
    assert abs(R.sum() - q_f.sum()) < 3 * tot_sig
    # the frame renderer against the same quadrature
    F2, fse = batched(lambda s: o.render_frame(2, 1024, 2, s, pose_new=w.edit.old_to_new, threads=T)[0],
                      range(60, 68))
    ferr = np.abs(q2f - q2c)
    assert (np.abs(F2 - q2f) <= 3 * fse + ferr + 1e-7).mean() > 0.95


# --- every strategy's MIS term integrates to what the strategy generates -------

@pytest.fixture(scope="module")
def sphere_records(oracle_lib):
    """Per-path records and per-technique images of all seven techniques on
    the clutter scene's moving sphere (16x16, depth 5, one direction)."""
    from concurrent.futures import ThreadPoolExecutor
    w = scenes.clutter_motion(width=16, height=16, depth=5, n_spheres=0)
    o = oracle_lib.OracleScene(w.scene)
    spp = 16384
    N = spp * 16 * 16
    parts = 8

    def part(k):  # per-path records need the single-threaded oracle: one call per sample range
        r = o.render_residual(spp, 5, 11, pose_new=w.edit.old_to_new, mask=0x7F, records=True, two_way=False,
                              rec_cap=20_000_000, threads=1, s0=N * k // parts, s1=N * (k + 1) // parts,
                              per_tech=True)
        return r["records"], r["per_tech"]

    with ThreadPoolExecutor(parts) as ex:
        res = list(ex.map(part, range(parts)))
    return {"N": N, "records": np.concatenate([r for r, _ in res]), "per_tech": sum(t for _, t in res)}


def test_strategy_terms_integrate_to_generated_paths(sphere_records):
    """Path tracing (7) reaches every dynamic path, so summing another
    strategy's MIS term over technique-7 paths, each divided by its
    technique-7 density, estimates how many paths that strategy generates per
    sample; it must match the count the strategy actually produces.  A term
    that counts configurations its sampler cannot reach (e.g. a ghost crossing
    the generating line misses) shows up as a ratio above one.  The scene is
    the clutter scene's moving sphere, whose ghost meets the object at an
    angle.  Every technique 1-6 is checked to three standard errors of the
    technique-7 estimate (per-sample grouping), and the sample is large enough
    that three standard errors stay below 10 %, so a 15 % error in any term
    fails."""
    N, rec = sphere_records["N"], sphere_records["records"]
    r7 = rec[rec["tech"] == 7]
    smp = r7["sample"].astype(np.int64)
    for t in (1, 2, 3, 4, 5, 6):
        direct = (rec["tech"] == t).sum() / N
        x = r7["mis_by_tech"][:, t] / r7["p_gen"]
        est = x.sum() / N
        se = np.bincount(smp, weights=x, minlength=N).std() / math.sqrt(N)
        print("technique %d: %.4f paths/sample, %.4f +- %.4f through technique 7" % (t, direct, est, se))
        assert direct > 0.01
        assert 3 * se / direct < 0.1, (t, se / direct)
        assert abs(est / direct - 1) < 3 * se / direct, (t, direct, est, se)


def test_per_technique_images_carry_their_mis_share(sphere_records):
    """The per-technique images (the decomposition of fig. importance_sample)
    hold each strategy's balance-heuristic share of the residual: technique
    t's image integrates g p_t, where g is the MIS-weighted path value, and
    the technique-7 paths estimate the same integral as the sum of g p_t / p_7.
    Checked on the image total of |g| (no cancellation between signs) to three
    standard errors; each per-technique image also equals the sum of its own
    records."""
    N, rec, pt = sphere_records["N"], sphere_records["records"], sphere_records["per_tech"]
    r7 = rec[rec["tech"] == 7]
    smp = r7["sample"].astype(np.int64)
    a7 = np.abs(r7["val"]).sum(1)
    for t in range(1, 8):
        rt = rec[rec["tech"] == t]
        img = np.zeros_like(pt[t - 1]).reshape(-1, 3)
        np.add.at(img, rt["pixel"], rt["val"])
        assert np.allclose(img.reshape(pt[t - 1].shape), pt[t - 1], rtol=1e-9, atol=1e-15), t
        direct = np.abs(rt["val"]).sum()
        x = a7 * r7["mis_by_tech"][:, t] / r7["mis_by_tech"][:, 7]
        est = x.sum()
        se = np.bincount(smp, weights=x, minlength=N).std() * math.sqrt(N)
        print("technique %d: sum |g| %.5g, %.5g +- %.3g through technique 7" % (t, direct, est, se))
        assert abs(est - direct) < 3 * se + 1e-12 * direct, (t, direct, est, se)
        if t != 7:
            assert 3 * se / direct < 0.15, (t, se / direct)


# --- the path-tracing baselines (correlated and from scratch) -----------------

def test_correlated_frames_cancel_off_the_edit_and_lower_the_variance(oracle_lib):
    """Correlated path tracing (both frames on the same random numbers)
    cancels exactly wherever a sample's path misses the object in both
    poses, and so has a far smaller variance than two independent frames;
    both are unbiased estimates of the same difference."""
    w = scenes.cornell_motion(width=8, height=8, depth=4)
    o = oracle_lib.OracleScene(w.scene)
    kw = dict(pose_new=w.edit.old_to_new, threads=T)

    def diff(seed, correlated):
        a = o.render_frame(2, 64, 4, seed, stream_dir=0, **kw)[0]
        b = o.render_frame(1, 64, 4, seed, stream_dir=0 if correlated else 1, **kw)[0]
        return a - b
    same = o.render_frame(2, 16, 4, 5, stream_dir=0, pose_new=oracle_lib.IDENTITY, threads=T)[0] - \
        o.render_frame(1, 16, 4, 5, stream_dir=0, threads=T)[0]
    assert np.count_nonzero(same) == 0
    C, cse = batched(lambda s: diff(s, True), range(30, 46))
    I, ise = batched(lambda s: diff(s, False), range(30, 46))
    z, _ = zscores(C, cse, I, ise)
    assert (np.abs(z) < 3).mean() > 0.95
    assert (cse ** 2).sum() < 0.5 * (ise ** 2).sum()
