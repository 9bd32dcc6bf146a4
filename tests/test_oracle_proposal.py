"""Oracle pins for the learned proposal (technique 8): vMF mixture
normalisation and sampling, back-propagation against finite differences,
generation density == MIS term, and unbiasedness with the extra strategy."""
import math

import numpy as np

from paper_2406_16302_amd import scenes


def _raw(rng, kappa_scale=3.0):
    raw = rng.normal(size=40)
    for l in range(8):
        raw[5 * l + 3] = rng.uniform(-2, kappa_scale)
    return raw


def test_vmf_lobes_integrate_to_one(oracle_lib):
    rng = np.random.default_rng(0)
    raw = _raw(rng, kappa_scale=6.0)
    # quadrature in (cos theta, phi) over the whole sphere, fine enough for kappa <= ~400
    n = 800
    ct = -1 + (np.arange(n) + 0.5) * 2 / n
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi
    C, P = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - C ** 2)
    w = np.stack([S * np.cos(P), S * np.sin(P), C], -1).reshape(-1, 3)
    dw = (2.0 / n) * (2 * math.pi / (2 * n))
    tot = sum(oracle_lib.vmf_pdf(raw, x) for x in w[::7]) * dw * 7
    assert abs(tot - 1.0) < 5e-3


def test_vmf_sampling_matches_pdf(oracle_lib):
    rng = np.random.default_rng(1)
    raw = np.zeros(40)
    raw[0:3] = [0.3, -0.2, 0.9]
    raw[3] = 1.5  # kappa ~ 1.7
    for l in range(1, 8):
        raw[5 * l + 4] = -30.0  # one effective lobe
    mu = raw[0:3] / np.linalg.norm(raw[0:3])
    us = rng.random((40000, 3)).astype(np.float32)
    c = np.array([oracle_lib.vmf_sample(raw, *u) @ mu for u in us])
    bins = np.linspace(-1, 1, 21)
    h, _ = np.histogram(c, bins)
    # expected bin mass of cos(theta) from the pdf by quadrature along theta
    exp = []
    for a, b in zip(bins[:-1], bins[1:]):
        xs = np.linspace(a, b, 41)
        t = np.cross(mu, [1, 0, 0])
        t /= np.linalg.norm(t)
        vals = [oracle_lib.vmf_pdf(raw, x * mu + math.sqrt(max(0, 1 - x * x)) * t) for x in xs]
        exp.append(np.trapezoid(vals, xs) * 2 * math.pi * len(c))
    exp = np.array(exp)
    m = exp > 20
    chi2 = ((h[m] - exp[m]) ** 2 / exp[m]).sum()
    assert chi2 < 45.0, chi2


def test_vmf_sampling_at_the_end_of_the_unit_interval(oracle_lib):
    """u1 = 0 on a lobe so sharp that e^{-2 kappa} is below the float range:
    the inversion's argument is 0 and its limit is c = -1, the antipode of
    the mean (not a NaN direction); u1 near 1 gives the mean itself."""
    raw = np.zeros(40)
    raw[0:3] = [0.3, -0.2, 0.9]
    raw[3] = 1e4  # kappa clamped at 1e4
    for l in range(1, 8):
        raw[5 * l + 4] = -30.0
    mu = raw[0:3] / np.linalg.norm(raw[0:3])
    for u2 in (0.0, 0.37):
        w = np.asarray(oracle_lib.vmf_sample(raw, 0.1, 0.0, u2))
        assert np.all(np.isfinite(w)), w
        assert abs(w @ mu + 1.0) < 1e-5, w @ mu
        w = np.asarray(oracle_lib.vmf_sample(raw, 0.1, np.float32(1.0 - 2 ** -24), u2))
        assert w @ mu > 1.0 - 1e-5


def test_backprop_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(2)
    P = oracle_lib.mlp_init(3)
    rec = np.zeros((24, 10), np.float32)
    rec[:, 0:3] = rng.uniform(-1, 1, (24, 3))
    n = rng.normal(size=(24, 3))
    rec[:, 3:6] = n / np.linalg.norm(n, axis=1, keepdims=True)
    w = rng.normal(size=(24, 3))
    rec[:, 6:9] = w / np.linalg.norm(w, axis=1, keepdims=True)
    rec[:, 9] = rng.uniform(0.1, 2.0, 24)
    loss, g = oracle_lib.mlp_loss_grad(P, rec, bf16=False)
    idx = rng.choice(P.size, 60, replace=False)
    num = []
    for i in idx:
        h = 1e-3 * max(1.0, abs(float(P[i])))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += np.float32(h)
        Pm[i] -= np.float32(h)
        hp = float(Pp[i]) - float(P[i])
        hm = float(P[i]) - float(Pm[i])
        lp, _ = oracle_lib.mlp_loss_grad(Pp, rec, bf16=False)
        lm, _ = oracle_lib.mlp_loss_grad(Pm, rec, bf16=False)
        num.append((lp - lm) / (hp + hm))
    num = np.array(num)
    err = np.linalg.norm(num - g[idx]) / np.linalg.norm(g[idx])
    assert err < 1e-3, err


def test_technique8_generation_density_equals_mis_term(oracle_lib):
    w = scenes.cornell_material(width=16, height=16, depth=5)
    o = oracle_lib.OracleScene(w.scene)
    P = oracle_lib.mlp_init(5)
    r = o.render_residual(8, 5, 3, material_mode=True, new_mat=w.edit.new_material, mask=0x87, two_way=False,
                          records=True, mlp=P)
    rec = r["records"]
    s = rec[(rec["tech"] == 8) & (rec["n_starts"] == 1)]
    assert len(s) > 50
    # both sensor sides occur: the camera sees x_D (i = -1) and eye walks (i >= 0)
    assert ((s["pair"] >> 4) == 0).sum() > 20 and ((s["pair"] >> 4) > 0).sum() > 20
    rel = np.abs(s["p_gen"] / s["mis_tech"] - 1)
    assert np.quantile(rel, 0.99) < 1e-4 and rel.max() < 1e-2, rel.max()
    assert (rec["p_gen"] <= rec["mis_tech"] * (1 + 1e-4)).all()


def test_technique8_keeps_the_estimator_unbiased(oracle_lib):
    w = scenes.cornell_material(width=8, height=8, depth=5)
    o = oracle_lib.OracleScene(w.scene)
    P = oracle_lib.mlp_init(7)
    kw = dict(material_mode=True, new_mat=w.edit.new_material, two_way=False, threads=8)
    A = np.array([o.render_residual(48, 5, s, mask=0x07, **kw)["image"] for s in range(100, 116)])
    B = np.array([o.render_residual(48, 5, s, mask=0x87, mlp=P, **kw)["image"] for s in range(200, 216)])
    ma, mb = A.mean(0), B.mean(0)
    sa, sb = A.std(0, ddof=1) / 4, B.std(0, ddof=1) / 4
    sig = np.sqrt(sa ** 2 + sb ** 2)
    m = sig > 0
    z = (ma - mb)[m] / sig[m]
    assert (np.abs(z) < 3).mean() > 0.97
    zm = (ma.mean() - mb.mean()) / (np.sqrt((sa ** 2).sum() + (sb ** 2).sum()) / ma.size)
    assert abs(zm) < 3.5


def test_technique8_alone_stays_unbiased_with_sharp_lobes(oracle_lib):
    # Technique 8 in place of techniques 2 and 3: its defensive uniform-sphere
    # component must cover the directions that sharp lobes (kappa ~ 200) never
    # reach in fp32 sampling.
    w = scenes.cornell_material(width=8, height=8, depth=5)
    o = oracle_lib.OracleScene(w.scene)
    P = oracle_lib.mlp_init(7)
    for lobe in range(8):
        P[11328 + 5 * lobe + 3] = 200.0
    kw = dict(material_mode=True, new_mat=w.edit.new_material, two_way=False, threads=8)
    A = np.array([o.render_residual(48, 5, s, mask=0x07, **kw)["image"] for s in range(300, 316)])
    B = np.array([o.render_residual(48, 5, s, mask=0x81, mlp=P, **kw)["image"] for s in range(400, 416)])
    ma, mb = A.mean(0), B.mean(0)
    sa, sb = A.std(0, ddof=1) / 4, B.std(0, ddof=1) / 4
    zm = (ma.mean() - mb.mean()) / (np.sqrt((sa ** 2).sum() + (sb ** 2).sum()) / ma.size)
    assert abs(zm) < 3.5, zm
    sig = np.sqrt(sa ** 2 + sb ** 2)
    m = sig > 0
    assert (np.abs((ma - mb)[m] / sig[m]) < 3).mean() > 0.97
