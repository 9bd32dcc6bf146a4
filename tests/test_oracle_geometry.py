"""Oracle geometry and BSDF pins: independent float64 brute-force ray casting,
BVH == brute force, BSDF normalisation and sampling histograms."""
import math

import numpy as np

from paper_2406_16302_amd import scenes


def np_closest(pos, idx, o, d):
    """Float64 Moller-Trumbore over every triangle (independent of the oracle)."""
    v0 = pos[idx[:, 0]].astype(np.float64)
    e1 = pos[idx[:, 1]].astype(np.float64) - v0
    e2 = pos[idx[:, 2]].astype(np.float64) - v0
    o = o.astype(np.float64)[:, None, :]
    d = d.astype(np.float64)[:, None, :]
    p = np.cross(d, e2[None])
    det = (e1[None] * p).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o - v0[None]
        u = (s * p).sum(-1) * inv
        q = np.cross(s, e1[None])
        v = (d * q).sum(-1) * inv
        t = (e2[None] * q).sum(-1) * inv
    ok = (det != 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
    t = np.where(ok, t, np.inf)
    best = t.argmin(1)
    bt = t[np.arange(len(t)), best]
    return np.where(np.isfinite(bt), bt, -1), np.where(np.isfinite(bt), best, -1)


def random_rays(n, rng, lo, hi):
    o = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d], 1).astype(np.float32)


def test_closest_hit_matches_float64_brute_force(oracle_lib):
    w = scenes.cornell_motion(width=8, height=8)
    sc = w.scene
    o = oracle_lib.OracleScene(sc, brute=True)
    rng = np.random.default_rng(1)
    rays = random_rays(20000, rng, -0.45, 0.45)
    t, ids = o.trace(rays)
    tb, ib = np_closest(sc.positions, sc.indices, rays[:, :3], rays[:, 3:])
    same = ids == ib
    assert same.mean() > 0.999
    m = same & (ids >= 0)
    assert np.allclose(t[m], tb[m], rtol=1e-4, atol=1e-6)


def test_bvh_equals_brute_force(oracle_lib):
    w = scenes.clutter_motion(width=8, height=8, n_spheres=40)
    sc = w.scene
    ob = oracle_lib.OracleScene(sc, brute=False)
    of = oracle_lib.OracleScene(sc, brute=True)
    rng = np.random.default_rng(2)
    rays = random_rays(3000, rng, np.array([-5, 0.01, -5]), np.array([5, 1.0, 5]))
    for pose in (oracle_lib.IDENTITY, w.edit.old_to_new):
        t1, i1 = ob.trace(rays, pose)
        t2, i2 = of.trace(rays, pose)
        assert np.array_equal(i1, i2)
        assert np.array_equal(t1, t2)


def _hemisphere_grid(n):
    # midpoint quadrature in (cos theta, phi) over the upper hemisphere
    ct = (np.arange(n) + 0.5) / n
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi
    C, P = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - C ** 2)
    w = np.stack([S * np.cos(P), S * np.sin(P), C], -1).reshape(-1, 3)
    dw = (1.0 / n) * (2 * math.pi / (2 * n))
    return w, dw


def _integrals(oracle_lib, m, wi, n=64):
    import ctypes as C
    mm = np.asarray(m, np.float32)
    nn = np.array([0, 0, 1.0])
    w, dw = _hemisphere_grid(n)
    rho_cos = np.zeros(3)
    pdf_int = 0.0
    rgb = np.zeros(3)
    for wo in w:
        pdf = oracle_lib.lib().orc_bsdf_eval(mm.ctypes.data_as(C.POINTER(C.c_float)),
                                             nn.ctypes.data_as(C.POINTER(C.c_double)),
                                             np.asarray(wi, np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                             np.asarray(wo, np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                             rgb.ctypes.data_as(C.POINTER(C.c_double)))
        rho_cos += rgb * wo[2] * dw
        pdf_int += pdf * dw
    return rho_cos, pdf_int


def test_lambertian_albedo_and_pdf(oracle_lib):
    m = scenes.mat(scenes.DIFFUSE, (0.3, 0.5, 0.9))
    wi = np.array([0.3, 0.1, 0.9])
    wi /= np.linalg.norm(wi)
    rc, pi = _integrals(oracle_lib, m, wi, n=48)
    assert np.allclose(rc, [0.3, 0.5, 0.9], rtol=2e-3)
    assert abs(pi - 1.0) < 2e-3


def test_ggx_energy_bounded_and_pdf(oracle_lib):
    for rough in (0.3, 0.6):
        m = scenes.mat(scenes.GGX, (1.0, 1.0, 1.0), rough)
        wi = np.array([0.0, 0.3, 0.95])
        wi /= np.linalg.norm(wi)
        rc, pi = _integrals(oracle_lib, m, wi, n=256)
        assert (rc <= 1.0 + 2e-3).all() and (rc > 0.3).all()
        # the pdf over reflected directions integrates to the probability that
        # a half-vector sample reflects above the surface: compare with the
        # sampler's measured success rate
        import ctypes as C
        mm = np.asarray(m, np.float32)
        n = np.array([0, 0, 1], np.float32)
        wi32 = wi.astype(np.float32)
        out = np.zeros(3, np.float32)
        us = np.random.default_rng(9).random((40000, 2)).astype(np.float32)
        ok = sum(oracle_lib.lib().orc_bsdf_sample(mm.ctypes.data_as(C.POINTER(C.c_float)),
                                                  n.ctypes.data_as(C.POINTER(C.c_float)),
                                                  wi32.ctypes.data_as(C.POINTER(C.c_float)), float(a), float(b),
                                                  out.ctypes.data_as(C.POINTER(C.c_float))) for a, b in us)
        frac = ok / len(us)
        assert abs(pi - frac) < 3 * np.sqrt(frac * (1 - frac) / len(us)) + 2e-3, (rough, pi, frac)
        assert pi <= 1.0 + 2e-3


def test_sampling_histograms_match_pdf(oracle_lib):
    import ctypes as C
    rng = np.random.default_rng(5)
    for m in (scenes.mat(scenes.DIFFUSE, (0.5, 0.5, 0.5)), scenes.mat(scenes.GGX, (0.9, 0.9, 0.9), 0.4)):
        mm = np.asarray(m, np.float32)
        n = np.array([0, 0, 1], np.float32)
        wi = np.array([0.5, 0.0, 0.866], np.float32)
        out = np.zeros(3, np.float32)
        cts = []
        N = 60000
        for u0, u1 in rng.random((N, 2)).astype(np.float32):
            ok = oracle_lib.lib().orc_bsdf_sample(mm.ctypes.data_as(C.POINTER(C.c_float)),
                                                  n.ctypes.data_as(C.POINTER(C.c_float)),
                                                  wi.ctypes.data_as(C.POINTER(C.c_float)), float(u0), float(u1),
                                                  out.ctypes.data_as(C.POINTER(C.c_float)))
            if ok:
                cts.append(out.copy())
        cts = np.array(cts)
        # expected histogram of cos(theta) from the pdf by quadrature
        bins = np.linspace(0, 1, 11)
        h, _ = np.histogram(cts[:, 2], bins=bins)
        w, dw = _hemisphere_grid(200)
        rgb = np.zeros(3)
        nn = np.array([0, 0, 1.0])
        pdfs = np.array([oracle_lib.lib().orc_bsdf_eval(mm.ctypes.data_as(C.POINTER(C.c_float)),
                                                        nn.ctypes.data_as(C.POINTER(C.c_double)),
                                                        wi.astype(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                                        x.ctypes.data_as(C.POINTER(C.c_double)),
                                                        rgb.ctypes.data_as(C.POINTER(C.c_double)))
                         for x in w.astype(np.float64)])
        exp = np.array([pdfs[(w[:, 2] >= a) & (w[:, 2] < b)].sum() * dw for a, b in zip(bins[:-1], bins[1:])]) * N
        mask = exp > 20
        chi2 = ((h[mask] - exp[mask]) ** 2 / exp[mask]).sum()
        assert chi2 < 40.0, (m, chi2, h, exp)
