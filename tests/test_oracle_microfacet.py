"""Pins of the oracle's GGX conductor and of its MLP forward pass.

The GGX reflectance of the oracle (D, Smith G1, Schlick F; Walter et al.
2007) is checked against facts that do not restate its formulas:

* at normal incidence (wi = wo = n) the reflectance is F0 / (4 pi alpha^2):
  the peak of D is 1/(pi alpha^2), G1 is 1 and the Fresnel term is F0;
* the projected area of the microfacets is the macro-surface's:
  the integral of D(h) (n.h) over the hemisphere of h is 1;
* the weak white furnace (Heitz 2014, "Understanding the masking-shadowing
  function"): for every outgoing direction wo the integral over the sphere of
  wi of G1(wo) D(h) / (4 |n.wo|), with h the half vector, is 1.  For a given
  D this fixes the masking function uniquely, so a G1 with alpha in place of
  alpha^2 (or a D with the wrong normalisation) fails;
* Schlick's term is the Fresnel factor of the half vector: with F0 = 0 it is
  (1 - |wi.h|)^5, so it vanishes for retro-reflection (h = wi) at every
  angle and tends to 1 at grazing h; a term taken at n.wi instead would not
  vanish for retro-reflection;
* the reflectance with F0 = 1 (where F is 1) factors as D(h) G1(wi) G1(wo) /
  (4 |n.wi| |n.wo|) with the D and G1 pinned above.

The MLP forward pass of the learned proposal is compared with a NumPy forward
of the parameter layout the library documents ([in][out] row-major weights,
biases after each matrix), in float64 and with bfloat16 rounding taken from
torch (round to nearest, ties to even)."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2406_16302_amd import scenes


def _eval(lib, m, n, wi, wo):
    rgb = np.zeros(3)
    mm = np.asarray(m, np.float32)
    lib.orc_bsdf_eval(mm.ctypes.data_as(C.POINTER(C.c_float)),
                      np.asarray(n, np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                      np.asarray(wi, np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                      np.asarray(wo, np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                      rgb.ctypes.data_as(C.POINTER(C.c_double)))
    return rgb


def _ggx_fns(oracle_lib):
    L = oracle_lib.lib()
    L.orc_ggx_D.restype = C.c_double
    L.orc_ggx_D.argtypes = [C.c_double, C.c_double]
    L.orc_ggx_G1.restype = C.c_double
    L.orc_ggx_G1.argtypes = [C.c_double, C.c_double]
    return L.orc_ggx_D, L.orc_ggx_G1


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.6, 0.9])
def test_ggx_normal_incidence_closed_form(oracle_lib, alpha):
    f0 = (0.2, 0.5, 0.9)
    n = np.array([0.0, 0.0, 1.0])
    rgb = _eval(oracle_lib.lib(), scenes.mat(scenes.GGX, f0, alpha), n, n, n)
    # the material row is float32: compare with its float32 values
    a32 = float(np.float32(alpha))
    want = np.array(f0, np.float32).astype(np.float64) / (4.0 * math.pi * a32 * a32)
    assert np.allclose(rgb, want, rtol=1e-12), (rgb, want)
    # the surface is two-sided: the same from below
    rgb2 = _eval(oracle_lib.lib(), scenes.mat(scenes.GGX, f0, alpha), n, -n, -n)
    assert np.allclose(rgb2, want, rtol=1e-12)


def _sphere_grid(n):
    """Midpoint quadrature on the sphere in (cos theta, phi): directions, weight."""
    ct = -1 + (np.arange(n) + 0.5) * 2.0 / n
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi
    Cc, P = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - Cc ** 2)
    w = np.stack([S * np.cos(P), S * np.sin(P), Cc], -1).reshape(-1, 3)
    return w, (2.0 / n) * (2 * math.pi / (2 * n))


def _hemi_grid_mu(n, alpha):
    """Quadrature over the upper hemisphere in the variable u with
    tan(theta) = alpha sqrt(u / (1 - u)) (dense near the pole where D is),
    written as u = 1 - v^2 so that integrands growing like 1/cos(theta) at the
    horizon stay bounded; midpoints in v and phi.  Returns directions and
    solid-angle weights."""
    v = (np.arange(n) + 0.5) / n
    u = 1.0 - v * v
    du_dv = 2.0 * v
    th = np.arctan(alpha * np.sqrt(u / (1 - u)))
    dth_du = alpha * 0.5 / np.sqrt(u * (1 - u)) / (1 + alpha ** 2 * u / (1 - u)) / (1 - u)
    ph = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * math.pi
    TH, P = np.meshgrid(th, ph, indexing="ij")
    J, _ = np.meshgrid(dth_du * du_dv, ph, indexing="ij")
    w = np.stack([np.sin(TH) * np.cos(P), np.sin(TH) * np.sin(P), np.cos(TH)], -1).reshape(-1, 3)
    wt = (np.sin(TH) * J).reshape(-1) * (1.0 / n) * (2 * math.pi / (2 * n))
    return w, wt


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.6, 0.9])
def test_ggx_D_projected_area_is_one(oracle_lib, alpha):
    D, _ = _ggx_fns(oracle_lib)
    h, wt = _hemi_grid_mu(200, alpha)
    tot = sum(D(alpha, float(c)) * c * q for c, q in zip(h[:, 2], wt))
    assert abs(tot - 1.0) < 1e-6, (alpha, tot)


@pytest.mark.parametrize("alpha", [0.2, 0.5, 0.8])
@pytest.mark.parametrize("theta_o_deg", [0.0, 30.0, 60.0, 80.0])
def test_ggx_weak_white_furnace(oracle_lib, alpha, theta_o_deg):
    """Integral over wi of G1(wo) D(h) / (4 |n.wo|) = 1 (upper-hemisphere h)."""
    D, G1 = _ggx_fns(oracle_lib)
    to = math.radians(theta_o_deg)
    wo = np.array([math.sin(to), 0.0, math.cos(to)])
    # integrate in the half-vector domain (dense where D is), dwi = 4 |wo.h| dh
    h, wt = _hemi_grid_mu(300, alpha)
    oh = h @ wo
    keep = oh > 0  # each wi on the sphere has exactly one h with wo.h >= 0
    g1o = G1(alpha, math.cos(to))
    d = np.array([D(alpha, float(c)) for c in h[keep, 2]])
    tot = (g1o * d / (4 * math.cos(to)) * 4 * oh[keep] * wt[keep]).sum()
    assert abs(tot - 1.0) < 1e-5, (alpha, theta_o_deg, tot)
    # a masking term with alpha in place of alpha^2 would miss the identity
    g_bad = 2.0 / (1.0 + math.sqrt(1.0 + alpha * math.tan(to) ** 2))
    if theta_o_deg >= 30.0:
        assert abs(tot / g1o * g_bad - 1.0) > 5e-3  # what the identity would see


def test_schlick_term_follows_the_half_vector(oracle_lib):
    lib = oracle_lib.lib()
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(3)
    for alpha in (0.25, 0.6):
        m0 = scenes.mat(scenes.GGX, (0.0, 0.0, 0.0), alpha)
        m1 = scenes.mat(scenes.GGX, (1.0, 1.0, 1.0), alpha)
        m3 = scenes.mat(scenes.GGX, (0.3, 0.3, 0.3), alpha)
        # retro-reflection: h = wi, so F = F0 at every angle (0 for F0 = 0)
        for th in (0.0, 0.4, 0.9, 1.3):
            w = np.array([math.sin(th), 0.0, math.cos(th)])
            assert np.all(_eval(lib, m0, n, w, w) == 0.0), th
            assert np.all(_eval(lib, m1, n, w, w) > 0.0)
        # general pairs: rho(F0 = 0) / rho(F0 = 1) = (1 - |wi.h|)^5
        for _ in range(200):
            wi = _unit(rng.normal(size=3) * [1, 1, 0.4] + [0, 0, 0.3])
            wo = _unit(rng.normal(size=3) * [1, 1, 0.4] + [0, 0, 0.3])
            if wi[2] <= 1e-3 or wo[2] <= 1e-3:
                continue
            r1 = _eval(lib, m1, n, wi, wo)
            if r1[0] <= 1e-300:
                continue
            h = _unit(wi + wo)
            ratio0 = _eval(lib, m0, n, wi, wo)[0] / r1[0]
            assert abs(ratio0 - (1 - abs(wi @ h)) ** 5) < 1e-12
            ratio3 = _eval(lib, m3, n, wi, wo)[0] / r1[0]
            f3 = float(np.float32(0.3))
            assert abs(ratio3 - (f3 + (1 - f3) * (1 - abs(wi @ h)) ** 5)) < 1e-12
    # grazing half vector: wi and wo nearly opposite, h . wi = sin(a) -> 0 and
    # F -> 1 for any F0, with 1 - F = (1 - F0)(1 - (1 - sin a)^5) ~ 5 (1 - F0) sin a
    f3 = float(np.float32(0.3))
    for a in (1e-2, 1e-3, 1e-5):
        wi = np.array([math.cos(a), 0.0, math.sin(a)])
        wo = np.array([-math.cos(a), 0.0, math.sin(a)])
        r = _eval(lib, scenes.mat(scenes.GGX, (0.3, 0.3, 0.3), 0.5), n, wi, wo) / _eval(
            lib, scenes.mat(scenes.GGX, (1.0, 1.0, 1.0), 0.5), n, wi, wo)
        assert np.all(np.abs(1.0 - r) <= 5 * (1 - f3) * math.sin(a) * (1 + 1e-9)), (a, r)


def test_ggx_reflectance_factors_into_pinned_terms(oracle_lib):
    D, G1 = _ggx_fns(oracle_lib)
    lib = oracle_lib.lib()
    rng = np.random.default_rng(4)
    n = np.array([0.0, 0.0, 1.0])
    checked = 0
    for alpha in (0.15, 0.45, 0.85):
        m1 = scenes.mat(scenes.GGX, (1.0, 1.0, 1.0), alpha)
        for _ in range(100):
            wi = _unit(rng.normal(size=3) + [0, 0, 0.8])
            wo = _unit(rng.normal(size=3) + [0, 0, 0.8])
            if wi[2] <= 1e-3 or wo[2] <= 1e-3:
                continue
            h = _unit(wi + wo)
            a32 = float(np.float32(alpha))
            want = D(a32, float(h[2])) * G1(a32, float(wi[2])) * G1(a32, float(wo[2])) / (4 * wi[2] * wo[2])
            got = _eval(lib, m1, n, wi, wo)
            assert np.allclose(got, want, rtol=1e-12), (alpha, got, want)
            # two-sided: mirrored below the surface
            flip = np.array([1.0, 1.0, -1.0])
            assert np.allclose(_eval(lib, m1, n, wi * flip, wo * flip), want, rtol=1e-12)
            checked += 1
    assert checked > 150


# ----------------------------------------------------------------- MLP forward

_SHAPES = [(6, 64), (64, 64), (64, 64), (64, 40)]


def _np_forward(params, x, round_fn=None):
    """Forward of the documented layout in float64.  round_fn rounds weights
    and the input of every layer (after a float32 conversion, as the kernels
    hold activations in float32); biases stay as given."""
    r = (lambda a: a) if round_fn is None else round_fn
    off = 0
    a = r(np.asarray(x, np.float64))
    for li, (fi, fo) in enumerate(_SHAPES):
        W = np.asarray(params[off:off + fi * fo], np.float32).reshape(fi, fo)
        off += fi * fo
        b = np.asarray(params[off:off + fo], np.float64)
        off += fo
        z = a @ r(W.astype(np.float64)) + b
        if li < 3:
            a = r(np.maximum(z, 0.0))
        else:
            a = z
    assert off == len(params)
    return a


def _torch_bf16(a):
    import torch
    t = torch.from_numpy(np.asarray(a, np.float64).astype(np.float32))
    return t.to(torch.bfloat16).to(torch.float32).double().numpy()


def _params_with_ties(seed):
    rng = np.random.default_rng(seed)
    p = np.concatenate([np.concatenate([rng.uniform(-math.sqrt(6 / fi), math.sqrt(6 / fi), fi * fo),
                                        rng.normal(0, 0.1, fo)]) for fi, fo in _SHAPES]).astype(np.float32)
    # exact bfloat16 ties (the low 16 bits are 0x8000) on both sides of even/odd
    # mantissas, so round-half-to-even is exercised rather than half-up
    bits = p.view(np.uint32).copy()
    sel = rng.choice(len(p), 600, replace=False)
    bits[sel] = (bits[sel] & 0xFFFF0000) | 0x8000
    return bits.view(np.float32)


def test_mlp_forward_matches_numpy_float64(oracle_lib):
    p = _params_with_ties(7)
    x = np.random.default_rng(8).uniform(-1, 1, (300, 6))
    got = oracle_lib.mlp_forward(p, x, bf16=False)
    want = _np_forward(p, x)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12), np.abs(got - want).max()
    # a transposed weight matrix ([out][in]) would not match
    bad = p.copy()
    bad[448:448 + 4096] = bad[448:448 + 4096].reshape(64, 64).T.ravel()
    assert not np.allclose(oracle_lib.mlp_forward(bad, x, bf16=False), want, rtol=1e-6)


def test_mlp_bf16_forward_matches_torch_rounding(oracle_lib):
    pytest.importorskip("torch")
    p = _params_with_ties(9)
    x = np.random.default_rng(10).uniform(-1, 1, (300, 6))
    got = oracle_lib.mlp_forward(p, x, bf16=True)
    want = _np_forward(p, x, _torch_bf16)
    assert np.allclose(got, want, rtol=1e-11, atol=1e-11), np.abs(got - want).max()
    # rounding half-up instead of half-to-even changes the result
    def half_up(a):
        b = np.asarray(a, np.float64).astype(np.float32).view(np.uint32)
        b = ((b + np.uint32(0x8000)) & np.uint32(0xFFFF0000)).view(np.float32)
        return b.astype(np.float64)
    assert not np.allclose(_np_forward(p, x, half_up), got, rtol=1e-9, atol=1e-9)
