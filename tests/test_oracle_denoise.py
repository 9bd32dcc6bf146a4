"""Pins of the denoiser's plain definition (oracle/denoise.py): facts that do
not restate its formula -- a constant residual with zero variance passes
unchanged, with every edge-stopping weight switched off the interior equals
the composition of the dilated B3-spline convolutions (scipy), pixels deep
inside a region no dynamic path reached keep their exact zero, and the
pixel-centre rays of the guide hit what a float64 brute-force caster hits."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes


def _flat_g(H, W, depth=3.0):
    g = np.zeros((H, W, 4))
    g[..., 2] = 1.0
    g[..., 3] = depth
    return g


def test_constant_residual_with_zero_variance_is_unchanged():
    from oracle import denoise
    a = np.full((20, 24, 3), 0.125)
    out = denoise.denoise(a, a.copy(), _flat_g(20, 24))
    assert np.allclose(out, 0.25, rtol=1e-14, atol=0)


def test_without_edge_stopping_the_interior_is_the_b3_wavelet_smoothing():
    from scipy import ndimage
    from oracle import denoise
    rng = np.random.default_rng(3)
    H = W = 48
    a = rng.normal(0.5, 0.2, (H, W, 3))
    b = rng.normal(0.5, 0.2, (H, W, 3))
    out = denoise.denoise(a, b, _flat_g(H, W), iterations=3, sigma_n=0.0, sigma_z=1e30, sigma_l=1e30)
    h = np.array([1, 4, 6, 4, 1]) / 16.0
    ref = a + b
    for it in range(3):
        s = 1 << it
        k = np.zeros(4 * s + 1)
        k[::s] = h
        k2 = np.outer(k, k)
        ref = np.stack([ndimage.convolve(ref[..., c], k2, mode="constant") for c in range(3)], -1)
    m = 2 * (1 + 2 + 4)
    assert np.allclose(out[m:-m, m:-m], ref[m:-m, m:-m], rtol=1e-12, atol=1e-12)
    # near the border the missing taps renormalise (a plain convolution would darken)
    assert np.abs(out[0, 0] - ref[0, 0]).max() > 1e-3


def test_zero_region_keeps_its_zero():
    from oracle import denoise
    rng = np.random.default_rng(4)
    H, W = 64, 64
    a = rng.normal(0.0, 1.0, (H, W, 3))
    b = rng.normal(0.0, 1.0, (H, W, 3))
    a[16:48, 16:48] = 0.0
    b[16:48, 16:48] = 0.0
    out = denoise.denoise(a, b, _flat_g(H, W), iterations=3)
    # each pass's variance blur carries the noisy front one pixel further in;
    # deeper than that the weights to every differing neighbour vanish
    assert np.count_nonzero(out[20:44, 20:44]) == 0
    assert np.count_nonzero(out[:8]) > 0


def test_guide_rays_hit_what_brute_force_hits(oracle_lib):
    from oracle import denoise
    from test_oracle_geometry import np_closest
    w = scenes.cornell_motion(width=24, height=20)
    sc = w.scene
    o = oracle_lib.OracleScene(sc, brute=True)
    g = denoise.gbuffer(o, sc, oracle_lib.IDENTITY)
    orig, d = denoise.camera_rays(sc.camera)
    t, ids = np_closest(sc.positions, sc.indices, orig, d)
    ok = ids >= 0
    gg = g.reshape(-1, 4)
    assert ok.mean() > 0.9
    assert np.array_equal(gg[:, 3] >= 0, ok)
    assert np.allclose(gg[ok, 3], t[ok], rtol=1e-5)
    # normals are unit and face the camera
    assert np.allclose(np.linalg.norm(gg[ok, :3], axis=1), 1.0)
    assert ((gg[ok, :3] * d[ok]).sum(1) < 0).all()
