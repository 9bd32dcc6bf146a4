"""Plain NumPy definition of the residual denoiser (test infrastructure).

Only tests/ and the CPU legs of bench.py use it.  It shares no code with the
HIP library: the filter is written out from its definition, in float64,
one tap at a time.

The filter is an edge-avoiding a-trous wavelet transform (Dammertz et al.
2010, "Edge-avoiding a-trous wavelet transform for fast global illumination
filtering") with the variance-guided luminance weight and the squared-weight
variance update of spatiotemporal variance-guided filtering (Schied et al.
2017), applied to a residual image R = a + b whose per-pixel variance is
estimated from two independent halves as (a - b)^2 (mean over channels):

    pass i (stride s = 2^i), centre p, taps q = p + s (dx, dy), |dx|,|dy| <= 2:
      w_pq = h(dx) h(dy) * wn * wz * wl        (h = 1/16, 1/4, 3/8, 1/4, 1/16)
      wn   = max(0, n_p . n_q)^sigma_n         (both hit; 0 if one ray misses)
      wz   = exp(-|z_p - z_q| / (sigma_z z_p + 1e-6))
      wl   = exp(-|l_p - l_q| / (sigma_l sd_p))  (1 where l_p = l_q)
      sd_p = sqrt(3x3 Gaussian (1/4, 1/2, 1/4) of the variance around p)
      R'_p = sum_q w_pq R_q / sum_q w_pq,  v'_p = sum_q w_pq^2 v_q / (sum_q w_pq)^2
    where l is the mean of the three channels; the centre tap has weight
    h(0)^2; taps outside the image are left out (the weights renormalise).
"""
from __future__ import annotations

import numpy as np

B3 = {0: 0.375, 1: 0.25, -1: 0.25, 2: 0.0625, -2: 0.0625}


def camera_rays(camera):
    """Pixel-centre rays of the pinhole camera (eye, target, up, vfov, W, H)."""
    c = np.asarray(camera, np.float64)
    eye, tgt, up = c[0:3], c[3:6], c[6:9]
    W, H = int(c[10]), int(c[11])
    fwd = (tgt - eye) / np.linalg.norm(tgt - eye)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = np.tan(np.radians(c[9]) * 0.5)
    aspect = W / H
    px, py = np.meshgrid(np.arange(W), np.arange(H))
    sx = (2.0 * ((px + 0.5) / W) - 1.0) * aspect * th
    sy = (1.0 - 2.0 * ((py + 0.5) / H)) * th
    d = fwd[None, None] + right[None, None] * sx[..., None] + upv[None, None] * sy[..., None]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.broadcast_to(eye, d.shape).reshape(-1, 3), d.reshape(-1, 3)


def gbuffer(osc, scene, pose):
    """Normal (facing the camera) and hit distance per pixel centre, from the
    oracle's ray tracer with the object at `pose`; (0, 0, 0, -1) on a miss."""
    o, d = camera_rays(scene.camera)
    rays = np.concatenate([o, d], 1).astype(np.float32)
    t, ids = osc.trace(rays, pose)
    g = np.zeros((len(rays), 4))
    g[:, 3] = -1.0
    hit = ids >= 0
    P = np.asarray(pose, np.float64).reshape(3, 4)
    tri = scene.indices[ids[hit]]
    v = scene.positions.astype(np.float64)[tri]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    dyn = scene.tri_object[ids[hit]] == 1
    n[dyn] = n[dyn] @ P[:, :3].T
    flip = (n * d[hit]).sum(1) > 0
    n[flip] *= -1
    g[hit, :3] = n
    g[hit, 3] = t[hit]
    return g.reshape(scene.height, scene.width, 4)


def denoise(a, b, g, iterations=3, sigma_n=64.0, sigma_z=0.1, sigma_l=2.0):
    """The filter as defined in the module docstring (float64, one tap at a time)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    g = np.asarray(g, np.float64)
    H, W, _ = a.shape
    R = a + b
    v = ((a - b) ** 2).mean(-1)
    for it in range(iterations):
        s = 1 << it
        # 3x3 Gaussian of the variance (taps outside the image left out)
        vb = np.zeros((H, W))
        vw = np.zeros((H, W))
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = (0.5 if dx == 0 else 0.25) * (0.5 if dy == 0 else 0.25)
                ys0, ys1 = max(0, -dy), min(H, H - dy)
                xs0, xs1 = max(0, -dx), min(W, W - dx)
                vb[ys0:ys1, xs0:xs1] += k * v[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
                vw[ys0:ys1, xs0:xs1] += k
        sd = np.sqrt(np.maximum(vb / vw, 0.0))
        lum = R.mean(-1)
        sw = np.zeros((H, W))
        sr = np.zeros((H, W, 3))
        sv = np.zeros((H, W))
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                oy, ox = dy * s, dx * s
                ys0, ys1 = max(0, -oy), min(H, H - oy)
                xs0, xs1 = max(0, -ox), min(W, W - ox)
                if ys0 >= ys1 or xs0 >= xs1:
                    continue
                P = (slice(ys0, ys1), slice(xs0, xs1))
                Q = (slice(ys0 + oy, ys1 + oy), slice(xs0 + ox, xs1 + ox))
                w = np.full((ys1 - ys0, xs1 - xs0), B3[dx] * B3[dy])
                if dx or dy:
                    gp, gq = g[P], g[Q]
                    miss_p, miss_q = gp[..., 3] < 0, gq[..., 3] < 0
                    w = np.where(miss_p != miss_q, 0.0, w)
                    both = ~miss_p & ~miss_q
                    nd = np.maximum(0.0, (gp[..., :3] * gq[..., :3]).sum(-1))
                    wn = np.where(both, nd ** sigma_n, 1.0)
                    wz = np.where(both, np.exp(-np.abs(gp[..., 3] - gq[..., 3]) / (sigma_z * gp[..., 3] + 1e-6)),
                                  1.0)
                    dl = np.abs(lum[P] - lum[Q])
                    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
                        wl = np.where(dl > 0, np.exp(-dl / (sigma_l * sd[P])), 1.0)
                    wl = np.nan_to_num(wl, nan=0.0)
                    w = w * wn * wz * wl
                sw[P] += w
                sr[P] += w[..., None] * R[Q]
                sv[P] += w * w * v[Q]
        R = sr / sw[..., None]
        v = sv / (sw * sw)
    return R
