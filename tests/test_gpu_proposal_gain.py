"""What the trained proposal gains over the estimator without it.

The proposal is trained by the library's own kernels on records of the
estimator's technique-2/3 paths, then technique 8 takes the place of
techniques 2 and 3 (which it generalises: same start x_D, same two sensor
sides, a learned light-side direction), every other strategy kept.  Error is
the per-pixel MSE against a high-sample reference of the plain estimator,
averaged over independent seeds; cost is the device time of the call.
Both estimators must agree with the reference in the mean (unbiasedness),
and the learned one must have lower error at the same samples per pixel.
On the motion workload it must also have lower error x time (higher
efficiency).  On the material edit it does not with equal sample counts
(see the material-edit test); with the residual-aware per-technique counts
of rpi_allocate_samples it does, and that is asserted there."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _run(sc, ed, ws, spp, seed, mask, flags, prop=None, train=None, counts=None):
    from paper_2406_16302_amd import native
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    p = native.Params.make(spp, ws.depth, seed, mask=mask, flags=flags, proposal=prop, train_records=train,
                           technique_spp=counts)
    st = native.render_residual(sc, ed, p, out, stats=True)
    return out.double(), st


def _gain(ws, base, flags, spp_ref, spp_rec, spp, K, steps):
    from paper_2406_16302_amd import native
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    ref = torch.zeros((sc.height, sc.width, 3), dtype=torch.float64, device="cuda")
    chunks = 8
    for c in range(chunks):
        ref += _run(sc, ed, ws, spp_ref // chunks, 50_000 + c, base, flags)[0]
    ref /= chunks
    cap = 4_000_000
    buf = torch.zeros((cap, 10), dtype=torch.float32, device="cuda")
    _, st = _run(sc, ed, ws, spp_rec, 777, base, flags, train=buf)
    n = min(st["train_records"], cap)
    prop = native.Proposal(sc, None, seed=3)
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    prop.train(buf, n, steps, batch=16384, lr=1e-3, seed=11, losses=losses)
    L = losses.cpu().numpy()
    learned = (base & ~0x6) | 0x80
    res = {}
    ref_sum = ref.sum().item()
    var_ref = None
    # the learned estimator with residual-aware per-technique sample counts
    counts = native.allocate_samples(sc, ed, native.Params.make(spp, ws.depth, 999, mask=learned, flags=flags,
                                                                proposal=prop), pilot_spp=4)
    print("allocation", counts)
    for label, mask, pr, tc in (("plain", base, None, None), ("learned", learned, prop, None),
                                ("allocated", learned, prop, counts)):
        err, ms, sums = [], [], []
        for k in range(K):
            img, s = _run(sc, ed, ws, spp, 1000 + k, mask, flags, prop=pr, counts=tc)
            err.append(((img - ref) ** 2).mean().item())
            ms.append(s["milliseconds"])
            sums.append(img.sum().item())
        # unbiasedness: the image sum of the K-run mean against the reference's;
        # the reference is the plain estimator at spp_ref / spp times the samples
        v = np.var(sums, ddof=1)
        if var_ref is None:
            var_ref = v * spp / spp_ref
        z = (np.mean(sums) - ref_sum) / np.sqrt(v / K + var_ref)
        res[label] = (float(np.mean(err)), float(np.std(err, ddof=1) / np.sqrt(K)), float(np.median(ms)), float(z))
    print(ws.name, "records %d, loss %.3f -> %.3f" % (n, L[:20].mean(), L[-20:].mean()))
    for k, (m, se, t, d) in res.items():
        print("  %-8s mse %.4g +- %.2g  ms %.2f  efficiency %.4g  z(mean - ref) %.2f" % (k, m, se, t, 1 / (m * t), d))
    return res


def _check(res, mse_ratio_max, eff_ratio_min=None, alloc_eff_min=None):
    mp, sp, tp, zp = res["plain"]
    ml, sl, tl, zl = res["learned"]
    ma, sa, ta, za = res["allocated"]
    assert abs(zp) < 4 and abs(zl) < 4 and abs(za) < 4, (zp, zl, za)
    assert ml < mse_ratio_max * mp, (ml, mp)
    if eff_ratio_min is not None:
        assert (mp * tp) / (ml * tl) > eff_ratio_min, ((mp, tp), (ml, tl))
    if alloc_eff_min is not None:
        assert (mp * tp) / (ma * ta) > alloc_eff_min, ((mp, tp), (ma, ta))


def test_gain_on_the_motion_workload():
    # the clutter-motion scene (106k triangles, moving 20k-triangle sphere) at 128x128
    ws = scenes.clutter_motion(width=128, height=128, depth=5)
    res = _gain(ws, ws.mask, 1, spp_ref=2048, spp_rec=32, spp=8, K=24, steps=3000)
    _check(res, 0.9, 1.05)


def test_gain_on_the_material_edit():
    # the 983k-triangle material-edit scene at 256x256 (the learned-proposal
    # workload's scene).  Most of this residual's error comes from technique
    # 1 (the edited surface lit directly: the glossy highlight E x_D L, which
    # only technique 1 samples), and the proposal does not touch it.  The gain
    # is lower error at the same samples per pixel (about 10%); technique 8's
    # extra work (its walks and MLP passes) costs more time than that saves,
    # so the equal-time target is not met on this workload and only the
    # equal-sample gain is asserted.
    ws = scenes.material_edit(width=256, height=256, depth=6)
    res = _gain(ws, 0x07, 0, spp_ref=512, spp_rec=32, spp=8, K=12, steps=3000)
    # with residual-aware sample counts (more samples for technique 1, fewer
    # for technique 8) the learned estimator beats the plain one at equal time
    _check(res, 0.95, alloc_eff_min=1.0)
