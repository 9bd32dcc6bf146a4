"""The path-tracing baselines of the paper's comparisons (Sec. 6.2) through
the C ABI, against the oracle on the same Philox streams: correlated path
tracing (both frames on the same random numbers) and path tracing of each
frame from scratch, each giving I_new - I_old."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("correlated", [True, False])
@pytest.mark.parametrize("name", ["cornell", "clutter"])
def test_frame_difference_matches_oracle(name, correlated):
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    if name == "cornell":
        ws = scenes.cornell_motion(width=32, height=32, depth=4)
        spp = 16
    else:
        ws = scenes.clutter_motion(width=48, height=40, depth=4, n_spheres=60)  # ragged 16x16 blocks
        spp = 4
    print(name, "correlated" if correlated else "independent", flush=True)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    native.render_frame_difference(sc, ed, correlated, native.Params.make(spp, ws.depth, 91), out)
    native.sync_status()
    o = oracle.OracleScene(ws.scene)
    kw = dict(pose_new=ws.edit.old_to_new, threads=8)
    ref = o.render_frame(2, spp, ws.depth, 91, stream_dir=0, **kw)[0] - \
        o.render_frame(1, spp, ws.depth, 91, stream_dir=0 if correlated else 1, **kw)[0]
    g = out.cpu().numpy().astype(np.float64)
    assert np.abs(ref).sum() > 0
    # the difference of two fp32 frames: compare against the frames' own scale
    frame = o.render_frame(2, spp, ws.depth, 91, stream_dir=0, **kw)[0]
    err = np.sqrt(((g - ref) ** 2).sum())
    assert err <= 1e-3 * np.sqrt((ref ** 2).sum()) + 1e-6 * np.sqrt((frame ** 2).sum()), \
        (err, rel_l2(g, ref))
    if correlated:
        # where every sample's path misses the object in both poses the
        # difference cancels exactly, on both sides
        assert (ref == 0).mean() > 0.1
        assert ((ref == 0) == (g == 0)).mean() > 0.99


def test_frame_difference_equals_two_frames():
    """The fused difference kernel equals two separate frame renders on the
    same streams, up to float rounding."""
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=32, height=32, depth=5)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    p = native.Params.make(8, 5, 13)
    d = torch.zeros((32, 32, 3), dtype=torch.float32, device="cuda")
    native.render_frame_difference(sc, ed, False, p, d)
    f_new = torch.zeros_like(d)
    f_old = torch.zeros_like(d)
    native.render_frame(sc, ed, native.FRAME_NEW, p, f_new)
    native.render_frame(sc, ed, native.FRAME_OLD, p, f_old)
    native.sync_status()
    ref = (f_new.double() - f_old.double()).cpu().numpy()
    assert rel_l2(d.cpu().numpy().astype(np.float64), ref) < 1e-4
