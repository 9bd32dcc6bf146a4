"""Edge cases through the C ABI against the oracle: an empty sample range,
the smallest and largest depths, one-pixel and one-row images, one sample
per pixel, and a window ending exactly at the stream's end."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _parity(ws, **kw):
    from gpu_parity import compare_records, gpu_residual, oracle_residual, rel_l2
    g = gpu_residual(ws, records=True, **kw)
    o = oracle_residual(ws, records=True, **kw)
    c = compare_records(g["records"], o["records"])
    print(ws.name, kw, c, flush=True)
    assert c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"] <= max(1, 1e-3 * c["oracle"]), c
    if np.abs(o["image"]).sum() > 0:
        assert rel_l2(g["image"], o["image"]) <= 1e-3
    else:
        assert np.count_nonzero(g["image"]) == 0
    return c


def test_empty_sample_range_gives_zero():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=16, height=16, depth=4, spp=2)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.full((16, 16, 3), 9.0, dtype=torch.float32, device="cuda")
    st = native.render_residual(sc, ed, native.Params.make(2, 4, 1, sample_begin=100, sample_end=100), out,
                                stats=True)
    assert st["paths"] == 0 and st["samples"] == 0
    assert torch.count_nonzero(out) == 0


@pytest.mark.parametrize("depth", [2, 7])
def test_smallest_and_largest_depth(depth):
    # depth 2: only light seen through the pinhole (E L) and E x L paths; depth 7: the most the kernels hold
    c = _parity(scenes.cornell_motion(width=16, height=16, spp=2, depth=depth))
    if depth == 7:
        assert c["oracle"] > 1000


@pytest.mark.parametrize("w,h", [(1, 1), (37, 1), (1, 29)])
def test_degenerate_image_shapes(w, h):
    _parity(scenes.cornell_motion(width=w, height=h, spp=64 if w * h == 1 else 8, depth=4))


def test_one_sample_per_pixel_and_window_at_stream_end():
    ws = scenes.clutter_motion(width=40, height=24, spp=1, depth=5, n_spheres=40)
    N = 40 * 24
    _parity(ws)
    _parity(ws, s0=N - 77, s1=N)


def _deep_cluster(ws, n=20000):
    """Append n static triangles whose positions converge geometrically to a
    point inside the box (spacing and size halve every few hundred
    triangles): binned SAH cannot split them evenly, and the 4-wide collapse
    of the binary tree uses its whole stack budget (39 entries on some path;
    checked on the host when the scene is built)."""
    import dataclasses
    sc = ws.scene
    k = np.arange(n, dtype=np.float64)
    t = 1.0 - 2.0 ** (-k / 800.0)
    c = np.array([0.15, -0.2, -0.35])[None] + t[:, None] * np.array([-0.3, 0.25, 0.1])[None]
    s = (0.02 * 2.0 ** (-k / 1600.0))[:, None]
    tri = np.stack([c + s * np.array([1.0, 0.0, 0.2]), c + s * np.array([-0.5, 0.87, 0.0]),
                    c + s * np.array([-0.5, -0.87, -0.2])], 1)
    nv = len(sc.positions)
    return dataclasses.replace(ws, scene=dataclasses.replace(
        sc, positions=np.concatenate([sc.positions, tri.reshape(-1, 3).astype(np.float32)]),
        indices=np.concatenate([sc.indices, (nv + np.arange(3 * n)).reshape(-1, 3).astype(sc.indices.dtype)]),
        tri_material=np.concatenate([sc.tri_material, np.zeros(n, sc.tri_material.dtype)]),
        tri_object=np.concatenate([sc.tri_object, np.zeros(n, sc.tri_object.dtype)])))


def test_deep_bvh_at_the_stack_budget():
    """Residual records and a frame of the new scene against the oracle on a
    scene whose BVH needs the traversal stack's full depth."""
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = _deep_cluster(scenes.cornell_motion(width=32, height=32, depth=5, spp=4))
    print("deep cluster", len(ws.scene.indices), "triangles", flush=True)
    c = _parity(ws)
    assert c["oracle"] > 1000
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((32, 32, 3), dtype=torch.float32, device="cuda")
    native.render_frame(sc, ed, native.FRAME_NEW, native.Params.make(8, ws.depth, 17), out)
    native.sync_status()
    ref = oracle.OracleScene(ws.scene).render_frame(2, 8, ws.depth, 17, stream_dir=0, pose_new=ws.edit.old_to_new,
                                                    threads=8)[0]
    assert rel_l2(out.cpu().numpy().astype(np.float64), ref) < 1e-3
