"""Batched residual jobs (one captured hipGraph of persistent launches)
against per-job renders and against the oracle."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _jobs(sizes, offsets, base=None):
    out = []
    for (w, h), off in zip(sizes, offsets):
        po = base if base is not None else scenes.translation((0, 0, 0))
        pn = scenes.translation(off)
        out.append({"pose_old": po, "pose_new": pn, "out": torch.zeros((h, w, 3), dtype=torch.float32, device="cuda")})
    return out


def _direct(ws, w, h, off, job, spp, depth):
    from paper_2406_16302_amd import native
    sc = native.Scene(ws.scene.with_resolution(w, h))
    e = scenes.Edit(scenes.EDIT_RIGID, scenes.translation(off))
    ed = native.Edit(sc, e)
    p = native.Params.make(spp, depth, ws.seed, job=job)
    out = torch.zeros((h, w, 3), dtype=torch.float32, device="cuda")
    native.render_residual(sc, ed, p, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_batch_equals_per_job_renders_and_replays():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=32, height=32, depth=4)
    sc = native.Scene(ws.scene)
    sizes = [(32, 32), (48, 24), (16, 40)]
    offs = [(0.1, 0, 0.05), (0.05, 0, -0.08), (-0.07, 0.02, 0.0)]
    p = native.Params.make(4, 4, ws.seed, job=5)
    jobs = _jobs(sizes, offs)
    st = native.render_residual_batch(sc, jobs, p, stats=True)
    torch.cuda.synchronize()
    assert st["paths"] > 1000
    for j, ((w, h), off) in enumerate(zip(sizes, offs)):
        ref = _direct(ws, w, h, off, 5 + j, 4, 4)
        got = jobs[j]["out"].cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max()), j
    # replay with new poses and new output tensors, with eager work in between
    offs2 = [(0.0, 0, 0.1), (0.12, 0, 0.0), (0.03, 0.0, 0.03)]
    for rep in range(3):
        junk = torch.randn(1000, device="cuda").sum()
        jobs2 = _jobs(sizes, offs2 if rep % 2 == 0 else offs)
        native.render_residual_batch(sc, jobs2, p)
        torch.cuda.synchronize()
        use = offs2 if rep % 2 == 0 else offs
        for j, ((w, h), off) in enumerate(zip(sizes, use)):
            ref = _direct(ws, w, h, off, 5 + j, 4, 4)
            got = jobs2[j]["out"].cpu().numpy()
            assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max()), (rep, j)
        del junk


def test_batch_matches_oracle_with_moving_old_pose():
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=24, height=24, depth=4)
    sc = native.Scene(ws.scene)
    po = scenes.translation((-0.03, 0.0, 0.02))
    sizes = [(24, 24), (40, 20)]
    offs = [(0.1, 0, 0.05), (0.06, 0.0, -0.04)]
    jobs = _jobs(sizes, offs, base=po)
    p = native.Params.make(4, 4, 99, job=11)
    native.render_residual_batch(sc, jobs, p)
    torch.cuda.synchronize()
    for j, ((w, h), off) in enumerate(zip(sizes, offs)):
        o = oracle.OracleScene(ws.scene.with_resolution(w, h))
        ref = o.render_residual(4, 4, 99, pose_old=po, pose_new=scenes.translation(off), job=11 + j, threads=8)
        assert rel_l2(jobs[j]["out"].cpu().numpy().astype(np.float64), ref["image"]) < 1e-3, j


def test_autotune_returns_a_configuration():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=32, height=32, depth=3)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    t = native.autotune(sc, ed, native.Params.make(16, 3, 1))
    assert t["queue_cap"] in (1 << 23, 1 << 24, 1 << 25) and t["walk_blocks_per_cu"] in (16, 32)
    assert t["ms_per_msample"] > 0


def test_batch_with_balance_across_directions_matches_oracle():
    """RPI_FLAG_BALANCE in the batched launch: each job against the oracle's
    cross-direction balance heuristic with its own poses and job index."""
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=24, height=24, depth=4)
    sc = native.Scene(ws.scene)
    sizes = [(24, 24), (32, 16)]
    offs = [(0.1, 0, 0.05), (-0.06, 0.0, 0.07)]
    jobs = _jobs(sizes, offs)
    p = native.Params.make(4, 4, 71, job=3, flags=native.FLAG_TWO_WAY | native.FLAG_BALANCE)
    native.render_residual_batch(sc, jobs, p)
    torch.cuda.synchronize()
    for j, ((w, h), off) in enumerate(zip(sizes, offs)):
        o = oracle.OracleScene(ws.scene.with_resolution(w, h))
        ref = o.render_residual(4, 4, 71, pose_new=scenes.translation(off), job=3 + j, threads=8, balance=True)
        assert np.abs(ref["image"]).sum() > 0
        assert rel_l2(jobs[j]["out"].cpu().numpy().astype(np.float64), ref["image"]) < 1e-3, j
