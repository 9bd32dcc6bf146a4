"""Parity at the workloads' full sizes and in the launch configuration the
benchmark times.

* Windows of sample indices of every (technique, direction) stream of the
  full-size workloads, compared with the oracle record by record.  These
  calls plan rounds from their window (twice the window's samples).
* The clutter workload's whole stream at the benchmark's round of 2^25
  samples (set with rpi_set_tuning, as the autotuner picks it): the records
  of the last 8192 samples of every stream, whose slots lie just below 2^25,
  against the oracle; and the same sample range rendered with rounds of 2^25
  and of 2^20 samples gives the same image bit for bit.
* The batched animation (32 jobs up to 1024^2, one graph) against per-job
  renders, and windows of its largest jobs against the oracle.
* Technique 8 on the 983k-triangle scene with weights trained on the GPU.
The tiny Cornell workload is compared whole."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _window(ws, s0, n, max_div=1e-3, **kw):
    from gpu_parity import compare_records, gpu_residual, oracle_residual
    g = gpu_residual(ws, records=True, s0=s0, s1=s0 + n, **kw)
    o = oracle_residual(ws, records=True, s0=s0, s1=s0 + n, mlp=kw.get("mlp"))
    c = compare_records(g["records"], o["records"])
    div = (c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"]) / max(c["oracle"], 1)
    print(ws.name, "window [%d, %d)" % (s0, s0 + n), c, flush=True)
    assert c["oracle"] > 500
    assert div <= max_div, c
    return g, o


def test_cornell_workload_whole():
    # 64x64, depth 3, 16 spp, all seven techniques, both directions
    from gpu_parity import compare_records, gpu_residual, oracle_residual, rel_l2
    ws = scenes.cornell_motion()
    g = gpu_residual(ws, records=True)
    o = oracle_residual(ws, records=True)
    c = compare_records(g["records"], o["records"])
    rel = rel_l2(g["image"], o["image"])
    print("cornell_motion full", "rel_l2=%.3g" % rel, c)
    assert (c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"]) <= 1e-3 * c["oracle"]
    assert rel <= 1e-3


def test_cornell_workload_resting_on_the_floor_whole():
    # the configuration's reading: the cube rests on the floor (coplanar contact)
    from gpu_parity import compare_records, gpu_residual, oracle_residual, rel_l2
    ws = scenes.cornell_motion(lift=0.0)
    g = gpu_residual(ws, records=True)
    o = oracle_residual(ws, records=True)
    c = compare_records(g["records"], o["records"])
    rel = rel_l2(g["image"], o["image"])
    print("cornell_motion resting full", "rel_l2=%.3g" % rel, c)
    assert (c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"]) <= 1e-3 * c["oracle"]
    assert rel <= 1e-3


def test_clutter_workload_window():
    # 512x512, depth 5, 64 spp: the benchmark's workload
    ws = scenes.clutter_motion()
    _window(ws, 9_000_000, 16384)


def test_material_edit_workload_window():
    # 1024x1024, depth 6, 32 spp, 983k triangles
    ws = scenes.material_edit()
    _window(ws, 20_000_000, 8192)


def test_clutter_stream_at_the_benchmark_round():
    """The whole clutter stream (2^24 samples per technique and direction) in
    one round of 2^25 slots per technique, as the benchmark runs it; the
    records of samples [2^24 - 8192, 2^24) of every stream (slots up to
    2^25 - 1) against the oracle."""
    from gpu_parity import compare_records, oracle_residual
    from paper_2406_16302_amd import native
    ws = scenes.clutter_motion()
    N = ws.spp * ws.scene.width * ws.scene.height
    assert N == 1 << 24
    sc = native.Scene(ws.scene)
    native.set_tuning(sc, 1 << 25, 16, 16)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    print("clutter full stream, round 2^25, records", flush=True)
    st = native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed,
                                                             flags=native.FLAG_TWO_WAY | native.FLAG_RECORDS),
                                out, stats=True)
    rec = sc.records()
    assert len(rec) == st["paths"] + int((np.frombuffer(rec[:, 4].tobytes(), np.int32) < 0).sum())
    s0 = N - 8192
    g = rec[rec[:, 2] >= s0]
    del rec
    o = oracle_residual(ws, records=True, s0=s0, s1=N)
    c = compare_records(g, o["records"])
    print("window [%d, %d)" % (s0, N), c, flush=True)
    assert c["oracle"] > 5000
    assert (c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"]) <= 1e-3 * c["oracle"], c


def test_round_size_does_not_change_the_image():
    """2^23 samples per stream rendered in rounds of 2^25 samples (slots past
    2^24) and in rounds of 2^20: the same Philox streams and paths, and the
    same image bit for bit."""
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.clutter_motion()
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    imgs, paths = [], []
    for q in (1 << 25, 1 << 20):
        out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
        print("clutter [0, 2^23) round", q, flush=True)
        st = native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, sample_end=1 << 23,
                                                                 queue_cap=q), out, stats=True)
        imgs.append(out.cpu().numpy().astype(np.float64))
        paths.append(st["paths"])
    assert paths[0] == paths[1] and paths[0] > 10_000_000
    # the splat accumulates in fixed point: the rounds do not change a bit
    assert np.array_equal(imgs[0], imgs[1]), rel_l2(imgs[0], imgs[1])


def test_batched_animation_full_size():
    """The 32-job Bezier animation (images 256^2..1024^2, 16 spp, one captured
    graph) against per-job renders with the same Philox job words, then a
    window of its 1024^2 jobs against the oracle."""
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.clutter_motion(spp=16)
    sc = native.Scene(ws.scene)
    native.set_tuning(sc, 1 << 25, 16, 16)
    jobs = scenes.bezier_jobs()
    assert len(jobs) == 32
    outs = [torch.zeros((j["height"], j["width"], 3), dtype=torch.float32, device="cuda") for j in jobs]
    jl = [{"pose_old": j["pose_old"], "pose_new": j["pose_new"], "out": o} for j, o in zip(jobs, outs)]
    p = native.Params.make(16, ws.depth, ws.seed, flags=native.FLAG_TWO_WAY, job=100)
    print("batch of 32 jobs", flush=True)
    st = native.render_residual_batch(sc, jl, p, stats=True)
    total = 0
    imgs = [o.cpu() for o in outs]
    for i, j in enumerate(jobs):
        # the same job alone (a one-job batch: the job's own poses, image size
        # and Philox job word)
        ref = torch.zeros_like(outs[i])
        one = [{"pose_old": j["pose_old"], "pose_new": j["pose_new"], "out": ref}]
        st1 = native.render_residual_batch(sc, one, native.Params.make(16, ws.depth, ws.seed,
                                                                       flags=native.FLAG_TWO_WAY, job=100 + i),
                                           stats=True)
        total += st1["paths"]
        r = rel_l2(imgs[i].numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64))
        assert r < 1e-5, (i, r)
    assert total == st["paths"]
    # oracle windows on the largest jobs
    big = [i for i, j in enumerate(jobs) if j["width"] == 1024][:2]
    assert big
    pw = native.Params.make(16, ws.depth, ws.seed, flags=native.FLAG_TWO_WAY, job=100, sample_end=4096)
    for o_ in outs:
        o_.zero_()
    native.render_residual_batch(sc, jl, pw)
    native.sync_status()
    for i in big:
        j = jobs[i]
        osc = oracle.OracleScene(ws.scene.with_resolution(j["width"], j["height"]))
        ref = osc.render_residual(16, ws.depth, ws.seed, pose_old=j["pose_old"], pose_new=j["pose_new"], s0=0,
                                  s1=4096, threads=8, job=100 + i)["image"]
        r = rel_l2(outs[i].cpu().numpy().astype(np.float64), ref)
        print("job %d (1024^2) window [0, 4096): rel L2 %.3g" % (i, r), flush=True)
        assert np.abs(ref).sum() > 0 and r < 1e-3


def test_technique8_trained_on_the_material_workload():
    """Technique 8 on the 983k-triangle material edit with weights trained on
    the GPU from the estimator's own records: a window of records against the
    oracle running the same weights."""
    from paper_2406_16302_amd import native
    ws = scenes.material_edit()
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    cap = 2_000_000
    buf = torch.zeros((cap, 10), dtype=torch.float32, device="cuda")
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    print("material edit: records for training", flush=True)
    st = native.render_residual(sc, ed, native.Params.make(1, ws.depth, 777, mask=0x07, flags=0, train_records=buf),
                                out, stats=True)
    n = min(st["train_records"], cap)
    assert n > 100_000
    prop = native.Proposal(sc, None, seed=3)
    prop.train(buf, n, 400, batch=16384, lr=1e-3, seed=11)
    torch.cuda.synchronize()
    w = prop.get_weights()
    ws.mask = 0x81  # techniques 1 and 8
    _window(ws, 12_000_000, 4096, mlp=w)
