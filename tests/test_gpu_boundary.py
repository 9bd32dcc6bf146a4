"""The boundary's options through the C ABI on the GPU, against the oracle
on the same Philox streams: per-technique images (fig. importance_sample),
path mapping off (fig. ablat_pathmapping), the splat tile edge, PyTorch's
caching allocator behind the allocator hook, and rpi_sync_status."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _render(sc, ed, p):
    from paper_2406_16302_amd import native
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    st = native.render_residual(sc, ed, p, out, stats=True)
    native.sync_status()
    return out, st


def test_per_technique_images_match_oracle_and_sum_to_total():
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=32, height=32, depth=5, spp=8)
    print("cornell_motion 32x32 d5 spp8 per-technique", flush=True)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    timg = torch.full((8, 32, 32, 3), 7.0, dtype=torch.float32, device="cuda")  # overwritten
    p = native.Params.make(ws.spp, ws.depth, ws.seed, technique_images=timg)
    out, st = _render(sc, ed, p)
    t = timg.cpu()
    # the total is the technique images added in technique order, bit for bit
    acc = torch.zeros_like(t[0])
    for k in range(8):
        acc = acc + t[k]
    assert torch.equal(acc, out.cpu())
    assert torch.count_nonzero(t[7]) == 0  # technique 8 did not run
    o = oracle.residual_for(ws, oracle.OracleScene(ws.scene), threads=8, per_tech=True)
    assert rel_l2(out.cpu().numpy().astype(np.float64), o["image"]) < 1e-3
    for k in range(7):
        ref = o["per_tech"][k]
        assert np.abs(ref).sum() > 0, k
        assert rel_l2(t[k].numpy().astype(np.float64), ref) < 1e-3, k
    # the same call without the flag gives the same total up to float rounding
    out2, _ = _render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed))
    assert rel_l2(out2.cpu().numpy().astype(np.float64), out.cpu().numpy().astype(np.float64)) < 1e-5


@pytest.mark.parametrize("name", ["cornell", "clutter"])
def test_mapping_off_matches_oracle(name):
    import oracle
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    if name == "cornell":
        ws = scenes.cornell_motion(width=32, height=32, depth=5, spp=8)
    else:
        ws = scenes.clutter_motion(width=48, height=48, depth=4, spp=4, n_spheres=60)
    print(name, "mapping off", flush=True)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    p = native.Params.make(ws.spp, ws.depth, ws.seed, flags=native.FLAG_TWO_WAY | native.FLAG_NO_MAPPING)
    out, st = _render(sc, ed, p)
    assert st["paths"] > 1000 and st["accepted"] == 0 and st["rejected"][0] == st["paths"]
    o = oracle.residual_for(ws, oracle.OracleScene(ws.scene), threads=8, no_mapping=True)
    assert o["stats"]["unmapped"] == o["stats"]["paths"]
    assert rel_l2(out.cpu().numpy().astype(np.float64), o["image"]) < 1e-3
    # with the mapping the result differs (correlated pairs are subtracted)
    with_map, st2 = _render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed))
    assert st2["accepted"] > 0
    assert rel_l2(with_map.cpu().numpy().astype(np.float64), out.cpu().numpy().astype(np.float64)) > 1e-2


def test_mapping_off_is_rejected_where_it_does_not_apply():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_material(width=16, height=16, depth=4, spp=2)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((16, 16, 3), dtype=torch.float32, device="cuda")
    for flags in (native.FLAG_NO_MAPPING, native.FLAG_NO_MAPPING | native.FLAG_TWO_WAY):
        with pytest.raises(native.RpiError) as e:
            native.render_residual(sc, ed, native.Params.make(2, 4, 1, mask=0x07, flags=flags), out)
        assert e.value.code == -2


def test_splat_is_bitwise_reproducible():
    """The splat sums records in fixed point (integer adds commute): two runs,
    two round sizes (which regroup the records into rounds), both tile edges
    and the allocation-free variant give the same image bit for bit."""
    from paper_2406_16302_amd import native
    ws = scenes.clutter_motion(width=80, height=56, depth=5, spp=8, n_spheres=60)  # ragged tiles
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    imgs = []
    for q, t in ((0, 0), (0, 0), (1 << 16, 0), (4096, 16), (999, 32)):
        imgs.append(_render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, queue_cap=q, tile=t))[0].cpu())
    assert torch.count_nonzero(imgs[0]) > 1000
    for k in range(1, len(imgs)):
        assert torch.equal(imgs[k], imgs[0]), k
    out = torch.full((56, 80, 3), 5.0, dtype=torch.float32, device="cuda")
    native.render_residual_noalloc(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed), out)
    native.sync_status()
    assert torch.equal(out.cpu(), imgs[0])
    # accumulate adds this call's image onto the output
    acc = imgs[0].cuda().clone()
    native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, flags=native.FLAG_TWO_WAY |
                                                      native.FLAG_ACCUMULATE), acc)
    native.sync_status()
    assert torch.equal(acc.cpu(), imgs[0] + imgs[0])


def test_bad_tile_edge_is_rejected():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=40, height=24, depth=4, spp=2)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((24, 40, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(native.RpiError):
        native.render_residual(sc, ed, native.Params.make(2, 4, 1, tile=8), out)


def test_torch_allocator_backs_the_scene_and_workspace():
    from gpu_parity import rel_l2
    from paper_2406_16302_amd import native
    ws = scenes.cornell_motion(width=32, height=32, depth=4, spp=8)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    sc_t = native.Scene(ws.scene, allocator="torch")
    held = torch.cuda.memory_allocated() - before
    assert held > 0  # the scene's BVHs and tables live in torch's pool
    ed_t = native.Edit(sc_t, ws.edit)
    peak0 = torch.cuda.max_memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    a, st = _render(sc_t, ed_t, native.Params.make(ws.spp, ws.depth, ws.seed, queue_cap=1 << 16))
    assert torch.cuda.max_memory_allocated() - torch.cuda.memory_allocated() > 1 << 20  # the workspace came from torch
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    b, _ = _render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, queue_cap=1 << 16))
    assert rel_l2(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) < 1e-5
    del ed_t, sc_t
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before <= 2 * a.numel() * 4 + (1 << 12)
    del peak0


def test_sync_status_reports_ok():
    from paper_2406_16302_amd import native
    native.sync_status()
    s = torch.cuda.Stream()
    native.sync_status(s)


@pytest.mark.parametrize("name", ["cornell_motion", "cornell_material", "cornell_motion_balance"])
def test_unequal_technique_counts_match_oracle(name):
    """Per-technique sample counts (balance heuristic over unequal counts)
    against the oracle on the same Philox streams, record by record; with
    RPI_FLAG_BALANCE the mapped path's strategy sum carries the same count
    ratios."""
    from gpu_parity import compare_records, rel_l2
    import oracle
    from paper_2406_16302_amd import native
    balance = name.endswith("_balance")
    if name.startswith("cornell_motion"):
        ws = scenes.cornell_motion(width=32, height=32, depth=5, spp=4)
        counts = [8, 2, 4, 6, 2, 4, 1, 0]
    else:
        ws = scenes.cornell_material(width=32, height=32, depth=5, spp=4)
        counts = [12, 1, 3, 0, 0, 0, 0, 0]
    print(name, "technique counts", counts, flush=True)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    material = ws.edit.kind == scenes.EDIT_MATERIAL
    flags = (0 if material else native.FLAG_TWO_WAY) | native.FLAG_RECORDS | (native.FLAG_BALANCE if balance else 0)
    out = torch.zeros((32, 32, 3), dtype=torch.float32, device="cuda")
    st = native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, mask=ws.mask, flags=flags,
                                                           technique_spp=counts), out, stats=True)
    per_dir = 1 if material else 2
    assert st["samples"] == per_dir * 32 * 32 * sum(c for t, c in enumerate(counts) if (ws.mask >> t) & 1)
    g = sc.records()
    o = oracle.residual_for(ws, oracle.OracleScene(ws.scene), threads=1, records=True, tech_spp=counts,
                            balance=balance)
    c = compare_records(g, o["records"])
    print(c, flush=True)
    assert c["oracle"] > 1000
    assert c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"] <= 1e-3 * c["oracle"]
    assert rel_l2(out.cpu().numpy().astype(np.float64), o["image"]) < 1e-3


def test_sample_allocation_from_a_pilot():
    """rpi_allocate_samples: one count per enabled technique, none for the
    others; the allocation it returns renders an unbiased residual (the sum
    of the image agrees with equal counts) and, printed, what it gains."""
    from paper_2406_16302_amd import native
    ws = scenes.cornell_material(width=64, height=64, depth=5, spp=8)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    p = native.Params.make(ws.spp, ws.depth, ws.seed, mask=0x07, flags=0)
    counts = native.allocate_samples(sc, ed, p, pilot_spp=4)
    print("allocation", counts, flush=True)
    assert all(c >= 1 for c in counts[:3]) and all(c == 0 for c in counts[3:])
    out = torch.zeros((64, 64, 3), dtype=torch.float32, device="cuda")
    sums = {}
    for label, tc in (("equal", None), ("allocated", counts)):
        v = []
        for k in range(16):
            native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, 500 + k, mask=0x07, flags=0,
                                                              technique_spp=tc), out)
            v.append(out.double().sum().item())
        sums[label] = (np.mean(v), np.std(v, ddof=1) / 4.0)
    (m0, s0), (m1, s1) = sums["equal"], sums["allocated"]
    print(sums, flush=True)
    assert abs(m0 - m1) < 4 * np.hypot(s0, s1)


@pytest.mark.parametrize("name", ["cornell", "clutter"])
def test_balance_across_directions_matches_oracle(name):
    """RPI_FLAG_BALANCE: accepted pairs divided by the strategy sums of both
    frames (the mapped path's sum in the other frame, its ghost crossings on
    the two edges at the moved vertex, |T'| for a re-traced x_1) against the
    oracle on the same Philox streams, record by record."""
    from gpu_parity import compare_records, rel_l2
    import oracle
    from paper_2406_16302_amd import native
    if name == "cornell":
        ws = scenes.cornell_motion(width=32, height=32, depth=5, spp=8)
    else:
        ws = scenes.clutter_motion(width=48, height=48, depth=4, spp=4, n_spheres=60)
    print(name, "balance across directions", flush=True)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    flags = native.FLAG_TWO_WAY | native.FLAG_BALANCE | native.FLAG_RECORDS
    out, st = _render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed, flags=flags))
    assert st["accepted"] > 100
    g = sc.records()
    o = oracle.residual_for(ws, oracle.OracleScene(ws.scene), threads=1, records=True, balance=True)
    c = compare_records(g, o["records"])
    print(c, flush=True)
    assert c["oracle"] > 1000
    assert c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"] <= 1e-3 * c["oracle"]
    assert rel_l2(out.cpu().numpy().astype(np.float64), o["image"]) < 1e-3
    # the weighting changes the image (it is not c = 1/2 in disguise)
    half, _ = _render(sc, ed, native.Params.make(ws.spp, ws.depth, ws.seed))
    assert rel_l2(half.cpu().numpy().astype(np.float64), out.cpu().numpy().astype(np.float64)) > 1e-3


def test_balance_is_rejected_where_it_does_not_apply():
    from paper_2406_16302_amd import native
    ws = scenes.cornell_material(width=16, height=16, depth=4, spp=2)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((16, 16, 3), dtype=torch.float32, device="cuda")
    for flags in (native.FLAG_BALANCE, native.FLAG_BALANCE | native.FLAG_TWO_WAY):
        with pytest.raises(native.RpiError) as e:
            native.render_residual(sc, ed, native.Params.make(2, 4, 1, mask=0x07, flags=flags), out)
        assert e.value.code == -2
    wm = scenes.cornell_motion(width=16, height=16, depth=4, spp=2)
    scm = native.Scene(wm.scene)
    edm = native.Edit(scm, wm.edit)
    with pytest.raises(native.RpiError) as e:
        native.render_residual(scm, edm, native.Params.make(2, 4, 1, flags=native.FLAG_BALANCE), out)
    assert e.value.code == -2
