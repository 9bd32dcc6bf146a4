"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (its tuned queue, the full image and sample count), on
sampled outputs the oracle computes one by one: a window of sample indices
of every (technique, direction) stream, compared record by record.  The
tiny Cornell workload is compared whole."""
import numpy as np
import pytest

from paper_2406_16302_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _window(ws, s0, n, max_div=1e-3):
    from gpu_parity import compare_records, gpu_residual, oracle_residual
    g = gpu_residual(ws, records=True, s0=s0, s1=s0 + n)
    o = oracle_residual(ws, records=True, s0=s0, s1=s0 + n)
    c = compare_records(g["records"], o["records"])
    div = (c["value_mismatch"] + c["missing_on_gpu"] + c["extra_on_gpu"]) / max(c["oracle"], 1)
    print(ws.name, "window [%d, %d)" % (s0, s0 + n), c)
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


def test_clutter_workload_window():
    # 512x512, depth 5, 64 spp: the benchmark's workload
    ws = scenes.clutter_motion()
    _window(ws, 9_000_000, 16384)


def test_material_edit_workload_window():
    # 1024x1024, depth 6, 32 spp, 983k triangles
    ws = scenes.material_edit()
    _window(ws, 20_000_000, 8192)
