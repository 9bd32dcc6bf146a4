"""Helpers for the GPU-vs-oracle parity tests (same Philox streams)."""
import numpy as np

import oracle
from paper_2406_16302_amd import native
from paper_2406_16302_amd.scenes import EDIT_MATERIAL


def gpu_residual(ws, spp=None, depth=None, seed=None, mask=None, s0=0, s1=-1, records=False, queue_cap=0,
                 stats=False, scene=None, mlp=None, proposal=None, train_records=None):
    import torch
    sc = scene or native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    flags = 0
    if ws.two_way and ws.edit.kind != EDIT_MATERIAL:
        flags |= native.FLAG_TWO_WAY
    if records:
        flags |= native.FLAG_RECORDS
    if mlp is not None and proposal is None:
        proposal = native.Proposal(sc, mlp)
    p = native.Params.make(spp or ws.spp, depth or ws.depth, seed if seed is not None else ws.seed,
                           mask=mask or ws.mask, flags=flags, sample_begin=s0, sample_end=s1, queue_cap=queue_cap,
                           proposal=proposal, train_records=train_records)
    stats = stats or train_records is not None
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    st = native.render_residual(sc, ed, p, out, stats=stats)
    torch.cuda.synchronize()
    res = {"image": out.cpu().numpy().astype(np.float64), "stats": st}
    if records:
        res["records"] = sc.records()
    return res


def oracle_residual(ws, spp=None, depth=None, seed=None, mask=None, s0=0, s1=-1, records=False, threads=8, mlp=None):
    o = oracle.OracleScene(ws.scene)
    kw = dict(spp=spp or ws.spp, depth=depth or ws.depth, seed=seed if seed is not None else ws.seed,
              mask=mask or ws.mask, s0=s0, s1=s1, threads=1 if records else threads, records=records, mlp=mlp)
    return oracle.residual_for(ws, o, **kw)


def rel_l2(a, b):
    return float(np.sqrt(((a - b) ** 2).sum()) / max(np.sqrt((b ** 2).sum()), 1e-30))


def compare_records(g, o, rtol=1e-3, atol_rel=1e-6):
    """Match per-path records by (dir, tech, sample, pair); return counts."""
    gk = {}
    for r in g:
        key = (int(r[0]), int(r[1]), int(r[2]), int(r[3]))
        gk[key] = (int(r[4]), np.frombuffer(r[5:8].tobytes(), np.float32).astype(np.float64))
    scale = max(np.abs(o["val"]).max(), 1e-30) if len(o) else 1.0
    ok = mism = miss = 0
    ok_keys = set()
    for r in o:
        key = (int(r["dir"]), int(r["tech"]), int(r["sample"]), int(r["pair"]))
        if key not in gk:
            miss += 1
            continue
        pix, val = gk[key]
        ok_keys.add(key)
        if pix == int(r["pixel"]) and np.all(np.abs(val - r["val"]) <= rtol * np.abs(r["val"]) + atol_rel * scale):
            ok += 1
        else:
            mism += 1
    extra = sum(1 for k, (pix, val) in gk.items() if k not in ok_keys and pix >= 0)
    return {"oracle": len(o), "gpu": len(g), "match": ok, "value_mismatch": mism, "missing_on_gpu": miss,
            "extra_on_gpu": extra}
