#!/usr/bin/env python3
"""Benchmark of the residual path estimator on one MI355X.

Default run (the headline line): the batched animation, the largest of the
workloads -- 32 consecutive frames of the clutter scene's moving sphere along
a seeded Bezier curve, each a residual against the previous frame, images of
256^2..1024^2 (16.8 M pixels), 16 samples per pixel per technique and
direction, depth 5, all seven techniques, both directions, one captured
hipGraph per step.  A step is one replay of that graph: start sampling ->
walks -> MIS / mapping / evaluation in both frames -> tile splat, for every
job.

Next to it, in "workloads", the other configurations, each timed the same
way, with the roofline of its dominant kernel and of its walk phase, and
with the equal-time residual MSE of the estimator against the path-tracing
baselines (correlated, from scratch), the ablations (mapping off) and the
learned proposal, all against a reference residual of 64 times the budget:
  clutter_motion   ~110k triangles, moving 20,480-triangle sphere, 512^2, d5, 64 spp
  material_edit    983k triangles, GGX edit, 1024^2, d6, 32 spp, techniques 1-3
  proposal         the material edit with technique 8 (MLP trained on the GPU)
  cornell_sweep    Cornell box, displacement sweep with and without mapping
Equal-time MSE: each method's MSE at its own budget, scaled by its device
time to the estimator's (MSE x time is constant for an unbiased Monte Carlo
estimator), so MSE_equal_time = MSE * t_method / t_estimator.  The denoised
residual (biased) is listed at its own budget and time.

The CPU oracle is timed on the host cores (all of them, and one) on bounded
samples of the clutter workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

METRIC = "residual paths/s & Mrays/s at 1 GPU; equal-time residual MSE vs plain GPU path"
HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES = 112, 48  # 4-wide node: six box planes and the links (its padding is not read)
KERNEL_NAMES = {t: "walk_kernel<%d>" % t for t in range(1, 9)}          # start phase of technique t
KERNEL_NAMES.update({16 + t: "walk_task_kernel<%d>" % t for t in range(1, 9)})  # its walk phase
KERNEL_NAMES.update({9: "connect_kernel", 10: "splat", 12: "proposal_pdf_kernel", 13: "t8_start_kernel",
                     14: "start_order_kernel"})
KIDS = sorted(KERNEL_NAMES)
WALK_KIDS = [k for k in KIDS if k <= 8 or k >= 14]
RAY_TYPES = ["closest", "shadow", "camera", "ghost", "map_retrace", "map_visibility"]
HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["rpi_kernels.hip", "rpi_device.h", "rpi_internal.h", "rpi_mlp.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for each CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mse", action="store_true", help="skip the equal-time MSE comparisons")
    ap.add_argument("--sub-steps", type=int, default=5, help="timed steps of each sub-workload")
    ap.add_argument("--tuning", default=None,
                    help="queue_cap,walk_blocks_per_cu,connect_blocks_per_cu: use this launch configuration "
                         "instead of running the autotuner (profiling runs)")
    ap.add_argument("--workload", default="all",
                    choices=["all", "batch", "clutter_motion", "material_edit", "proposal", "cornell_sweep"],
                    help="all (default): the headline batch plus every sub-workload; otherwise one of them "
                         "alone (profiling runs)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only a device-to-device copy of 1 GiB, three times (HBM counter calibration)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- measured HBM traffic
def traffic_file(kernel, workload):
    name = kernel.replace("<", "").replace(">", "")
    return os.path.join(HERE, "profiles", "%s_%s_hbm_traffic.md" % (name, workload))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2406_16302_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, queue_cap):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources with the same
    round size (else None)."""
    try:
        with open(traffic_file(kernel, workload)) as fh:
            m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
        rec = json.loads(m.group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_hash") != kernel_source_hash() or \
            rec.get("queue_cap") != queue_cap:
        return None
    return rec.get("traffic_bytes_per_launch")


def measured_valu(workload, queue_cap):
    """VALU utilisation per kernel group from the committed rocprofv3 counter
    summary (SQ_INSTS_VALU over the dispatch time against the chip's wave64
    issue rate; SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU) for the
    lanes), if it was taken on the current kernel sources with the same round
    size (else {})."""
    try:
        with open(os.path.join(HERE, "profiles", "valu_utilisation_%s.md" % workload)) as fh:
            m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
        rec = json.loads(m.group(1))
    except (OSError, AttributeError, ValueError):
        return {}
    if rec.get("source_hash") != kernel_source_hash() or rec.get("queue_cap") != queue_cap:
        return {}
    return rec.get("groups", {})


def copy_only():
    import torch
    n = 1 << 28  # float32 elements: 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}), flush=True)


# ----------------------------------------------------------------- rooflines
_ACHIEVABLE = []


def achievable_hbm_gbs():
    """HBM bandwidth a plain device copy reaches here: 1 GiB copied five
    times, (bytes read + bytes written) / the median HIP-event time."""
    if not _ACHIEVABLE:
        import torch
        n = 1 << 28  # float32 elements: 1 GiB
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        del a, b
        torch.cuda.empty_cache()
        _ACHIEVABLE.append(2.0 * 4 * n / (float(np.median(ts)) / 1e3) / 1e9)
    return _ACHIEVABLE[0]


def kernel_bytes(cw, k):
    return cw["kernel_nodes"][k] * NODE_BYTES + cw["kernel_tris"][k] * TRI_BYTES + cw["kernel_bytes_written"][k]


def rooflines(cw, kms, klaunch, steps, workload, queue_cap):
    """The dominant kernel's roofline and the walk phase's (all start- and
    walk-phase kernels together): algorithmic bytes per launch (BVH nodes x
    112 B + triangles x 48 B + record bytes written, counted by the
    instrumented pass) / the HIP-event-timed launch duration, against the
    published peak and against what a device copy reaches; with each, the
    VALU utilisation of the committed counter summary (null once the kernel
    sources or the round size differ)."""
    kid = max(KIDS, key=lambda k: kms[k])
    launches = max(klaunch[kid] / steps, 1)
    avg_ms = kms[kid] / max(klaunch[kid], 1)
    kb = kernel_bytes(cw, kid)
    achieved = (kb / launches) / (avg_ms / 1e3) / 1e9
    top = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "achievable": round(achievable_hbm_gbs(), 1),
           "frac_of_achievable": round(achieved / achievable_hbm_gbs(), 4),
           "traffic": measured_traffic(KERNEL_NAMES[kid], workload, queue_cap),
           "kernel": KERNEL_NAMES[kid], "avg_launch_ms": round(avg_ms, 4),
           "algorithmic_bytes_per_launch": int(kb / launches),
           "device_time_share": round(float(kms[kid] / kms[KIDS].sum()), 3)}
    valu = measured_valu(workload, queue_cap)
    top["valu"] = valu.get(KERNEL_NAMES[kid])
    wb = sum(kernel_bytes(cw, k) for k in WALK_KIDS)
    wms = float(sum(kms[k] for k in WALK_KIDS)) / steps
    wach = wb / (wms / 1e3) / 1e9 if wms > 0 else 0.0
    walk = {"bound": "hbm", "achieved": round(wach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(wach / HBM_PEAK_GBS, 4), "achievable": round(achievable_hbm_gbs(), 1),
            "frac_of_achievable": round(wach / achievable_hbm_gbs(), 4),
            "kernels": "walk_kernel<t> + walk_task_kernel<t>",
            "ms_per_step": round(wms, 2), "algorithmic_bytes_per_step": int(wb),
            "device_time_share": round(float(sum(kms[k] for k in WALK_KIDS) / kms[KIDS].sum()), 3),
            "valu": valu.get("walk_phase")}
    return top, walk


# ----------------------------------------------------------------- workloads
def make_workload(name):
    from paper_2406_16302_amd import scenes
    if name in ("material_edit", "proposal"):
        return scenes.material_edit()
    return scenes.clutter_motion()


def set_launch(native, sc, ed, params, args):
    if args.tuning:
        q, wb, cb = (int(x) for x in args.tuning.split(","))
        native.set_tuning(sc, q, wb, cb)
        return {"queue_cap": q, "walk_blocks_per_cu": wb, "connect_blocks_per_cu": cb}
    t = native.autotune(sc, ed, params)
    return {k: t[k] for k in ("queue_cap", "walk_blocks_per_cu", "connect_blocks_per_cu")}


def time_residual(native, sc, ed, params, steps, warmup, out):
    """Warmup, then `steps` timed calls with per-kernel HIP events; returns
    (ms per step by the host clock, per-kernel ms, launches, paths/step)."""
    import torch
    for _ in range(warmup):
        native.render_residual(sc, ed, params(0), out)
    torch.cuda.synchronize()
    kms, kl, paths = np.zeros(32), np.zeros(32), []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = native.render_residual(sc, ed, params(native.FLAG_TIME_KERNELS), out, stats=True)
        kms += np.array(st["kernel_ms"])
        kl += np.array(st["kernel_launches"])
        paths.append(st["paths"])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, kms, kl, float(np.mean(paths))


def device_ms(fn, reps=3):
    """Median wall time of fn() up to the end of its device work, after one
    untimed call (every method is timed the same way, allocations included)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def mse(a, b):
    return float(((a.double() - b.double()) ** 2).mean().item())


def reference_residual(native, sc, ed, make, n, seed0):
    """Mean of n estimator renders with independent seeds (n x the budget)."""
    import torch
    acc = torch.zeros((sc.height, sc.width, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    for k in range(n):
        native.render_residual(sc, ed, make(seed0 + 7919 * k), out)
        acc += out.double()
    torch.cuda.synchronize()
    return (acc / n).float()


def equal_time(methods, t_ref):
    """methods: name -> (mse, ms) at each method's own budget; returns
    name -> {mse, ms, mse_equal_time (scaled to t_ref), efficiency vs the estimator}."""
    out = {}
    base = methods["residual"][0] * methods["residual"][1]
    for k, (m, ms) in methods.items():
        out[k] = {"mse": m, "ms": round(ms, 3), "mse_equal_time": m * ms / t_ref,
                  "efficiency_vs_residual": round(base / (m * ms), 4) if m > 0 else None}
    return out


def pt_baselines(native, sc, ed, spp, depth, ref, t_res, seed):
    """Correlated path tracing and path tracing from scratch (I_new - I_old),
    at a budget near the estimator's device time."""
    import torch
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    res = {}
    for name, corr in (("correlated_pt", True), ("pt_scratch", False)):
        p1 = native.Params.make(spp, depth, seed)
        t1 = device_ms(lambda: native.render_frame_difference(sc, ed, corr, p1, out), reps=2)
        s = max(1, int(round(spp * t_res / max(t1, 1e-3))))
        s = min(s, 4096)
        p = native.Params.make(s, depth, seed)
        ms = device_ms(lambda: native.render_frame_difference(sc, ed, corr, p, out), reps=2)
        res[name] = (mse(out, ref), ms, s)
    return res


def bench_single(name, args):
    """One residual workload: timed steps, rooflines, equal-time MSE."""
    import torch
    from paper_2406_16302_amd import native
    ws = make_workload(name)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    material = ws.edit.kind == native.EDIT_MATERIAL
    base = 0 if material else native.FLAG_TWO_WAY
    mask, prop, prop_summary = ws.mask, None, None
    if name == "proposal":
        prop, prop_summary = train_proposal(sc, ed, ws)
        mask = (ws.mask & ~0x6) | 0x80

    def params(flags, seed=None, m=None):
        return native.Params.make(ws.spp, ws.depth, ws.seed if seed is None else seed, mask=mask if m is None else m,
                                  flags=base | flags, proposal=prop)

    launch = set_launch(native, sc, ed, params(0), args)
    log("%s: %d triangles, %dx%d, launch %s" % (name, len(ws.scene.indices), sc.width, sc.height, launch))
    cw = native.render_residual(sc, ed, params(native.FLAG_COUNT_WORK), out, stats=True)
    steps = args.steps if args.workload == name else args.sub_steps
    ms, kms, kl, paths = time_residual(native, sc, ed, params, steps, args.warmup, out)
    rays = float(sum(cw["rays"]))
    top, walk = rooflines(cw, kms, kl, steps, name, launch["queue_cap"])
    rec = {"value": round(paths / (ms / 1e3), 1), "unit": "residual paths/s", "ms_per_step": round(ms, 2),
           "steps": steps, "mrays_per_s": round(rays / (ms / 1e3) / 1e6, 1), "paths_per_step": int(paths),
           "rays_per_step": int(rays), "rays_by_type": {k: int(v) for k, v in zip(RAY_TYPES, cw["rays"])},
           "config": {"workload": name, "triangles": int(len(ws.scene.indices)),
                      "object_triangles": int((ws.scene.tri_object == 1).sum()),
                      "image": "%dx%d" % (sc.width, sc.height), "max_depth": ws.depth, "spp": ws.spp,
                      "techniques": {"clutter_motion": "1-7", "material_edit": "1-3", "proposal": "1, 8"}[name],
                      "two_way": not material, "launch": launch},
           "kernel_ms_per_step": {KERNEL_NAMES[k]: round(kms[k] / steps, 2) for k in KIDS if kms[k] > 0},
           "roofline": top, "roofline_walk_phase": walk}
    log("%s: %.1f ms/step, %.1f M paths/s" % (name, ms, rec["value"] / 1e6))
    if prop_summary is not None:
        rec["proposal"] = prop_summary
    if not args.no_mse:
        t_res = device_ms(lambda: native.render_residual(sc, ed, params(0), out), reps=3)
        ref_mask = ws.mask  # the plain estimator is the reference for the proposal too
        ref = reference_residual(native, sc, ed, lambda s: params(0, s, ref_mask), 64, 9001)
        native.render_residual(sc, ed, params(0), out)
        methods = {"residual": (mse(out, ref), t_res)}
        spp_used = {"residual": ws.spp}
        # residual-aware allocation of the techniques' sample counts (pilot of spp/8)
        counts = native.allocate_samples(sc, ed, params(0), pilot_spp=max(2, ws.spp // 8))
        pal = native.Params.make(ws.spp, ws.depth, ws.seed, mask=mask, flags=base, proposal=prop,
                                 technique_spp=counts)
        t_al = device_ms(lambda: native.render_residual(sc, ed, pal, out), reps=3)
        native.render_residual(sc, ed, pal, out)
        methods["residual_allocated"] = (mse(out, ref), t_al)
        spp_used["residual_allocated"] = counts
        if name == "proposal":
            t_plain = device_ms(lambda: native.render_residual(sc, ed, params(0, None, ref_mask), out), reps=3)
            native.render_residual(sc, ed, params(0, None, ref_mask), out)
            methods["plain_estimator"] = (mse(out, ref), t_plain)
            spp_used["plain_estimator"] = ws.spp
            # technique 8 added to techniques 1-3 as one more strategy, the
            # counts of all four allocated from a pilot
            madd = ws.mask | 0x80
            cadd = native.allocate_samples(sc, ed, params(0, None, madd), pilot_spp=max(2, ws.spp // 8))
            padd = native.Params.make(ws.spp, ws.depth, ws.seed, mask=madd, flags=base, proposal=prop,
                                      technique_spp=cadd)
            t_add = device_ms(lambda: native.render_residual(sc, ed, padd, out), reps=3)
            native.render_residual(sc, ed, padd, out)
            methods["added_to_1_3_allocated"] = (mse(out, ref), t_add)
            spp_used["added_to_1_3_allocated"] = cadd
        if not material:
            pnm = native.Params.make(ws.spp, ws.depth, ws.seed, mask=mask, flags=base | native.FLAG_NO_MAPPING)
            t_nm = device_ms(lambda: native.render_residual(sc, ed, pnm, out), reps=2)
            native.render_residual(sc, ed, pnm, out)
            methods["residual_no_mapping"] = (mse(out, ref), t_nm)
            spp_used["residual_no_mapping"] = ws.spp
        if not material and name != "proposal":
            # accepted pairs weighted by the balance heuristic over both frames' strategies
            pbl = native.Params.make(ws.spp, ws.depth, ws.seed, mask=mask, flags=base | native.FLAG_BALANCE)
            t_bl = device_ms(lambda: native.render_residual(sc, ed, pbl, out), reps=2)
            native.render_residual(sc, ed, pbl, out)
            methods["residual_balance"] = (mse(out, ref), t_bl)
            spp_used["residual_balance"] = ws.spp
        if name != "proposal":
            # the residual-aware denoiser on the same budget: two half estimates, then the filter
            N = ws.spp * sc.width * sc.height
            ha, hb, dn = torch.zeros_like(out), torch.zeros_like(out), torch.zeros_like(out)
            pa = native.Params.make(ws.spp, ws.depth, ws.seed, mask=mask, flags=base, sample_end=N // 2)
            pb = native.Params.make(ws.spp, ws.depth, ws.seed, mask=mask, flags=base, sample_begin=N // 2)

            def halves_and_filter():
                native.render_residual(sc, ed, pa, ha)
                native.render_residual(sc, ed, pb, hb)
                native.denoise_residual(sc, ed, ha, hb, dn)
            t_dn = device_ms(halves_and_filter, reps=2)
            methods["residual_denoised"] = (mse(dn, ref), t_dn)
            spp_used["residual_denoised"] = ws.spp
            for k, (m, t, s) in pt_baselines(native, sc, ed, 4, ws.depth, ref, t_res, 4242).items():
                methods[k] = (m, t)
                spp_used[k] = s
        et = equal_time(methods, t_res)
        for k in et:
            et[k]["spp"] = spp_used[k]
        rec["equal_time_mse"] = {"reference": "mean of 64 renders of the plain estimator (techniques %s), "
                                              "independent seeds" % rec["config"]["techniques"].replace(
                                                  "1, 8", "1-3"),
                                 "methods": et}
        log("%s equal-time MSE: %s" % (name, {k: "%.3g" % v["mse_equal_time"] for k, v in et.items()}))
    return rec


def train_proposal(sc, ed, ws):
    """Records from the plain estimator (10 M), then Adam on the GPU
    (20 epochs of batches of 16,384)."""
    import torch
    from paper_2406_16302_amd import native
    cap = 10_000_000
    buf = torch.zeros((cap, 10), dtype=torch.float32, device="cuda")
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    n = 0
    seed = 777
    while n < cap:  # record passes until the buffer holds 10 M records
        st = native.render_residual(sc, ed, native.Params.make(ws.spp, ws.depth, seed, mask=0x07, flags=0,
                                                               train_records=buf[n:]), out, stats=True)
        n = min(cap, n + st["train_records"])
        seed += 1
        if st["train_records"] == 0:
            break
    t1 = time.perf_counter()
    prop = native.Proposal(sc, None, seed=3)
    batch = 16384
    steps = max(200, 20 * n // batch)  # 20 epochs
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prop.train(buf, n, steps, batch=batch, lr=1e-3, seed=11, losses=losses)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    L = losses.cpu().numpy()
    flop = 3 * 22272 * batch * steps
    summary = {"records": int(n), "record_passes": seed - 777, "collect_s": round(t1 - t0, 3),
               "train_steps": steps, "batch": batch, "train_s": round(t3 - t2, 3),
               "train_records_per_s": round(batch * steps / (t3 - t2), 1),
               "train_tflops": round(flop / (t3 - t2) / 1e12, 3), "loss_first": round(float(L[:20].mean()), 4),
               "loss_last": round(float(L[-20:].mean()), 4)}
    log("proposal: %s" % summary)
    del buf
    return prop, summary


def cornell_sweep(args):
    """Config-1 hard cases (the paper's Table 2 trends): the Cornell box with
    the cube resting on the floor, its displacement scaled from 0.1x to 3x,
    estimator with and without path mapping, correlated PT and PT from
    scratch, equal-time MSE against a 64x-budget estimator reference.  Run at
    256x256 (16 spp, depth 3) so that the device times are not launch-bound."""
    import torch
    from paper_2406_16302_amd import native, scenes
    rows = []
    for scale in (0.1, 0.3, 1.0, 3.0):
        off = (0.1 * scale, 0.0, 0.05 * scale)
        ws = scenes.cornell_motion(width=256, height=256, spp=16, depth=3, lift=0.0, offset=off)
        sc = native.Scene(ws.scene)
        native.set_tuning(sc, 1 << 22, 16, 16)
        ed = native.Edit(sc, ws.edit)
        out = torch.zeros((256, 256, 3), dtype=torch.float32, device="cuda")
        mk = lambda s, fl=0: native.Params.make(ws.spp, ws.depth, s, flags=native.FLAG_TWO_WAY | fl)
        ref = reference_residual(native, sc, ed, mk, 64, 5003)
        p0 = mk(ws.seed)
        t_res = device_ms(lambda: native.render_residual(sc, ed, p0, out), reps=3)
        native.render_residual(sc, ed, p0, out)
        methods = {"residual": (mse(out, ref), t_res)}
        counts = native.allocate_samples(sc, ed, p0, pilot_spp=4)
        pa = native.Params.make(ws.spp, ws.depth, ws.seed, flags=native.FLAG_TWO_WAY, technique_spp=counts)
        t_al = device_ms(lambda: native.render_residual(sc, ed, pa, out), reps=3)
        native.render_residual(sc, ed, pa, out)
        methods["residual_allocated"] = (mse(out, ref), t_al)
        pn = mk(ws.seed, native.FLAG_NO_MAPPING)
        t_nm = device_ms(lambda: native.render_residual(sc, ed, pn, out), reps=3)
        native.render_residual(sc, ed, pn, out)
        methods["residual_no_mapping"] = (mse(out, ref), t_nm)
        pb = mk(ws.seed, native.FLAG_BALANCE)
        t_bl = device_ms(lambda: native.render_residual(sc, ed, pb, out), reps=3)
        native.render_residual(sc, ed, pb, out)
        methods["residual_balance"] = (mse(out, ref), t_bl)
        for k, (m, t, s) in pt_baselines(native, sc, ed, 16, ws.depth, ref, t_res, 4243).items():
            methods[k] = (m, t)
        et = equal_time(methods, t_res)
        rows.append({"displacement": [round(x, 4) for x in off],
                     "mse_equal_time": {k: v["mse_equal_time"] for k, v in et.items()},
                     "efficiency_vs_residual": {k: v["efficiency_vs_residual"] for k, v in et.items()},
                     "ms": {k: v["ms"] for k, v in et.items()}})
        log("sweep x%.1f: %s" % (scale, rows[-1]["efficiency_vs_residual"]))
        del sc, ed
    return {"config": {"workload": "cornell_sweep", "image": "256x256", "spp": 16, "max_depth": 3,
                       "object": "cube resting on the floor", "techniques": "1-7", "two_way": True},
            "rows": rows}


def bench_batch(args, steps):
    """The headline: 32 Bezier frames in one captured graph per step."""
    import torch
    from paper_2406_16302_amd import native, scenes
    ws = scenes.clutter_motion(spp=16)
    sc = native.Scene(ws.scene)
    jobs = scenes.bezier_jobs()
    outs = [torch.zeros((j["height"], j["width"], 3), dtype=torch.float32, device="cuda") for j in jobs]
    jl = [{"pose_old": j["pose_old"], "pose_new": j["pose_new"], "out": o} for j, o in zip(jobs, outs)]

    def params(flags=0, seed=None):
        return native.Params.make(16, ws.depth, ws.seed if seed is None else seed, mask=ws.mask,
                                  flags=native.FLAG_TWO_WAY | flags)

    if args.tuning:
        q, wb, cb = (int(x) for x in args.tuning.split(","))
        native.set_tuning(sc, q, wb, cb)
    t0 = time.perf_counter()
    st = native.render_residual_batch(sc, jl, params(), stats=True)  # autotune on the largest job, capture
    log("batch: first call (autotune + capture) %.1f s, %d paths" % (time.perf_counter() - t0, st["paths"]))
    for _ in range(args.warmup):
        native.render_residual_batch(sc, jl, params())
    torch.cuda.synchronize()
    paths = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = native.render_residual_batch(sc, jl, params(), stats=True)
        paths.append(st["paths"])
        log("batch step: %.1f ms device time" % st["milliseconds"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    # the same plan and kernels launched directly: per-kernel HIP events
    # (one step) and the instrumented pass (algorithmic bytes, rays)
    stt = native.render_residual_batch(sc, jl, params(native.FLAG_TIME_KERNELS), stats=True)
    cw = native.render_residual_batch(sc, jl, params(native.FLAG_COUNT_WORK), stats=True)
    kms, kl = np.array(stt["kernel_ms"]), np.array(stt["kernel_launches"])
    tun = native.get_tuning(sc)
    top, walk = rooflines(cw, kms, kl, 1, "batch", tun["queue_cap"])
    rays = float(sum(cw["rays"]))
    pix = sum(j["width"] * j["height"] for j in jobs)
    rec = {"value": round(float(np.mean(paths)) / (ms / 1e3), 1), "ms_per_step": round(ms, 2),
           "mrays_per_s": round(rays / (ms / 1e3) / 1e6, 1), "paths_per_step": int(np.mean(paths)),
           "rays_per_step": int(rays), "rays_by_type": {k: int(v) for k, v in zip(RAY_TYPES, cw["rays"])},
           "config": {"workload": "batch_bezier_32", "jobs": len(jobs), "pixels": pix,
                      "image_sizes": sorted({j["width"] for j in jobs}), "spp": 16, "max_depth": ws.depth,
                      "triangles": int(len(ws.scene.indices)), "techniques": "1-7", "two_way": True,
                      "graph": True, "launch": tun},
           "kernel_ms_per_step": {KERNEL_NAMES[k]: round(kms[k], 2) for k in KIDS if kms[k] > 0},
           "kernel_timing": "HIP events around each launch of one direct (non-graph) pass of the same plan",
           "roofline": top, "roofline_walk_phase": walk}
    if not args.no_mse:
        # batched vs the same jobs one after another (plain per-job calls), equal time
        import torch as _t
        ed_list = []
        t_seq = 0.0
        for i, j in enumerate(jobs):
            one = [{"pose_old": j["pose_old"], "pose_new": j["pose_new"], "out": outs[i]}]
            p1 = native.Params.make(16, ws.depth, ws.seed, mask=ws.mask, flags=native.FLAG_TWO_WAY, job=i)
            native.render_residual_batch(sc, one, p1)  # capture this shape
            _t.cuda.synchronize()
            t_seq += device_ms(lambda: native.render_residual_batch(sc, one, p1), reps=1)
        rec["batched_vs_sequential"] = {"batched_ms": round(ms, 2), "sequential_ms": round(t_seq, 2),
                                        "speedup": round(t_seq / ms, 3),
                                        "mse_ratio_at_equal_time": round(ms / t_seq, 4),
                                        "note": "same estimator and samples: at equal time the MSE scales "
                                                "with the time per step"}
        del ed_list
    return rec


def cpu_baseline(target_s):
    """The oracle as it stands on the headline workload: the first n sample
    indices of every (technique, direction) stream of the animation's first
    job (its poses, image size and Philox job word), on all host cores, then
    on one core."""
    import oracle
    from paper_2406_16302_amd import scenes
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    ws = scenes.clutter_motion(spp=16)
    j = scenes.bezier_jobs()[0]
    o = oracle.OracleScene(ws.scene.with_resolution(j["width"], j["height"]))

    def run(th, target):
        n = 256
        while True:
            t0 = time.perf_counter()
            r = o.render_residual(16, ws.depth, ws.seed, pose_old=j["pose_old"], pose_new=j["pose_new"], s0=0,
                                  s1=n, threads=th, job=0)
            dt = time.perf_counter() - t0
            if dt >= target * 0.5 or n >= (1 << 22):
                return n, r["stats"], dt
            n = int(n * max(2.0, min(16.0, target / max(dt, 1e-3))))
    n, st, dt = run(threads, target_s)
    n1, st1, dt1 = run(1, target_s)
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    what = "job 0 of the batched animation (%dx%d, 16 spp, depth 5, techniques 1-7, both directions)" % (
        j["width"], j["height"])
    return {"value": st["paths"] / dt, "unit": "residual paths/s", "cores": int(threads), "kind": "oracle",
            "mrays_per_s": round(st["rays"] / dt / 1e6, 3),
            "sample": "first %d sample indices of each of the 14 (technique, direction) streams of %s "
                      "(%d connected paths, %.1f s)" % (n, what, st["paths"], dt),
            "single_core": {"value": st1["paths"] / dt1, "unit": "residual paths/s", "cores": 1,
                            "mrays_per_s": round(st1["rays"] / dt1 / 1e6, 3),
                            "sample": "first %d sample indices of each stream (%d paths, %.1f s)" %
                                      (n1, st1["paths"], dt1)},
            "cpu": cpu}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (the estimator would shard "
              "sample ranges across GPUs, which is design only here)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_only:
        copy_only()
        return
    t_start = time.perf_counter()
    if args.workload in ("clutter_motion", "material_edit", "proposal"):
        rec = bench_single(args.workload, args)
        line = {"metric": METRIC, "n_gpus": 1, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
        line.update(rec)
        print(json.dumps(line), flush=True)
        return
    if args.workload == "cornell_sweep":
        print(json.dumps(cornell_sweep(args)), flush=True)
        return
    head = bench_batch(args, args.steps)
    line = {"metric": METRIC, "value": head.pop("value"), "unit": "residual paths/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded procedural scenes, random Bezier poses)"}
    line["config"] = head.pop("config")
    line.update(head)
    if args.workload == "all":
        subs = {}
        for name in ("clutter_motion", "material_edit", "proposal"):
            subs[name] = bench_single(name, args)
        subs["cornell_sweep"] = cornell_sweep(args) if not args.no_mse else None
        line["workloads"] = subs
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
