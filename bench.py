#!/usr/bin/env python3
"""Benchmark of the residual path estimator on one MI355X.

A step is one full pass of the estimator (all seven techniques, both frames,
start sampling -> walks -> MIS/mapping/evaluation -> tile splat) over the
clutter-motion workload: ~110k static triangles, a moving 20,480-triangle
sphere, 512x512, depth 5, 64 samples per pixel per technique per direction.

Prints one JSON line: residual paths/s (value), Mrays/s, the roofline entry of
the dominant kernel (algorithmic bytes from the instrumented variant / its
HIP-event-timed launch duration) and the CPU oracle timed on a bounded sample
of the same workload.
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
NODE_BYTES, TRI_BYTES = 64, 48
KERNEL_NAMES = {t: "walk_kernel<%d>" % t for t in range(1, 9)}          # start phase of technique t
KERNEL_NAMES.update({16 + t: "walk_task_kernel<%d>" % t for t in range(1, 9)})  # its walk phase
KERNEL_NAMES.update({9: "connect_kernel", 10: "splat", 12: "proposal_pdf_kernel", 13: "t8_start_kernel"})
KIDS = sorted(KERNEL_NAMES)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="a reduced workload (quick checks only)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only a device-to-device copy of 1 GiB, three times (HBM counter calibration)")
    return ap.parse_args()


HERE = os.path.dirname(os.path.abspath(__file__))
def traffic_file(kernel):
    name = kernel.replace("<", "").replace(">", "")
    return os.path.join(HERE, "profiles", "%s_clutter_motion_512x512_d5_hbm_traffic.md" % name)
KERNEL_SOURCES = ["rpi_kernels.hip", "rpi_device.h", "rpi_internal.h", "rpi_mlp.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2406_16302_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    try:
        with open(traffic_file(kernel)) as fh:
            m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
        rec = json.loads(m.group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


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


def workload(small):
    from paper_2406_16302_amd import scenes
    if small:
        return scenes.clutter_motion(width=128, height=128, spp=8)
    return scenes.clutter_motion()


def cpu_baseline(ws, target_s):
    """The oracle as it stands, on the first n sample indices of every
    (technique, direction) stream of the same workload, all host cores."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    o = oracle.OracleScene(ws.scene)
    n = 256
    while True:
        t0 = time.perf_counter()
        r = oracle.residual_for(ws, o, s0=0, s1=n, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s * 0.5 or n >= (1 << 22):
            break
        n = int(n * max(2.0, min(16.0, target_s / max(dt, 1e-3))))
    paths = r["stats"]["paths"]
    return {"value": paths / dt, "unit": "residual paths/s", "cores": int(threads), "kind": "oracle",
            "sample": "first %d sample indices of each of the 14 (technique, direction) streams of the "
                      "clutter-motion 512x512 d5 workload (%d connected paths, %.1f s)" % (n, paths, dt)}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_only:
        copy_only()
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (the estimator shards "
              "sample ranges across GPUs only by design, see DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_16302_amd import native
    ws = workload(args.small)
    sc = native.Scene(ws.scene)
    ed = native.Edit(sc, ws.edit)
    out = torch.zeros((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
    base = native.FLAG_TWO_WAY

    def params(flags):
        return native.Params.make(ws.spp, ws.depth, ws.seed, mask=ws.mask, flags=base | flags)

    log("scene built: %d triangles, %dx%d" % (len(ws.scene.indices), sc.width, sc.height))
    # instrumented pass (untimed): rays by type and algorithmic work per kernel
    cw = native.render_residual(sc, ed, params(native.FLAG_COUNT_WORK), out, stats=True)
    log("instrumented pass: %d paths, %d rays" % (cw["paths"], sum(cw["rays"])))
    for _ in range(args.warmup):
        native.render_residual(sc, ed, params(0), out)
    torch.cuda.synchronize()
    log("warmup done")
    kms = np.zeros(32)
    klaunch = np.zeros(32)
    paths = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = native.render_residual(sc, ed, params(native.FLAG_TIME_KERNELS), out, stats=True)
        kms += np.array(st["kernel_ms"])
        klaunch += np.array(st["kernel_launches"])
        paths.append(st["paths"])
        log("step: %.1f ms device time" % st["milliseconds"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    paths_per_step = float(np.mean(paths))
    rays_per_step = float(sum(cw["rays"]))
    value = paths_per_step / (ms_per_step / 1e3)

    # dominant kernel: largest share of device time; algorithmic bytes per launch =
    # (BVH nodes x 64 B + triangles x 48 B + record bytes written) of that kernel
    kid = max(KIDS, key=lambda k: kms[k])
    kbytes = (cw["kernel_nodes"][kid] * NODE_BYTES + cw["kernel_tris"][kid] * TRI_BYTES
              + cw["kernel_bytes_written"][kid])
    launches = max(klaunch[kid] / args.steps, 1)
    avg_ms = kms[kid] / max(klaunch[kid], 1)
    achieved = (kbytes / launches) / (avg_ms / 1e3) / 1e9
    traffic = None if args.small else measured_traffic(KERNEL_NAMES[kid])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[kid], "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": int(kbytes / launches),
                "device_time_share": round(float(kms[kid] / kms[KIDS].sum()), 3)}
    line = {"metric": METRIC, "value": round(value, 1), "unit": "residual paths/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "clutter_motion" + ("_small" if args.small else ""),
                       "triangles": int(len(ws.scene.indices)),
                       "object_triangles": int((ws.scene.tri_object == 1).sum()),
                       "image": "%dx%d" % (sc.width, sc.height), "max_depth": ws.depth, "spp": ws.spp,
                       "techniques": "1-7", "two_way": True},
            "mrays_per_s": round(rays_per_step / (ms_per_step / 1e3) / 1e6, 1),
            "paths_per_step": int(paths_per_step), "rays_per_step": int(rays_per_step),
            "rays_by_type": {k: int(v) for k, v in zip(["closest", "shadow", "camera", "ghost", "map_retrace",
                                                         "map_visibility"], cw["rays"])},
            "kernel_ms_per_step": {KERNEL_NAMES[k]: round(kms[k] / args.steps, 2) for k in KIDS if kms[k] > 0},
            "roofline": roofline}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(ws, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
