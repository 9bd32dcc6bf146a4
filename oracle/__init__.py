"""ctypes wrapper around the CPU oracle (oracle.cpp).

Test infrastructure only: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

TECH_MASK_ALL = 0x7F
EDIT_MATERIAL = 1  # edit kind of a material change in the shared input format (rigid motion is 0)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (scalar, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("spp", C.c_int), ("depth", C.c_int), ("mask", C.c_uint32), ("two_way", C.c_int),
                ("seed", C.c_uint64), ("job", C.c_uint32), ("alpha_min", C.c_float),
                ("d_min", C.c_float), ("jac_max", C.c_float), ("c_weight", C.c_float),
                ("s0", C.c_int64), ("s1", C.c_int64), ("threads", C.c_int),
                ("material_mode", C.c_int), ("no_mapping", C.c_int), ("tech_spp", C.c_int32 * 8),
                ("balance", C.c_int)]


RECORD_DTYPE = np.dtype([("dir", "<i4"), ("tech", "<i4"), ("sample", "<u4"), ("k", "<i4"),
                         ("pixel", "<i4"), ("reason", "<i4"), ("n_starts", "<i4"), ("pair", "<i4"),
                         ("val", "<f8", 3), ("mis_total", "<f8"), ("mis_tech", "<f8"),
                         ("p_gen", "<f8"), ("train", "<f8", 10), ("mis_by_tech", "<f8", 9)])

MLP_NPARAM = 11368


def mlp_init(seed=0):
    """He-uniform weights and zero biases (object-space input of 6, hidden 64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((6, 64), (64, 64), (64, 64), (64, 40)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, (fan_in, fan_out)).astype(np.float32).ravel())
        parts.append(np.zeros(fan_out, np.float32))
    p = np.concatenate(parts)
    assert p.size == MLP_NPARAM
    return p


def mlp_forward(params, x, bf16=True):
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    out = np.zeros((len(x), 40))
    pp = np.ascontiguousarray(params, np.float32)
    lib().orc_mlp_forward(_p(pp, C.c_float), _p(x, C.c_double), len(x), int(bf16), _p(out, C.c_double))
    return out


def mlp_loss_grad(params, records, bf16=True):
    rec = np.ascontiguousarray(records, np.float32).reshape(-1, 10)
    g = np.zeros(MLP_NPARAM)
    pp = np.ascontiguousarray(params, np.float32)
    loss = lib().orc_mlp_loss_grad(_p(pp, C.c_float), _p(rec, C.c_float), len(rec), int(bf16), _p(g, C.c_double))
    return loss, g


def vmf_pdf(raw, w):
    r = np.ascontiguousarray(raw, np.float64)
    ww = np.ascontiguousarray(w, np.float64)
    return lib().orc_vmf_pdf(_p(r, C.c_double), _p(ww, C.c_double))


def vmf_sample(raw, u0, u1, u2):
    r = np.ascontiguousarray(raw, np.float64)
    out = np.zeros(3, np.float32)
    lib().orc_vmf_sample(_p(r, C.c_double), u0, u1, u2, _p(out, C.c_float))
    return out


STAT_NAMES = ["samples", "paths", "accepted", "r1", "r2", "r3", "r4", "r5", "r6", "zero_mis",
              "t1", "t2", "t3", "t4", "t5", "t6", "t7", "t8", "unmapped",
              "rays"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
        i32p, i64p, u32p = C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_uint32)
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_scene_create.restype = C.c_void_p
        L.orc_scene_create.argtypes = [f32p, C.c_int, i32p, C.c_int, i32p, i32p, f32p, C.c_int, f32p,
                                       f32p, C.c_int]
        L.orc_scene_destroy.argtypes = [C.c_void_p]
        L.orc_scene_eps.restype = C.c_double
        L.orc_scene_eps.argtypes = [C.c_void_p]
        L.orc_object_area.restype = C.c_double
        L.orc_object_area.argtypes = [C.c_void_p]
        L.orc_trace.argtypes = [C.c_void_p, f32p, f32p, C.c_int, f32p, i32p]
        L.orc_bsdf_eval.restype = C.c_double
        L.orc_bsdf_eval.argtypes = [f32p, f64p, f64p, f64p, f64p]
        L.orc_bsdf_sample.argtypes = [f32p, f32p, f32p, C.c_float, C.c_float, f32p]
        L.orc_render_frame.argtypes = [C.c_void_p, f32p, f32p, f32p, C.c_int, C.POINTER(Params), f64p, i64p]
        L.orc_render_frame_dir.argtypes = [C.c_void_p, f32p, f32p, f32p, C.c_int, C.c_int, C.POINTER(Params), f64p,
                                           i64p]
        L.orc_render_residual.argtypes = [C.c_void_p, f32p, f32p, f32p, C.POINTER(Params), f64p, f64p, i64p,
                                          C.c_void_p, C.c_int64, i64p, f32p]
        L.orc_mlp_forward.argtypes = [f32p, f64p, C.c_int, C.c_int, f64p]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_mlp_loss_grad.argtypes = [f32p, f32p, C.c_int, C.c_int, f64p]
        L.orc_vmf_pdf.restype = C.c_double
        L.orc_vmf_pdf.argtypes = [f64p, f64p]
        L.orc_vmf_sample.argtypes = [f64p, C.c_float, C.c_float, C.c_float, f32p]
        L.orc_proposal_input.argtypes = [C.c_void_p, f32p, f32p, f64p]
        L.orc_map_check.argtypes = [C.c_void_p, f32p, f32p, C.POINTER(Params), i64p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


IDENTITY = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)


def scene_diag(scene) -> float:
    p = scene.positions.astype(np.float64)
    return float(np.sqrt(((p.max(0) - p.min(0)) ** 2).sum()))


class OracleScene:
    def __init__(self, scene, brute: bool | None = None):
        self.scene = scene
        self._arrs = [np.ascontiguousarray(scene.positions, np.float32),
                      np.ascontiguousarray(scene.indices, np.int32),
                      np.ascontiguousarray(scene.tri_material, np.int32),
                      np.ascontiguousarray(scene.tri_object, np.int32),
                      np.ascontiguousarray(scene.materials, np.float32),
                      np.ascontiguousarray(scene.env, np.float32),
                      np.ascontiguousarray(scene.camera, np.float32)]
        pos, idx, tm, to, mats, env, cam = self._arrs
        if brute is None:
            brute = len(idx) <= 2048
        self.h = lib().orc_scene_create(_p(pos, C.c_float), len(pos), _p(idx, C.c_int), len(idx),
                                        _p(tm, C.c_int), _p(to, C.c_int), _p(mats, C.c_float), len(mats),
                                        _p(env, C.c_float), _p(cam, C.c_float), int(brute))
        self.W, self.H = scene.width, scene.height

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_scene_destroy(self.h)
            self.h = None

    @property
    def eps(self):
        return lib().orc_scene_eps(self.h)

    @property
    def object_area(self):
        return lib().orc_object_area(self.h)

    def trace(self, rays: np.ndarray, pose=IDENTITY):
        rays = np.ascontiguousarray(rays, np.float32)
        n = len(rays)
        t = np.zeros(n, np.float32)
        ids = np.zeros(n, np.int32)
        pose = np.ascontiguousarray(pose, np.float32)
        lib().orc_trace(self.h, _p(pose, C.c_float), _p(rays, C.c_float), n, _p(t, C.c_float), _p(ids, C.c_int))
        return t, ids

    def _params(self, spp, depth, mask, two_way, seed, job, alpha_min, d_min, jac_max, c_weight, s0, s1,
                threads, material_mode, no_mapping=False, tech_spp=None, balance=False):
        if d_min is None:
            d_min = np.float32(0.01 * scene_diag(self.scene))
        ts = (C.c_int32 * 8)(*([int(x) for x in tech_spp] if tech_spp is not None else [0] * 8))
        return Params(spp, depth, mask, int(two_way), seed, job, alpha_min, float(d_min), jac_max, c_weight,
                      s0, s1, threads, int(material_mode), int(no_mapping), ts, int(balance))

    def render_frame(self, which, spp, depth, seed, pose_old=IDENTITY, pose_new=IDENTITY, new_mat=None,
                     s0=0, s1=-1, threads=1, job=0, stream_dir=None):
        """which: 1 old frame, 2 new frame.  stream_dir: the Philox direction
        word (default: the frame's own, 0 new / 1 old)."""
        pm = self._params(spp, depth, 0, 0, seed, job, 0.2, 1.0, 10.0, 0.5, s0, s1, threads, 0)
        img = np.zeros((self.H, self.W, 3), np.float64)
        st = np.zeros(4, np.int64)
        po = np.ascontiguousarray(pose_old, np.float32)
        pn = np.ascontiguousarray(pose_new, np.float32)
        nm = None if new_mat is None else np.ascontiguousarray(new_mat, np.float32)
        d = (0 if which == 2 else 1) if stream_dir is None else int(stream_dir)
        lib().orc_render_frame_dir(self.h, _p(po, C.c_float), _p(pn, C.c_float),
                                   None if nm is None else _p(nm, C.c_float), which, d, C.byref(pm),
                                   _p(img, C.c_double), _p(st, C.c_int64))
        return img, {"samples": int(st[0]), "paths": int(st[1])}

    def render_residual(self, spp, depth, seed, pose_old=IDENTITY, pose_new=IDENTITY, new_mat=None,
                        material_mode=False, mask=TECH_MASK_ALL, two_way=True, alpha_min=0.2, d_min=None,
                        jac_max=10.0, c_weight=0.5, s0=0, s1=-1, threads=1, job=0, per_tech=False,
                        records=False, rec_cap=4_000_000, mlp=None, no_mapping=False, tech_spp=None,
                        balance=False):
        """tech_spp: per-technique samples per pixel (8 values, 0 = spp; the
        full sample range only): unequal counts in the balance heuristic."""
        if tech_spp is not None and any(tech_spp) and (s0 != 0 or s1 != -1):
            raise ValueError("per-technique sample counts need the full sample range")
        pm = self._params(spp, depth, mask, two_way, seed, job, alpha_min, d_min, jac_max, c_weight, s0, s1,
                          threads, material_mode, no_mapping, tech_spp, balance)
        img = np.zeros((self.H, self.W, 3), np.float64)
        timg = np.zeros((8, self.H, self.W, 3), np.float64) if per_tech else None
        st = np.zeros(32, np.int64)
        po = np.ascontiguousarray(pose_old, np.float32)
        pn = np.ascontiguousarray(pose_new, np.float32)
        nm = None if new_mat is None else np.ascontiguousarray(new_mat, np.float32)
        recs = np.zeros(rec_cap if records else 0, RECORD_DTYPE)
        cnt = np.zeros(1, np.int64)
        mp = None if mlp is None else np.ascontiguousarray(mlp, np.float32)
        lib().orc_render_residual(self.h, _p(po, C.c_float), _p(pn, C.c_float),
                                  None if nm is None else _p(nm, C.c_float), C.byref(pm), _p(img, C.c_double),
                                  None if timg is None else _p(timg, C.c_double), _p(st, C.c_int64),
                                  recs.ctypes.data if records else None, rec_cap if records else 0,
                                  _p(cnt, C.c_int64), None if mp is None else _p(mp, C.c_float))
        stats = {n: int(st[i]) for i, n in enumerate(STAT_NAMES)}
        out = {"image": img, "stats": stats}
        if per_tech:
            out["per_tech"] = timg
        if records:
            out["records"] = recs[: min(int(cnt[0]), rec_cap)]
        return out


def map_check(osc: OracleScene, pose_new, spp, depth, seed, s0=0, s1=-1, alpha_min=0.2, d_min=None,
              jac_max=10.0):
    pm = osc._params(spp, depth, TECH_MASK_ALL, 1, seed, 0, alpha_min, d_min, jac_max, 0.5, s0, s1, 1, 0)
    out = np.zeros(4, np.int64)
    po = np.ascontiguousarray(IDENTITY)
    pn = np.ascontiguousarray(pose_new, np.float32)
    lib().orc_map_check(osc.h, _p(po, C.c_float), _p(pn, C.c_float), C.byref(pm), _p(out, C.c_int64))
    return {"checked": int(out[0]), "accept_mismatch": int(out[1]), "roundtrip_mismatch": int(out[2]),
            "accepted": int(out[3])}


def residual_for(ws, osc: OracleScene, **kw):
    """Run the oracle's residual estimator for a scenes.Workload."""
    e = ws.edit
    args = dict(spp=ws.spp, depth=ws.depth, seed=ws.seed, mask=ws.mask, two_way=ws.two_way)
    if e.kind == EDIT_MATERIAL:
        args.update(material_mode=True, new_mat=e.new_material, two_way=False)
    else:
        args.update(pose_old=IDENTITY, pose_new=e.old_to_new)
    args.update(kw)
    return osc.render_residual(**args)
