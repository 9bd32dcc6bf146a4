"""ctypes binding of librpi.so with the names of include/rpi.h.

Argument marshalling only: host arrays go to rpi_build_scene, device tensors
(torch, ROCm) and the current HIP stream go to the rendering calls.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpi.so")

RPI_OK = 0
EDIT_RIGID, EDIT_MATERIAL = 0, 1
FLAG_TWO_WAY, FLAG_ACCUMULATE, FLAG_COUNT_WORK, FLAG_RECORDS, FLAG_TIME_KERNELS = 1, 2, 4, 8, 16
FLAG_NO_MAPPING, FLAG_PER_TECHNIQUE, FLAG_BALANCE = 32, 64, 128
FRAME_OLD, FRAME_NEW = 0, 1
PROPOSAL_NPARAM, TRAIN_RECORD_FLOATS = 11368, 10


class RpiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rpi error %d: %s" % (code, msg))
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [("positions", C.POINTER(C.c_float)), ("num_vertices", C.c_int32),
                ("indices", C.POINTER(C.c_int32)), ("num_triangles", C.c_int32),
                ("tri_material", C.POINTER(C.c_int32)), ("tri_object", C.POINTER(C.c_int32)),
                ("materials", C.POINTER(C.c_float)), ("num_materials", C.c_int32),
                ("env", C.POINTER(C.c_float)), ("camera", C.POINTER(C.c_float))]


class EditDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("old_to_new", C.c_float * 12), ("new_material", C.c_float * 8)]


class Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64),
                ("strategy_mask", C.c_uint32), ("flags", C.c_uint32), ("alpha_min", C.c_float),
                ("d_min", C.c_float), ("jac_max", C.c_float), ("c_weight", C.c_float),
                ("sample_begin", C.c_int64), ("sample_end", C.c_int64), ("queue_cap", C.c_int32),
                ("job", C.c_uint32), ("proposal", C.c_void_p), ("d_train_records", C.c_void_p),
                ("train_capacity", C.c_int64), ("train_weighting", C.c_int32),
                ("d_technique_images", C.c_void_p), ("tile", C.c_int32), ("technique_spp", C.c_int32 * 8)]

    @staticmethod
    def make(spp, depth, seed, mask=0x7F, flags=FLAG_TWO_WAY, alpha_min=0.2, d_min=-1.0, jac_max=10.0,
             c_weight=0.5, sample_begin=0, sample_end=-1, queue_cap=0, job=0, proposal=None, train_records=None,
             train_weighting=0, technique_images=None, tile=0, technique_spp=None):
        """proposal: a Proposal (technique 8 with mask bit 7); train_records: a
        float32 device tensor [cap, 10] receiving technique-3 training records;
        technique_images: a float32 device tensor [8, H, W, 3] (sets
        FLAG_PER_TECHNIQUE); technique_spp: 8 per-technique samples per pixel
        (0 = spp)."""
        p = Params(spp, depth, seed, mask, flags, alpha_min, d_min, jac_max, c_weight, sample_begin,
                   sample_end, queue_cap, job)
        p.tile = int(tile)
        if technique_spp is not None:
            for i, v in enumerate(technique_spp):
                p.technique_spp[i] = int(v)
        if technique_images is not None:
            p.d_technique_images = _devptr(technique_images, technique_images.numel()).value
            p._technique_ref = technique_images
            p.flags |= FLAG_PER_TECHNIQUE
        if proposal is not None:
            p.proposal = proposal.h.value
            p._proposal_ref = proposal
        if train_records is not None:
            cap = train_records.shape[0]
            p.d_train_records = _devptr(train_records, cap * TRAIN_RECORD_FLOATS).value
            p.train_capacity = cap
        p.train_weighting = int(train_weighting)
        return p


class Stats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("paths", C.c_int64), ("accepted", C.c_int64),
                ("rejected", C.c_int64 * 7), ("by_tech", C.c_int64 * 9), ("rays", C.c_int64 * 6),
                ("nodes_visited", C.c_int64), ("tris_tested", C.c_int64), ("milliseconds", C.c_double),
                ("kernel_ms", C.c_double * 32), ("kernel_launches", C.c_int64 * 32),
                ("kernel_nodes", C.c_int64 * 32), ("kernel_tris", C.c_int64 * 32),
                ("kernel_bytes_written", C.c_int64 * 32), ("train_records", C.c_int64),
                ("technique_ms", C.c_double * 9)]

    def as_dict(self):
        return {"samples": self.samples, "paths": self.paths, "accepted": self.accepted,
                "rejected": list(self.rejected), "by_tech": list(self.by_tech), "rays": list(self.rays),
                "nodes_visited": self.nodes_visited, "tris_tested": self.tris_tested,
                "milliseconds": self.milliseconds, "kernel_ms": list(self.kernel_ms),
                "kernel_launches": list(self.kernel_launches), "kernel_nodes": list(self.kernel_nodes),
                "kernel_tris": list(self.kernel_tris), "kernel_bytes_written": list(self.kernel_bytes_written),
                "train_records": self.train_records, "technique_ms": list(self.technique_ms)}


class Tuning(C.Structure):
    _fields_ = [("queue_cap", C.c_int32), ("walk_blocks_per_cu", C.c_int32), ("connect_blocks_per_cu", C.c_int32),
                ("ms_per_msample", C.c_double)]


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("allocate", _ALLOC_FN), ("deallocate", _FREE_FN), ("ctx", C.c_void_p)]


def torch_allocator():
    """An rpi_allocator backed by PyTorch's caching allocator (memory
    handed back is reused in stream order, as the library requires)."""
    import torch

    def alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # out of memory: the library reports OUT_OF_MEMORY
            return None

    def free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = Allocator(_ALLOC_FN(alloc), _FREE_FN(free), None)
    a._keep = (alloc, free)
    return a


class DenoiseParams(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("sigma_normal", C.c_float), ("sigma_depth", C.c_float),
                ("sigma_value", C.c_float)]


class Job(C.Structure):
    _fields_ = [("pose_old", C.c_float * 12), ("pose_new", C.c_float * 12), ("width", C.c_int32),
                ("height", C.c_int32), ("d_out", C.c_void_p)]


_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RpiError(-4, "librpi.so is not built (run __graft_entry__.build() or "
                               "python paper_2406_16302_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.rpi_build_scene.argtypes = [C.POINTER(SceneDesc), C.POINTER(Allocator), C.POINTER(vp)]
        L.rpi_sync_status.argtypes = [vp]
        L.rpi_destroy_scene.argtypes = [vp]
        L.rpi_apply_edit.argtypes = [vp, C.POINTER(EditDesc), C.POINTER(vp)]
        L.rpi_destroy_edit.argtypes = [vp]
        L.rpi_render_residual.argtypes = [vp, vp, C.POINTER(Params), vp, C.POINTER(Stats), vp]
        L.rpi_render_frame.argtypes = [vp, vp, C.c_int32, C.POINTER(Params), vp, vp]
        L.rpi_render_residual_noalloc.argtypes = [vp, vp, C.POINTER(Params), vp, vp]
        L.rpi_render_frame_difference.argtypes = [vp, vp, C.c_int32, C.POINTER(Params), vp, vp]
        L.rpi_render_residual_batch.argtypes = [vp, C.POINTER(Job), C.c_int32, C.POINTER(Params),
                                                C.POINTER(Stats), vp]
        L.rpi_get_records.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.rpi_autotune.argtypes = [vp, vp, C.POINTER(Params), C.POINTER(Tuning), vp]
        L.rpi_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.rpi_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.rpi_allocate_samples.argtypes = [vp, vp, C.POINTER(Params), C.c_int32, C.POINTER(C.c_int32), vp]
        L.rpi_denoise_residual.argtypes = [vp, vp, vp, vp, C.POINTER(DenoiseParams), vp, vp]
        L.rpi_render_gbuffer.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.rpi_proposal_create.argtypes = [vp, vp, C.c_uint64, C.POINTER(vp)]
        L.rpi_proposal_destroy.argtypes = [vp]
        L.rpi_proposal_set_weights.argtypes = [vp, vp]
        L.rpi_proposal_get_weights.argtypes = [vp, vp]
        L.rpi_proposal_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.rpi_proposal_loss_grad.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.rpi_proposal_train.argtypes = [vp, vp, C.c_int64, C.POINTER(TrainParams), vp, vp]
        L.rpi_last_error.restype = C.c_char_p
        L.rpi_version.restype = C.c_char_p
        for f in ("rpi_allocate_samples", "rpi_denoise_residual", "rpi_render_gbuffer", "rpi_get_tuning", "rpi_render_residual_noalloc", "rpi_render_frame_difference", "rpi_sync_status", "rpi_build_scene", "rpi_destroy_scene", "rpi_apply_edit", "rpi_destroy_edit",
                  "rpi_render_residual", "rpi_render_frame", "rpi_render_residual_batch", "rpi_get_records",
                  "rpi_autotune", "rpi_set_tuning", "rpi_proposal_create", "rpi_proposal_destroy", "rpi_proposal_set_weights",
                  "rpi_proposal_get_weights", "rpi_proposal_forward", "rpi_proposal_loss_grad",
                  "rpi_proposal_train"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(rc):
    if rc != RPI_OK:
        raise RpiError(rc, load_library().rpi_last_error().decode())


def _fp(a, t=C.c_float):
    return a.ctypes.data_as(C.POINTER(t))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _devptr(t, n):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise RpiError(-1, "output must be a contiguous float32 device tensor")
    if t.numel() != n:
        raise RpiError(-1, "output has %d elements, expected %d" % (t.numel(), n))
    return C.c_void_p(t.data_ptr())


class Scene:
    """rpi_build_scene over a scenes.Scene (host arrays copied by the library).
    allocator: None (hipMalloc / hipMallocAsync), "torch" (PyTorch's caching
    allocator) or an Allocator."""

    def __init__(self, sc, allocator=None):
        L = load_library()
        self.src = sc
        arrs = [np.ascontiguousarray(sc.positions, np.float32), np.ascontiguousarray(sc.indices, np.int32),
                np.ascontiguousarray(sc.tri_material, np.int32), np.ascontiguousarray(sc.tri_object, np.int32),
                np.ascontiguousarray(sc.materials, np.float32), np.ascontiguousarray(sc.env, np.float32),
                np.ascontiguousarray(sc.camera, np.float32)]
        pos, idx, tm, to, mats, env, cam = arrs
        d = SceneDesc(_fp(pos), len(pos), _fp(idx, C.c_int32), len(idx), _fp(tm, C.c_int32), _fp(to, C.c_int32),
                      _fp(mats), len(mats), _fp(env), _fp(cam))
        if allocator == "torch":
            allocator = torch_allocator()
        self.allocator = allocator  # kept alive as long as the scene
        h = C.c_void_p()
        _check(L.rpi_build_scene(C.byref(d), C.byref(allocator) if allocator is not None else None, C.byref(h)))
        self.h = h
        self.width, self.height = sc.width, sc.height

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.rpi_destroy_scene(self.h)
            self.h = None

    def records(self):
        L = load_library()
        n = C.c_int64()
        _check(L.rpi_get_records(self.h, None, 0, C.byref(n)))
        out = np.zeros((n.value, 8), np.uint32)
        _check(L.rpi_get_records(self.h, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        return out


class Edit:
    """rpi_apply_edit: rigid motion (old_to_new 3x4) or a material edit."""

    def __init__(self, scene: Scene, edit):
        L = load_library()
        d = EditDesc()
        d.kind = int(edit.kind)
        m = np.asarray(edit.old_to_new, np.float32).reshape(12)
        for i in range(12):
            d.old_to_new[i] = float(m[i])
        if edit.new_material is not None:
            nm = np.asarray(edit.new_material, np.float32).reshape(8)
            for i in range(8):
                d.new_material[i] = float(nm[i])
        h = C.c_void_p()
        _check(L.rpi_apply_edit(scene.h, C.byref(d), C.byref(h)))
        self.h = h
        self.scene = scene
        self.kind = int(edit.kind)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.rpi_destroy_edit(self.h)
            self.h = None


def render_residual(scene: Scene, edit: Edit, params: Params, out, stats=False, stream=None):
    L = load_library()
    st = Stats() if stats else None
    _check(L.rpi_render_residual(scene.h, edit.h, C.byref(params), _devptr(out, scene.width * scene.height * 3),
                                 C.byref(st) if st is not None else None, _stream(stream)))
    return st.as_dict() if st is not None else None


def render_residual_noalloc(scene: Scene, edit: Edit, params: Params, out, stream=None):
    """rpi_render_residual_noalloc: the residual with the library's static
    workspace (no device allocation in the call)."""
    _check(load_library().rpi_render_residual_noalloc(scene.h, edit.h, C.byref(params),
                                                      _devptr(out, scene.width * scene.height * 3), _stream(stream)))


def render_frame(scene: Scene, edit: Edit | None, which: int, params: Params, out, stream=None):
    """Plain path tracing of one frame: which = FRAME_OLD (0) or FRAME_NEW (1)."""
    L = load_library()
    _check(L.rpi_render_frame(scene.h, edit.h if edit is not None else None, int(which), C.byref(params),
                              _devptr(out, scene.width * scene.height * 3), _stream(stream)))


def render_frame_difference(scene: Scene, edit: Edit, correlated: bool, params: Params, out, stream=None):
    """I_new - I_old by path tracing: correlated (the same random numbers in
    both frames) or from scratch (independent streams)."""
    L = load_library()
    _check(L.rpi_render_frame_difference(scene.h, edit.h, 1 if correlated else 0, C.byref(params),
                                         _devptr(out, scene.width * scene.height * 3), _stream(stream)))


def allocate_samples(scene: Scene, edit: Edit, params: Params, pilot_spp=4, stream=None):
    """rpi_allocate_samples: per-technique samples per pixel from a pilot."""
    out = (C.c_int32 * 8)()
    _check(load_library().rpi_allocate_samples(scene.h, edit.h, C.byref(params), int(pilot_spp), out,
                                               _stream(stream)))
    return [int(x) for x in out]


def denoise_residual(scene: Scene, edit: Edit, a, b, out, iterations=0, sigma_normal=0.0, sigma_depth=0.0,
                     sigma_value=0.0, stream=None):
    """rpi_denoise_residual: R = a + b (two independent half estimates)
    filtered with the residual-aware a-trous filter into out."""
    n = scene.width * scene.height * 3
    dp = DenoiseParams(int(iterations), float(sigma_normal), float(sigma_depth), float(sigma_value))
    _check(load_library().rpi_denoise_residual(scene.h, edit.h, _devptr(a, n), _devptr(b, n), C.byref(dp),
                                               _devptr(out, n), _stream(stream)))


def render_gbuffer(scene: Scene, edit: Edit | None, which: int, out, stream=None):
    """rpi_render_gbuffer: normal (facing the camera) and hit distance per pixel centre."""
    _check(load_library().rpi_render_gbuffer(scene.h, edit.h if edit is not None else None, int(which),
                                             _devptr(out, scene.width * scene.height * 4), _stream(stream)))


def sync_status(stream=None):
    """rpi_sync_status: wait for the stream, raise on a device error."""
    _check(load_library().rpi_sync_status(_stream(stream)))


def autotune(scene: Scene, edit: Edit, params: Params, stream=None):
    L = load_library()
    t = Tuning()
    _check(L.rpi_autotune(scene.h, edit.h, C.byref(params), C.byref(t), _stream(stream)))
    return {"queue_cap": t.queue_cap, "walk_blocks_per_cu": t.walk_blocks_per_cu,
            "connect_blocks_per_cu": t.connect_blocks_per_cu, "ms_per_msample": t.ms_per_msample}


def set_tuning(scene: Scene, queue_cap, walk_blocks_per_cu, connect_blocks_per_cu):
    t = Tuning(int(queue_cap), int(walk_blocks_per_cu), int(connect_blocks_per_cu), 0.0)
    _check(load_library().rpi_set_tuning(scene.h, C.byref(t)))


def get_tuning(scene: Scene):
    """rpi_get_tuning: the launch configuration of later calls with queue_cap 0."""
    t = Tuning()
    _check(load_library().rpi_get_tuning(scene.h, C.byref(t)))
    return {"queue_cap": t.queue_cap, "walk_blocks_per_cu": t.walk_blocks_per_cu,
            "connect_blocks_per_cu": t.connect_blocks_per_cu}


def render_residual_batch(scene: Scene, jobs, params: Params, stats=False, stream=None):
    """jobs: list of dicts with pose_old, pose_new (3x4), out (float32 device tensor [H, W, 3])."""
    L = load_library()
    arr = (Job * len(jobs))()
    for i, j in enumerate(jobs):
        po = np.asarray(j["pose_old"], np.float32).reshape(12)
        pn = np.asarray(j["pose_new"], np.float32).reshape(12)
        for q in range(12):
            arr[i].pose_old[q] = float(po[q])
            arr[i].pose_new[q] = float(pn[q])
        h, w = j["out"].shape[0], j["out"].shape[1]
        arr[i].width, arr[i].height = w, h
        arr[i].d_out = _devptr(j["out"], w * h * 3).value
    st = Stats() if stats else None
    _check(L.rpi_render_residual_batch(scene.h, arr, len(jobs), C.byref(params),
                                       C.byref(st) if st is not None else None, _stream(stream)))
    return st.as_dict() if st is not None else None


def _devptr_any(t, n):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise RpiError(-1, "expected a contiguous float32 device tensor")
    if t.numel() < n:
        raise RpiError(-1, "tensor has %d elements, need %d" % (t.numel(), n))
    return C.c_void_p(t.data_ptr())


class Proposal:
    """rpi_proposal_*: the learned proposal of technique 8 (MLP weights on the device)."""

    def __init__(self, scene: Scene, params=None, seed=0):
        L = load_library()
        h = C.c_void_p()
        if params is not None:
            params = np.ascontiguousarray(params, np.float32).reshape(PROPOSAL_NPARAM)
        _check(L.rpi_proposal_create(scene.h, params.ctypes.data_as(C.c_void_p) if params is not None else None,
                                     int(seed), C.byref(h)))
        self.h = h
        self.scene = scene

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.rpi_proposal_destroy(self.h)
            self.h = None

    def set_weights(self, params):
        params = np.ascontiguousarray(params, np.float32).reshape(PROPOSAL_NPARAM)
        _check(load_library().rpi_proposal_set_weights(self.h, params.ctypes.data_as(C.c_void_p)))

    def get_weights(self):
        out = np.zeros(PROPOSAL_NPARAM, np.float32)
        _check(load_library().rpi_proposal_get_weights(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def forward(self, x, out, stream=None):
        n = x.shape[0]
        _check(load_library().rpi_proposal_forward(self.h, _devptr_any(x, 6 * n), n, _devptr_any(out, 40 * n),
                                                   _stream(stream)))

    def loss_grad(self, records, grad, loss=None, stream=None):
        n = records.shape[0]
        _check(load_library().rpi_proposal_loss_grad(
            self.h, _devptr_any(records, TRAIN_RECORD_FLOATS * n), n, _devptr_any(grad, PROPOSAL_NPARAM),
            _devptr_any(loss, 1) if loss is not None else None, _stream(stream)))

    def train(self, records, n, steps, batch=16384, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
              losses=None, stream=None):
        tp = TrainParams(int(steps), int(batch), lr, beta1, beta2, eps, int(seed))
        _check(load_library().rpi_proposal_train(
            self.h, _devptr_any(records, TRAIN_RECORD_FLOATS * n), int(n), C.byref(tp),
            _devptr_any(losses, steps) if losses is not None else None, _stream(stream)))
