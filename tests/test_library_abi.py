"""CPU checks of the C ABI: librpi.so loads and exports every function that
include/rpi.h declares, and host-side validation rejects malformed input
before any device work (no compute call is made without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2406_16302_amd import native, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INVALID, UNSUPPORTED = -1, -2


def test_header_functions_are_exported():
    lib = native.load_library()
    hdr = open(os.path.join(ROOT, "include", "rpi.h")).read()
    names = sorted(set(re.findall(r"^(?:rpi_status|const char\s*\*)\s*(rpi_\w+)\s*\(", hdr, re.M)))
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert lib.rpi_version().decode().startswith("rpi")


def test_header_flags_match_the_binding():
    hdr = open(os.path.join(ROOT, "include", "rpi.h")).read()
    flags = {m[0]: int(m[1]) for m in re.findall(r"#define RPI_FLAG_(\w+) (\d+)u", hdr)}
    assert flags == {"TWO_WAY": native.FLAG_TWO_WAY, "ACCUMULATE": native.FLAG_ACCUMULATE,
                     "COUNT_WORK": native.FLAG_COUNT_WORK, "RECORDS": native.FLAG_RECORDS,
                     "TIME_KERNELS": native.FLAG_TIME_KERNELS, "NO_MAPPING": native.FLAG_NO_MAPPING,
                     "PER_TECHNIQUE": native.FLAG_PER_TECHNIQUE, "BALANCE": native.FLAG_BALANCE}


def test_null_arguments_are_rejected_without_device_work():
    lib = native.load_library()
    assert lib.rpi_build_scene(None, None, None) == INVALID
    assert b"null" in lib.rpi_last_error()
    assert lib.rpi_render_residual(None, None, None, None, None, None) == INVALID
    assert lib.rpi_render_frame(None, None, 0, None, None, None) == INVALID
    assert lib.rpi_apply_edit(None, None, None) == INVALID


def _build(sc, allocator=None):
    """rpi_build_scene on a scenes.Scene; returns (status, message)."""
    lib = native.load_library()
    arrs = [np.ascontiguousarray(sc.positions, np.float32), np.ascontiguousarray(sc.indices, np.int32),
            np.ascontiguousarray(sc.tri_material, np.int32), np.ascontiguousarray(sc.tri_object, np.int32),
            np.ascontiguousarray(sc.materials, np.float32), np.ascontiguousarray(sc.env, np.float32),
            np.ascontiguousarray(sc.camera, np.float32)]
    pos, idx, tm, to, mats, env, cam = arrs
    f = lambda a, t=C.c_float: a.ctypes.data_as(C.POINTER(t))
    d = native.SceneDesc(f(pos), len(pos), f(idx, C.c_int32), len(idx), f(tm, C.c_int32), f(to, C.c_int32),
                         f(mats), len(mats), f(env), f(cam))
    h = C.c_void_p()
    rc = lib.rpi_build_scene(C.byref(d), C.byref(allocator) if allocator is not None else None, C.byref(h))
    return rc, lib.rpi_last_error().decode()


def _cornell():
    return scenes.cornell_motion(width=8, height=8).scene


def _copy(sc, **kw):
    d = dict(positions=sc.positions.copy(), indices=sc.indices.copy(), tri_material=sc.tri_material.copy(),
             tri_object=sc.tri_object.copy(), materials=sc.materials.copy(), env=sc.env.copy(),
             camera=sc.camera.copy())
    d.update(kw)
    return scenes.Scene(**d)


def _mutated(name):
    sc = _cornell()
    obj = np.nonzero(sc.tri_object == 1)[0]
    if name == "nan_vertex":
        p = sc.positions.copy()
        p[3, 1] = np.nan
        return _copy(sc, positions=p), INVALID, "non-finite vertex"
    if name == "inf_vertex":
        p = sc.positions.copy()
        p[0, 0] = np.inf
        return _copy(sc, positions=p), INVALID, "non-finite vertex"
    if name == "index_out_of_range":
        i = sc.indices.copy()
        i[5, 2] = len(sc.positions)
        return _copy(sc, indices=i), INVALID, "index out of range"
    if name == "negative_index":
        i = sc.indices.copy()
        i[2, 0] = -1
        return _copy(sc, indices=i), INVALID, "index out of range"
    if name == "material_id_out_of_range":
        m = sc.tri_material.copy()
        m[1] = len(sc.materials)
        return _copy(sc, tri_material=m), INVALID, "material id"
    if name == "bad_material_type":
        m = sc.materials.copy()
        m[0, 0] = 3.0
        return _copy(sc, materials=m), INVALID, "material type"
    if name == "ggx_zero_roughness":
        m = sc.materials.copy()
        m[0, 0], m[0, 4] = 1.0, 0.0
        return _copy(sc, materials=m), INVALID, "roughness"
    if name == "bad_fov":
        c = sc.camera.copy()
        c[9] = 0.0
        return _copy(sc, camera=c), INVALID, "camera"
    if name == "fractional_width":
        c = sc.camera.copy()
        c[10] = 8.5
        return _copy(sc, camera=c), INVALID, "camera"
    if name == "emissive_object":
        em = np.array([scenes.mat(scenes.EMITTER, (0, 0, 0), 1.0, (1, 1, 1))], np.float32)
        m = np.concatenate([sc.materials, em]).astype(np.float32)
        tm = sc.tri_material.copy()
        tm[obj] = len(m) - 1
        return _copy(sc, materials=m, tri_material=tm), UNSUPPORTED, "emissive dynamic object"
    if name == "zero_area_object":
        p = sc.positions.copy()
        for t in obj:  # collapse every object triangle onto its first vertex
            p[sc.indices[t, 1]] = p[sc.indices[t, 0]]
            p[sc.indices[t, 2]] = p[sc.indices[t, 0]]
        p[np.unique(sc.indices[obj])] = p[sc.indices[obj[0], 0]]
        return _copy(sc, positions=p), INVALID, "zero-area object"
    if name == "zero_area_emitter":
        em = np.nonzero(sc.materials[sc.tri_material, 0] == scenes.EMITTER)[0]
        i = sc.indices.copy()
        i[em[0], 2] = i[em[0], 1]
        return _copy(sc, indices=i), INVALID, "zero-area emitter"
    if name == "no_object":
        return _copy(sc, tri_object=np.zeros_like(sc.tri_object)), UNSUPPORTED, "no dynamic triangles"
    if name == "second_object":
        o = sc.tri_object.copy()
        o[obj[:2]] = 2
        return _copy(sc, tri_object=o), UNSUPPORTED, "several independently moving objects"
    if name == "negative_object":
        o = sc.tri_object.copy()
        o[0] = -1
        return _copy(sc, tri_object=o), INVALID, "negative tri_object"
    if name == "two_object_materials":
        tm = sc.tri_material.copy()
        tm[obj[0]] = 0 if tm[obj[1]] != 0 else 1
        return _copy(sc, tri_material=tm), UNSUPPORTED, "single material"
    raise KeyError(name)


@pytest.mark.parametrize("name", ["nan_vertex", "inf_vertex", "index_out_of_range", "negative_index",
                                  "material_id_out_of_range", "bad_material_type", "ggx_zero_roughness", "bad_fov",
                                  "fractional_width", "emissive_object", "zero_area_object", "zero_area_emitter",
                                  "no_object", "second_object", "negative_object", "two_object_materials"])
def test_build_scene_rejects_malformed_scenes(name):
    sc, code, msg = _mutated(name)
    rc, err = _build(sc)
    assert rc == code, (name, rc, err)
    assert msg in err, (name, err)


def test_allocator_hook_without_functions_is_rejected():
    rc, err = _build(_cornell(), native.Allocator())
    assert rc == INVALID and "allocator" in err


def _edit(kind, m=None, mat=None):
    d = native.EditDesc()
    d.kind = kind
    for i, x in enumerate(np.asarray(m if m is not None else np.eye(3, 4), np.float32).reshape(12)):
        d.old_to_new[i] = float(x)
    if mat is not None:
        for i, x in enumerate(np.asarray(mat, np.float32)):
            d.new_material[i] = float(x)
    lib = native.load_library()
    h = C.c_void_p()
    rc = lib.rpi_apply_edit(None, C.byref(d), C.byref(h))
    return rc, lib.rpi_last_error().decode()


def test_apply_edit_validates_the_description_first():
    rot = scenes.rotation_y(30.0, (0.1, 0.0, -0.2)).reshape(3, 4)
    # a valid rigid transform gets as far as the missing scene
    assert _edit(native.EDIT_RIGID, rot) == (INVALID, "null scene")
    skew = rot.copy()
    skew[0, 1] += 0.01
    assert _edit(native.EDIT_RIGID, skew) == (INVALID, "transform is not orthonormal")
    scaled = rot.copy()
    scaled[:, :3] *= 1.1
    assert _edit(native.EDIT_RIGID, scaled) == (INVALID, "transform is not orthonormal")
    mirror = np.eye(3, 4, dtype=np.float32)
    mirror[0, 0] = -1
    assert _edit(native.EDIT_RIGID, mirror) == (INVALID, "transform is mirrored (det <= 0)")
    nan = np.eye(3, 4, dtype=np.float32)
    nan[1, 3] = np.nan
    assert _edit(native.EDIT_RIGID, nan) == (INVALID, "non-finite transform")
    assert _edit(5)[0] == INVALID and "unknown edit kind" in _edit(5)[1]
    assert _edit(native.EDIT_MATERIAL, mat=scenes.mat(scenes.EMITTER, (0, 0, 0), 1.0, (1, 1, 1))) == \
        (UNSUPPORTED, "emissive new material")
    assert _edit(native.EDIT_MATERIAL, mat=scenes.mat(scenes.GGX, (0.5, 0.5, 0.5), 0.0))[0] == INVALID
    assert _edit(native.EDIT_MATERIAL, mat=scenes.mat(scenes.DIFFUSE, (0.5, np.nan, 0.5)))[0] == INVALID
    assert _edit(native.EDIT_MATERIAL, mat=scenes.mat(scenes.DIFFUSE, (0.5, 0.5, 0.5))) == (INVALID, "null scene")
