"""Seeded synthetic scenes and edits.

This module only builds input data (triangles, materials, camera, edit
transforms, render settings).  It holds none of the estimator's arithmetic:
both the HIP library and the CPU oracle consume the flat arrays it returns.

Array conventions (shared input format, documented in include/rpi.h):
  positions     float32 [V,3]   world space, object vertices at the OLD pose
  indices       int32   [F,3]   counter-clockwise seen from the normal side
  tri_material  int32   [F]
  tri_object    int32   [F]     0 = static, 1 = the dynamic / edited object
  materials     float32 [M,8]   type, albedo rgb, roughness, emission rgb
                                type 0 = Lambertian, 1 = GGX conductor,
                                type 2 = one-sided emitter (no reflection)
  env           float32 [3]     constant environment radiance
  camera        float32 [12]    eye xyz, target xyz, up xyz, vfov_deg, W, H

The paper's scenes are not available; these recipes stand in for them
(moving-object Cornell box, cluttered moving-object scene, material edit
on a large scene).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DIFFUSE, GGX, EMITTER = 0, 1, 2
EDIT_RIGID, EDIT_MATERIAL = 0, 1


@dataclass
class Scene:
    positions: np.ndarray
    indices: np.ndarray
    tri_material: np.ndarray
    tri_object: np.ndarray
    materials: np.ndarray
    env: np.ndarray
    camera: np.ndarray

    @property
    def width(self) -> int:
        return int(self.camera[10])

    @property
    def height(self) -> int:
        return int(self.camera[11])

    def with_resolution(self, w: int, h: int) -> "Scene":
        cam = self.camera.copy()
        cam[10], cam[11] = w, h
        return Scene(self.positions, self.indices, self.tri_material,
                     self.tri_object, self.materials, self.env, cam)


@dataclass
class Edit:
    kind: int = EDIT_RIGID
    old_to_new: np.ndarray = field(
        default_factory=lambda: np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32))
    new_material: np.ndarray | None = None  # float32 [8] for material edits


@dataclass
class Workload:
    name: str
    scene: Scene
    edit: Edit
    spp: int
    depth: int
    mask: int          # bit t-1 enables technique t (1..8)
    two_way: bool
    seed: int


class _Mesh:
    def __init__(self):
        self.p: list[np.ndarray] = []
        self.i: list[np.ndarray] = []
        self.m: list[np.ndarray] = []
        self.o: list[np.ndarray] = []
        self.nv = 0

    def add(self, pos, idx, mat, obj=0):
        pos = np.asarray(pos, np.float32).reshape(-1, 3)
        idx = np.asarray(idx, np.int64).reshape(-1, 3)
        self.p.append(pos)
        self.i.append(idx + self.nv)
        self.m.append(np.full(len(idx), mat, np.int32))
        self.o.append(np.full(len(idx), obj, np.int32))
        self.nv += len(pos)

    def add_quad(self, a, b, c, d, mat, obj=0):
        """Quad a,b,c,d counter-clockwise around its normal."""
        self.add([a, b, c, d], [[0, 1, 2], [0, 2, 3]], mat, obj)

    def build(self, materials, env, camera) -> Scene:
        return Scene(np.concatenate(self.p).astype(np.float32),
                     np.concatenate(self.i).astype(np.int32),
                     np.concatenate(self.m).astype(np.int32),
                     np.concatenate(self.o).astype(np.int32),
                     np.asarray(materials, np.float32).reshape(-1, 8),
                     np.asarray(env, np.float32).reshape(3),
                     np.asarray(camera, np.float32).reshape(12))


def mat(kind, albedo=(0, 0, 0), rough=1.0, emission=(0, 0, 0)):
    return [float(kind), *map(float, albedo), float(rough), *map(float, emission)]


def translation(t) -> np.ndarray:
    return np.array([1, 0, 0, t[0], 0, 1, 0, t[1], 0, 0, 1, t[2]], np.float32)


def rotation_y(deg, t=(0, 0, 0)) -> np.ndarray:
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    return np.array([c, 0, s, t[0], 0, 1, 0, t[1], -s, 0, c, t[2]], np.float32)


def rotation_y_about(deg, center, t=(0, 0, 0)) -> np.ndarray:
    """Rotation by deg about the vertical axis through center, then a
    translation t: x -> R (x - center) + center + t."""
    m = rotation_y(deg).reshape(3, 4).astype(np.float64)
    c = np.asarray(center, np.float64)
    m[:, 3] = c - m[:, :3] @ c + np.asarray(t, np.float64)
    return m.astype(np.float32).reshape(12)


# --- primitive meshes -------------------------------------------------------

def icosphere(level: int):
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
         (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
         (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, np.int64)


def cube_sphere(n: int):
    """Each cube face an n x n grid projected to the unit sphere: 12 n^2 tris."""
    verts, faces = [], []
    axes = [(0, 1, 2, 1.0), (0, 1, 2, -1.0), (1, 2, 0, 1.0), (1, 2, 0, -1.0),
            (2, 0, 1, 1.0), (2, 0, 1, -1.0)]
    g = np.linspace(-1.0, 1.0, n + 1)
    for ua, va, wa, sgn in axes:
        base = len(verts)
        for j in range(n + 1):
            for i in range(n + 1):
                p = np.zeros(3)
                p[ua], p[va], p[wa] = g[i], g[j], sgn
                verts.append(p / np.linalg.norm(p))
        for j in range(n):
            for i in range(n):
                a = base + j * (n + 1) + i
                b, c, d = a + 1, a + n + 2, a + n + 1
                faces += [(a, b, c), (a, c, d)]
    verts, faces = np.array(verts), np.array(faces, np.int64)
    # orient every triangle outward
    p0, p1, p2 = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, p0 + p1 + p2) < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    return verts, faces


def box_mesh(center, half):
    c, h = np.asarray(center, np.float64), np.asarray(half, np.float64)
    corners = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float64)
    v = c + corners * h
    # outward-facing quads (indices into corners ordered x,y,z bits)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    f = []
    for a, b, cc, d in quads:
        f += [(a, b, cc), (a, cc, d)]
    f = np.array(f, np.int64)
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, (p0 + p1 + p2) / 3 - c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


# --- workloads --------------------------------------------------------------

def cornell_motion(width=64, height=64, spp=16, depth=3, seed=1001,
                   offset=(0.1, 0.0, 0.05), two_cubes=False, lift=1e-3, rotate_deg=0.0) -> Workload:
    """Tiny Cornell box with a moving 12-triangle cube (24 triangles), or with
    a moving object made of two cubes with a gap between them (a non-convex
    object that shadows and reflects onto itself).  lift: height of the
    object above the floor (0: resting on it, its bottom face coplanar with
    the floor); rotate_deg: the edit also turns the cube about its vertical
    axis."""
    mats = [mat(DIFFUSE, (0.7, 0.7, 0.7)), mat(DIFFUSE, (0.7, 0.1, 0.1)),
            mat(DIFFUSE, (0.1, 0.7, 0.1)), mat(EMITTER, emission=(15, 15, 15)),
            mat(DIFFUSE, (0.7, 0.7, 0.7))]
    m = _Mesh()
    s = 0.5
    m.add_quad((-s, -s, s), (s, -s, s), (s, -s, -s), (-s, -s, -s), 0)   # floor, +y
    m.add_quad((-s, s, -s), (s, s, -s), (s, s, s), (-s, s, s), 0)       # ceiling, -y
    m.add_quad((-s, -s, -s), (s, -s, -s), (s, s, -s), (-s, s, -s), 0)   # back, +z
    m.add_quad((-s, -s, s), (-s, -s, -s), (-s, s, -s), (-s, s, s), 1)   # left, +x
    m.add_quad((s, -s, -s), (s, -s, s), (s, s, s), (s, s, -s), 2)       # right, -x
    ly, lh = 0.499, 0.1
    m.add_quad((-lh, ly, -lh), (lh, ly, -lh), (lh, ly, lh), (-lh, ly, lh), 3)  # light, -y
    if two_cubes:
        # two cubes of side 0.16, 0.06 apart
        for cx in (-0.16, 0.06):
            v, f = box_mesh((cx, -0.42 + lift, -0.05), (0.08, 0.08, 0.08))
            m.add(v, f, 4, obj=1)
        center = (-0.05, -0.42 + lift, -0.05)
    else:
        # cube of side 0.3
        center = (-0.05, -0.35 + lift, -0.05)
        v, f = box_mesh(center, (0.15, 0.15, 0.15))
        m.add(v, f, 4, obj=1)
    cam = [0, 0, 1.7, 0, 0, 0, 0, 1, 0, 40.0, width, height]
    scene = m.build(mats, (0, 0, 0), cam)
    xf = rotation_y_about(rotate_deg, center, offset) if rotate_deg else translation(offset)
    return Workload("cornell_motion", scene, Edit(EDIT_RIGID, xf), spp, depth, 0x7F, True, seed)


def cornell_material(width=64, height=64, spp=16, depth=3, seed=1011) -> Workload:
    """Cornell box with the cube's Lambertian albedo 0.7 turned into a GGX conductor."""
    w = cornell_motion(width, height, spp, depth, seed)
    edit = Edit(EDIT_MATERIAL, new_material=np.array(mat(GGX, (0.9, 0.6, 0.3), 0.35), np.float32))
    return Workload("cornell_material", w.scene, edit, spp, depth, 0x07, False, seed)


def clutter_motion(width=512, height=512, spp=64, depth=5, seed=1002,
                   n_spheres=400, env=(0.0, 0.0, 0.0)) -> Workload:
    """Ground plane, seeded icosphere clutter and a 20,480-triangle moving sphere."""
    rng = np.random.default_rng(seed)
    mats = [mat(DIFFUSE, (0.5, 0.5, 0.5)), mat(EMITTER, emission=(20, 20, 20)),
            mat(DIFFUSE, (0.6, 0.6, 0.6))]
    m = _Mesh()
    g = 6.0
    m.add_quad((-g, 0, g), (g, 0, g), (g, 0, -g), (-g, 0, -g), 0)
    lh = 0.75
    m.add_quad((-lh, 6, -lh), (lh, 6, -lh), (lh, 6, lh), (-lh, 6, lh), 1)
    v1, f1 = icosphere(1)
    v2, f2 = icosphere(2)
    placed = 0
    while placed < n_spheres:
        x, z = rng.uniform(-5, 5, 2)
        r = rng.uniform(0.05, 0.3)
        if math.hypot(x, z) < 1.3 + r:   # keep clear of the moving sphere's path
            continue
        if rng.uniform() < 0.5:
            mats.append(mat(DIFFUSE, rng.uniform(0.2, 0.8, 3)))
        else:
            f0 = rng.uniform(0.2, 0.9, 3)
            mats.append(mat(GGX, f0, rng.uniform(0.1, 0.8)))
        vv, ff = (v2, f2) if r >= 0.15 else (v1, f1)
        m.add(vv * r + np.array([x, r, z]), ff, len(mats) - 1)
        placed += 1
    vs, fs = icosphere(5)
    m.add(vs * 0.5 + np.array([0.0, 0.5, 0.0]), fs, 2, obj=1)
    t = rng.uniform(-0.5, 0.5, 2)
    cam = [0, 4, 9, 0, 0.5, 0, 0, 1, 0, 45.0, width, height]
    scene = m.build(mats, env, cam)
    return Workload("clutter_motion", scene,
                    Edit(EDIT_RIGID, translation((t[0], 0.0, t[1]))),
                    spp, depth, 0x7F, True, seed)


def material_edit(width=1024, height=1024, spp=32, depth=6, seed=1003,
                  n_meshes=20, grid=64) -> Workload:
    """Twenty seeded cube-spheres (~983k triangles); mesh 0 changes GGX material."""
    rng = np.random.default_rng(seed)
    mats = [mat(DIFFUSE, (0.5, 0.5, 0.5)), mat(EMITTER, emission=(15, 15, 15)),
            mat(EMITTER, emission=(10, 10, 10)), mat(GGX, (0.5, 0.5, 0.5), 0.3)]
    m = _Mesh()
    g = 10.0
    m.add_quad((-g, 0, g), (g, 0, g), (g, 0, -g), (-g, 0, -g), 0)
    m.add_quad((-3.5, 5, -0.5), (-2.5, 5, -0.5), (-2.5, 5, 0.5), (-3.5, 5, 0.5), 1)
    m.add_quad((2.5, 5, 1.5), (3.5, 5, 1.5), (3.5, 5, 2.5), (2.5, 5, 2.5), 2)
    vc, fc = cube_sphere(grid)
    centres = []
    while len(centres) < n_meshes:
        r = rng.uniform(0.3, 1.0)
        x, z = rng.uniform(-8, 8, 2)
        if len(centres) == 0:
            x, z = 0.0, 1.0
        if any(math.hypot(x - cx, z - cz) < r + cr + 0.05 for cx, cz, cr in centres):
            continue
        centres.append((x, z, r))
    for k, (x, z, r) in enumerate(centres):
        if k == 0:
            mid = 3
        elif rng.uniform() < 0.5:
            mats.append(mat(DIFFUSE, rng.uniform(0.2, 0.8, 3)))
            mid = len(mats) - 1
        else:
            mats.append(mat(GGX, rng.uniform(0.2, 0.9, 3), rng.uniform(0.1, 0.8)))
            mid = len(mats) - 1
        m.add(vc * r + np.array([x, r + 1e-3, z]), fc, mid, obj=1 if k == 0 else 0)
    cam = [0, 5, 14, 0, 0.5, 0, 0, 1, 0, 45.0, width, height]
    scene = m.build(mats, (0.2, 0.2, 0.2), cam)
    edit = Edit(EDIT_MATERIAL, new_material=np.array(mat(GGX, (0.8, 0.8, 0.8), 0.6), np.float32))
    return Workload("material_edit", scene, edit, spp, depth, 0x07, False, seed)


def bezier_jobs(seed=1004, n_jobs=32):
    """Per-frame rigid edits along a seeded cubic Bezier and per-job resolutions."""
    rng = np.random.default_rng(seed)
    p0 = np.array([0.0, 0.5, 0.0])
    ctrl = [p0] + [p0 + np.array([rng.uniform(-1.5, 1.5), 0.0, rng.uniform(-1.5, 1.5)])
                   for _ in range(3)]

    def bez(s):
        a = 1 - s
        return a ** 3 * ctrl[0] + 3 * a * a * s * ctrl[1] + 3 * a * s * s * ctrl[2] + s ** 3 * ctrl[3]

    jobs = []
    for i in range(n_jobs):
        c0, c1 = bez(i / n_jobs), bez((i + 1) / n_jobs)
        res = int(rng.choice([256, 512, 768, 1024]))
        jobs.append({"pose_old": translation(c0 - p0), "pose_new": translation(c1 - p0),
                     "width": res, "height": res})
    return jobs


def furnace(width=32, height=32, albedo_old=0.5, albedo_new=0.8, level=3, seed=7):
    """Convex Lambertian sphere in a closed, non-reflective emitting enclosure (L_e=1)."""
    mats = [mat(EMITTER, emission=(1, 1, 1)), mat(DIFFUSE, (albedo_old,) * 3)]
    m = _Mesh()
    v, f = box_mesh((0, 0, 0), (3, 3, 3))
    m.add(v, f[:, [0, 2, 1]], 0)   # inward-facing emitter walls
    vs, fs = icosphere(level)
    m.add(vs * 0.6, fs, 1, obj=1)
    cam = [0, 0, 2.5, 0, 0, 0, 0, 1, 0, 30.0, width, height]
    scene = m.build(mats, (0, 0, 0), cam)
    edit = Edit(EDIT_MATERIAL, new_material=np.array(mat(DIFFUSE, (albedo_new,) * 3), np.float32))
    return Workload("furnace", scene, edit, 4, 2, 0x07, False, seed)


def ghost_plane(width=16, height=16, seed=11, open_object=False):
    """A small moving box (or a single open quad) in front of a diffuse back
    plane under a quad light."""
    mats = [mat(DIFFUSE, (0.8, 0.8, 0.8)), mat(EMITTER, emission=(5, 5, 5)),
            mat(DIFFUSE, (0.6, 0.6, 0.6))]
    m = _Mesh()
    m.add_quad((-2, -2, -1), (2, -2, -1), (2, 2, -1), (-2, 2, -1), 0)
    m.add_quad((-0.5, 1.5, -0.5), (0.5, 1.5, -0.5), (0.5, 1.5, 0.5), (-0.5, 1.5, 0.5), 1)
    if open_object:
        m.add_quad((-0.3, 0.3, -0.4), (0.3, 0.3, -0.4), (0.3, 0.3, -0.6), (-0.3, 0.3, -0.6), 2, obj=1)
    else:
        v, f = box_mesh((0, 0, -0.5), (0.2, 0.2, 0.02))
        m.add(v, f, 2, obj=1)
    cam = [0, 0, 3, 0, 0, -1, 0, 1, 0, 50.0, width, height]
    scene = m.build(mats, (0, 0, 0), cam)
    return Workload("ghost_plane", scene, Edit(EDIT_RIGID, translation((0.25, 0.1, 0.0))),
                    4, 3, 0x7F, True, seed)


def config(n: int, **kw) -> Workload:
    return {1: cornell_motion, 2: clutter_motion, 3: material_edit}[n](**kw)
