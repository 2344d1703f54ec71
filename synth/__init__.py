"""Seeded synthetic inputs for batched LiDAR ray casting.

This module only *produces inputs*: triangle meshes, sensor poses and beam
patterns.  It holds none of the ray-casting arithmetic, and both the GPU
path's tests and the FP64 oracle's tests draw their inputs from it.

The paper's scenes (3DGS assets, real LiDAR captures; FGGS-LiDAR Sec. V) are
not available, so seeded synthetic scenes with the same structure stand in:

* ``room_sphere_scene`` -- closed 10 x 8 x 3 m box room (12 triangles) with a
  UV sphere (r = 1 m, 64 x 32 segments, 3,968 triangles) at a seeded spot;
  one seeded interior pose, 16 x 360 beam pattern over -15..+15 deg.
* ``indoor_scene`` -- closed indoor mesh: marching cubes (spacing ``h``) of a
  seeded signed-distance union of the room shell and 200 boxes / spheres /
  vertical cylinders with sizes uniform in 0.1..2 m.  At h = 3.5 cm this is
  about one million triangles; at h = 2 cm about three million.
* ``terrain_scene`` -- open outdoor heightfield (fractal value noise, 200 x
  200 m) plus randomly placed, partly sunk boxes.

Mesh layout everywhere: ``verts`` float32 [nv, 3], ``tris`` int32 [nt, 3].
Pose layout: float32 [12] row-major ``[R | t]``.  Beam directions: float32
[n_beams, 3], unit length (computed in FP64, then rounded), index
``j = elevation_index * n_az + azimuth_index``; sensor frame x forward,
y left, z up.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdfmesh.c")
_LIB = os.path.join(_HERE, "_sdfmesh.so")

ROOM_LO = (0.0, 0.0, 0.0)
ROOM_HI = (10.0, 8.0, 3.0)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.sdf_eval.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int64, P]
        lib.sdf_eval.restype = None
        lib.sdfmesh_build.argtypes = [P, ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_int64)]
        lib.sdfmesh_build.restype = ctypes.c_int
        lib.sdfmesh_free.argtypes = [P]
        lib.sdfmesh_free.restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Beam patterns and poses

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def workload_config(name: str) -> dict:
    """The stored definition of a benchmark workload -- its seeds, sizes,
    beam pattern and range -- from synth/configs/<name>.json, so every run of
    a workload draws the same inputs."""
    with open(os.path.join(CONFIG_DIR, name + ".json")) as fh:
        return json.load(fh)


def lidar_pattern(n_el: int, el_lo_deg: float, el_hi_deg: float, n_az: int) -> np.ndarray:
    """Spinning-LiDAR directions: elevations linspace(lo, hi, n_el) inclusive,
    azimuths a * 2pi / n_az.  FP64, rounded to float32; [n_el * n_az, 3]."""
    el = np.radians(np.linspace(el_lo_deg, el_hi_deg, n_el, dtype=np.float64))
    az = np.arange(n_az, dtype=np.float64) * (2.0 * math.pi / n_az)
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1)
    return np.ascontiguousarray(d.reshape(-1, 3).astype(np.float32))


def yaw_pose(position, yaw: float) -> np.ndarray:
    """Row-major [R | t] for a rotation about +z by ``yaw`` (float32 [12])."""
    c, s = math.cos(yaw), math.sin(yaw)
    x, y, z = (float(v) for v in position)
    return np.array([c, -s, 0.0, x, s, c, 0.0, y, 0.0, 0.0, 1.0, z], dtype=np.float32)


def rpy_pose(position, roll: float, pitch: float, yaw: float) -> np.ndarray:
    """Row-major [R | t] with R = Rz(yaw) Ry(pitch) Rx(roll) (float32 [12])."""
    cr, sr = math.cos(roll), math.sin(roll)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cy, sy = math.cos(yaw), math.sin(yaw)
    R = np.array([[cy * cp, cy * sp * sr - sy * cr, cy * sp * cr + sy * sr],
                  [sy * cp, sy * sp * sr + cy * cr, sy * sp * cr - cy * sr],
                  [-sp, cp * sr, cp * cr]], dtype=np.float64)
    P = np.zeros((3, 4), np.float64)
    P[:, :3] = R
    P[:, 3] = position
    return P.reshape(12).astype(np.float32)


# --------------------------------------------------------------------------
# Simple meshes

def box_room(lo=ROOM_LO, hi=ROOM_HI):
    """Closed axis-aligned box, 8 vertices, 12 triangles.

    Faces in order -x, +x, -y, +y, -z, +z; face f owns triangles 2f, 2f+1.
    Each face is the quad (p00, p10, p11, p01) over its two free axes
    (a, b) = ((f//2 + 1) % 3, (f//2 + 2) % 3), split along p00-p11:
    triangle 2f = (p00, p10, p11), triangle 2f+1 = (p00, p11, p01)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    verts = np.array([[(hi if (c >> k) & 1 else lo)[k] for k in range(3)] for c in range(8)],
                     dtype=np.float32)
    tris = []
    for f in range(6):
        ax, side = f // 2, f % 2
        a, b = (ax + 1) % 3, (ax + 2) % 3

        def corner(ua, ub):
            c = (side << ax) | (ua << a) | (ub << b)
            return c
        p00, p10, p11, p01 = corner(0, 0), corner(1, 0), corner(1, 1), corner(0, 1)
        tris.append((p00, p10, p11))
        tris.append((p00, p11, p01))
    return verts, np.array(tris, dtype=np.int32)


def grid_patch(n: int, size: float = 1.0, z: float = 0.0):
    """Open flat square [0, size]^2 at height z: an n x n grid of quads, each
    split along its diagonal; (n + 1)^2 vertices, 2 n^2 triangles."""
    g = np.linspace(0.0, size, n + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1).astype(np.float32)
    tris = []
    for j in range(n):
        for i in range(n):
            a = j * (n + 1) + i
            b, c, d = a + 1, a + n + 2, a + n + 1
            tris.append((a, b, c))
            tris.append((a, c, d))
    return verts, np.array(tris, dtype=np.int32)


def grid_box(lo, hi, n: int):
    """Closed axis-aligned box whose six faces are n x n grids of quads split
    along a diagonal, vertices shared along the box edges (watertight),
    outward-facing; 12 n^2 triangles."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    index = {}
    verts = []

    def vid(p):
        key = tuple(int(round(c)) for c in p)
        if key not in index:
            index[key] = len(verts)
            verts.append([lo[k] + (hi[k] - lo[k]) * key[k] / n for k in range(3)])
        return index[key]
    tris = []
    for ax in range(3):
        a, b = (ax + 1) % 3, (ax + 2) % 3
        for side in (0, n):
            for i in range(n):
                for j in range(n):
                    def pt(ui, uj):
                        p = [0, 0, 0]
                        p[ax], p[a], p[b] = side, ui, uj
                        return vid(p)
                    p00, p10, p11, p01 = pt(i, j), pt(i + 1, j), pt(i + 1, j + 1), pt(i, j + 1)
                    if side == n:
                        tris.append((p00, p10, p11))
                        tris.append((p00, p11, p01))
                    else:
                        tris.append((p00, p11, p10))
                        tris.append((p00, p01, p11))
    return np.array(verts, dtype=np.float32), np.array(tris, dtype=np.int32)


def uv_sphere(center, r: float, n_seg: int = 64, n_ring: int = 32):
    """UV sphere with vertices on the sphere (FP64, rounded to float32).
    2 * n_seg * (n_ring - 1) triangles (64 x 32 -> 3,968)."""
    c = np.asarray(center, np.float64)
    verts = [c + [0.0, 0.0, r]]
    for i in range(1, n_ring):
        th = math.pi * i / n_ring
        for j in range(n_seg):
            ph = 2.0 * math.pi * j / n_seg
            verts.append(c + r * np.array([math.sin(th) * math.cos(ph),
                                           math.sin(th) * math.sin(ph), math.cos(th)]))
    verts.append(c + [0.0, 0.0, -r])
    top, bot = 0, 1 + (n_ring - 1) * n_seg

    def ring(i, j):
        return 1 + i * n_seg + (j % n_seg)
    tris = []
    for j in range(n_seg):
        tris.append((top, ring(0, j), ring(0, j + 1)))
    for i in range(n_ring - 2):
        for j in range(n_seg):
            a, b = ring(i, j), ring(i, j + 1)
            c2, d = ring(i + 1, j), ring(i + 1, j + 1)
            tris.append((a, c2, d))
            tris.append((a, d, b))
    for j in range(n_seg):
        tris.append((bot, ring(n_ring - 2, j + 1), ring(n_ring - 2, j)))
    return np.array(verts, dtype=np.float32), np.array(tris, dtype=np.int32)


def plane_quad(half: float = 1000.0, z: float = 0.0):
    """Square at height z, [-half, half]^2, two triangles split along (-,-)-(+,+)."""
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]],
                 dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return v, t


def concat_meshes(*meshes):
    vs, ts, off = [], [], 0
    for v, t in meshes:
        vs.append(np.asarray(v, np.float32))
        ts.append(np.asarray(t, np.int32) + off)
        off += len(v)
    return np.ascontiguousarray(np.concatenate(vs)), np.ascontiguousarray(np.concatenate(ts))


def random_soup(rng: np.random.Generator, n: int, extent: float = 1.0):
    """n independent random triangles in [-extent, extent]^3 (not closed)."""
    v = rng.uniform(-extent, extent, size=(n * 3, 3)).astype(np.float32)
    t = np.arange(n * 3, dtype=np.int32).reshape(n, 3)
    return v, t


# --------------------------------------------------------------------------
# Scene descriptions

@dataclasses.dataclass
class Scene:
    name: str
    verts: np.ndarray
    tris: np.ndarray
    poses: np.ndarray          # float32 [E, 12]
    dirs: np.ndarray           # float32 [B, 3]
    t_min: float
    t_max: float
    n_az: int
    meta: dict

    @property
    def n_rays(self) -> int:
        return self.poses.shape[0] * self.dirs.shape[0]


def room_sphere_scene(seed: int = 0) -> Scene:
    """Closed 10 x 8 x 3 m box room (12 tris) + UV sphere r = 1 m (64 x 32,
    3,968 tris) whose centre keeps >= 1.1 m from every wall; one sensor at a
    seeded interior pose (>= 0.3 m from every surface, yaw uniform); 16 beams
    over -15..+15 deg x 360 azimuth steps; range [0, 100] m."""
    rng = np.random.default_rng(seed)
    lo, hi = np.array(ROOM_LO), np.array(ROOM_HI)
    c = rng.uniform(lo + 1.1, hi - 1.1)
    room = box_room()
    sph = uv_sphere(c, 1.0, 64, 32)
    verts, tris = concat_meshes(room, sph)
    while True:
        p = rng.uniform(lo + 0.3, hi - 0.3)
        if np.linalg.norm(p - c) >= 1.3:
            break
    pose = yaw_pose(p, rng.uniform(0.0, 2.0 * math.pi))[None]
    dirs = lidar_pattern(16, -15.0, 15.0, 360)
    return Scene("room_sphere", verts, tris, pose, dirs, 0.0, 100.0, 360,
                 {"sphere_center": c, "sphere_r": 1.0, "room_lo": lo, "room_hi": hi})


@dataclasses.dataclass
class SdfScene:
    room: np.ndarray        # [6] lo, hi
    types: np.ndarray       # int32 [n]
    params: np.ndarray      # float64 [n, 8]

    def sdf(self, pts) -> np.ndarray:
        pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
        out = np.empty(pts.shape[0], np.float64)
        _load().sdf_eval(_p(self.room), len(self.types), _p(self.types), _p(self.params),
                         _p(pts), pts.shape[0], _p(out))
        return out


def indoor_sdf(seed: int, n_prims: int = 200, size_lo: float = 0.1,
               size_hi: float = 2.0) -> SdfScene:
    """Seeded room shell + union of boxes (yaw-random), spheres and vertical
    cylinders; full sizes uniform in [size_lo, size_hi] m, centres uniform in
    the room, primitive type uniform."""
    rng = np.random.default_rng(seed)
    room = np.array(ROOM_LO + ROOM_HI, np.float64)
    types = rng.integers(0, 3, size=n_prims).astype(np.int32)
    params = np.zeros((n_prims, 8), np.float64)
    for i in range(n_prims):
        params[i, :3] = rng.uniform(room[:3], room[3:])
        s = rng.uniform(size_lo, size_hi, size=3)
        if types[i] == 0:
            params[i, 3:6] = 0.5 * s
            params[i, 6] = rng.uniform(0.0, 2.0 * math.pi)
        elif types[i] == 1:
            params[i, 3] = 0.5 * s[0]
        else:
            params[i, 3] = 0.5 * s[0]
            params[i, 4] = 0.5 * s[1]
    return SdfScene(room, types, np.ascontiguousarray(params))


def polygonise(sdf: SdfScene, h: float, pad: int = 3):
    """Closed mesh of the zero set of ``sdf`` with grid spacing h."""
    lib = _load()
    vp, tp = ctypes.c_void_p(), ctypes.c_void_p()
    nv, nt = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.sdfmesh_build(_p(sdf.room), len(sdf.types), _p(sdf.types), _p(sdf.params),
                           float(h), int(pad), ctypes.byref(vp), ctypes.byref(nv),
                           ctypes.byref(tp), ctypes.byref(nt))
    if rc != 0:
        raise MemoryError("sdfmesh_build failed")
    try:
        v = np.ctypeslib.as_array(ctypes.cast(vp, ctypes.POINTER(ctypes.c_float)),
                                  shape=(nv.value, 3)).copy()
        t = np.ctypeslib.as_array(ctypes.cast(tp, ctypes.POINTER(ctypes.c_int32)),
                                  shape=(nt.value, 3)).copy()
    finally:
        lib.sdfmesh_free(vp)
        lib.sdfmesh_free(tp)
    return v, t


def free_space_poses(sdf: SdfScene, n: int, seed: int, clearance: float = 0.3) -> np.ndarray:
    """n poses uniform in free space (field >= clearance), yaw uniform."""
    rng = np.random.default_rng(seed)
    lo, hi = sdf.room[:3], sdf.room[3:]
    out = []
    while len(out) < n:
        cand = rng.uniform(lo, hi, size=(max(64, 2 * (n - len(out))), 3))
        ok = sdf.sdf(cand) >= clearance
        for p in cand[ok]:
            if len(out) < n:
                out.append(yaw_pose(p, rng.uniform(0.0, 2.0 * math.pi)))
    return np.ascontiguousarray(np.stack(out))


_MESH_CACHE: dict = {}


def indoor_mesh(seed: int = 1, h: float = 0.035):
    key = (seed, h)
    if key not in _MESH_CACHE:
        sdf = indoor_sdf(seed)
        _MESH_CACHE[key] = (sdf,) + polygonise(sdf, h)
    return _MESH_CACHE[key]


def indoor_scene(seed: int = 1, h: float = 0.035, n_envs: int = 8, pose_seed: int = 100,
                 n_el: int = 32, n_az: int = 1024) -> Scene:
    """Closed indoor mesh (room + 200 primitives, marching cubes at spacing h)
    with ``n_envs`` seeded free-space poses and a 32-beam spinning pattern
    over -16..+15 deg x ``n_az`` azimuths; range [0.1, 120] m."""
    sdf, v, t = indoor_mesh(seed, h)
    poses = free_space_poses(sdf, n_envs, pose_seed)
    dirs = lidar_pattern(n_el, -16.0, 15.0, n_az)
    return Scene(f"indoor_h{h:g}", v, t, poses, dirs, 0.1, 120.0, n_az,
                 {"sdf": sdf, "h": h, "seed": seed})


# --------------------------------------------------------------------------
# Outdoor terrain

def _value_noise(rng, x, y, octaves=6, base_wavelength=50.0, amplitude=8.0):
    """Fractal (fBm) value noise on a seeded lattice, smoothstep-interpolated."""
    out = np.zeros_like(x)
    amp, wl = amplitude, base_wavelength
    for _ in range(octaves):
        n = int(np.ceil(220.0 / wl)) + 3
        lat = rng.uniform(-1.0, 1.0, size=(n, n))
        gx, gy = (x + 10.0) / wl, (y + 10.0) / wl
        ix, iy = np.floor(gx).astype(np.int64), np.floor(gy).astype(np.int64)
        fx, fy = gx - ix, gy - iy
        sx, sy = fx * fx * (3 - 2 * fx), fy * fy * (3 - 2 * fy)
        a = lat[ix, iy]
        b = lat[ix + 1, iy]
        c = lat[ix, iy + 1]
        d = lat[ix + 1, iy + 1]
        out += amp * ((a * (1 - sx) + b * sx) * (1 - sy) + (c * (1 - sx) + d * sx) * sy)
        amp *= 0.5
        wl *= 0.5
    return out


def _box_mesh(center, half, yaw):
    v, t = box_room(-np.asarray(half), np.asarray(half))
    v = v.astype(np.float64)
    c, s = math.cos(yaw), math.sin(yaw)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    return (v @ R.T + center).astype(np.float32), t


def terrain_scene(seed: int, n_tris_target: int, n_boxes: int = None, size: float = 200.0):
    """Heightfield over [0, size]^2 with grid g = size * sqrt(2 / N) (so about
    N triangles), fBm value noise (6 octaves, 50 m base wavelength, 8 m
    amplitude), plus 50..500 boxes (extent 0.5..5 m, yaw uniform, sunk 0.2 m
    into the ground).  Returns (verts, tris, heightfield sampler)."""
    rng = np.random.default_rng(seed)
    n_cells = max(2, int(round(math.sqrt(n_tris_target / 2.0))))
    g = size / n_cells
    xs = np.linspace(0.0, size, n_cells + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    noise_rng = np.random.default_rng(seed + 7919)
    Z = _value_noise(noise_rng, X, Y)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    idx = np.arange((n_cells + 1) ** 2).reshape(n_cells + 1, n_cells + 1)
    a, b = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    c, d = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], -1), np.stack([a, c, d], -1)])
    meshes = [(verts.astype(np.float32), tris.astype(np.int32))]

    def height(px, py):
        fx = np.clip(np.asarray(px) / g, 0, n_cells - 1e-9)
        fy = np.clip(np.asarray(py) / g, 0, n_cells - 1e-9)
        i, j = np.floor(fx).astype(int), np.floor(fy).astype(int)
        u, v = fx - i, fy - j
        z00, z10, z11, z01 = Z[i, j], Z[i + 1, j], Z[i + 1, j + 1], Z[i, j + 1]
        # matches the (a,b,c) / (a,c,d) split: lower triangle when v <= u
        lower = v <= u
        zl = z00 + u * (z10 - z00) + v * (z11 - z10)
        zu = z00 + v * (z01 - z00) + u * (z11 - z01)
        return np.where(lower, zl, zu)

    nb = n_boxes if n_boxes is not None else int(rng.integers(50, 501))
    boxes = []
    for _ in range(nb):
        half = rng.uniform(0.25, 2.5, size=3)
        cx, cy = rng.uniform(5.0, size - 5.0, size=2)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        cz = float(height(cx, cy)) + half[2] - 0.2
        meshes.append(_box_mesh(np.array([cx, cy, cz]), half, yaw))
        boxes.append((cx, cy, cz, *half, yaw))
    v, t = concat_meshes(*meshes)
    return v, t, height, np.array(boxes, np.float64).reshape(-1, 7)


def terrain_poses(height, boxes, n: int, seed: int, size: float = 200.0):
    """n poses 1.5..3 m above the terrain, outside every box, yaw uniform."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        x, y = rng.uniform(10.0, size - 10.0, size=2)
        inside = False
        for (cx, cy, cz, hx, hy, hz, yaw) in boxes:
            c, s = math.cos(yaw), math.sin(yaw)
            lx, ly = c * (x - cx) + s * (y - cy), -s * (x - cx) + c * (y - cy)
            if abs(lx) < hx + 0.5 and abs(ly) < hy + 0.5:
                inside = True
                break
        if inside:
            continue
        z = float(height(x, y)) + rng.uniform(1.5, 3.0)
        out.append(yaw_pose((x, y, z), rng.uniform(0.0, 2.0 * math.pi)))
    return np.ascontiguousarray(np.stack(out))


# --------------------------------------------------------------------------
# Uneven multi-scene batch

UNEVEN_PATTERNS = (
    # (n_el, el_lo, el_hi, n_az)
    (16, -15.0, 15.0, 360),
    (64, -25.0, 3.0, 1024),
    (128, -22.5, 22.5, 2048),
)


@dataclasses.dataclass
class UnevenWorld:
    scenes: list            # [(verts, tris)]
    env_scene: np.ndarray   # int32 [E]: scene of each environment
    env_pattern: np.ndarray # int32 [E]: index into patterns
    poses: np.ndarray       # float32 [E, 12]
    patterns: list          # float32 [B_i, 3] per pattern
    n_az: list
    t_min: float = 0.1
    t_max: float = 120.0

    @property
    def n_rays(self) -> int:
        return int(sum(len(self.patterns[p]) for p in self.env_pattern))


def uneven_world(seed: int = 0, n_scenes: int = 64, n_envs: int = 1024,
                 tri_lo: float = 50_000, tri_hi: float = 5_000_000) -> UnevenWorld:
    """Resident outdoor scenes with log-uniform triangle counts in
    [tri_lo, tri_hi] (heightfield + 50..500 boxes each); every environment is
    bound to a uniformly drawn scene and beam pattern, with a pose 1.5..3 m
    above that scene's ground."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi), n_scenes))
    scenes, samplers = [], []
    for k, n in enumerate(sizes):
        v, t, height, boxes = terrain_scene(seed * 1000 + k, int(n))
        scenes.append((v, t))
        samplers.append((height, boxes))
    env_scene = rng.integers(0, n_scenes, n_envs).astype(np.int32)
    env_pattern = rng.integers(0, len(UNEVEN_PATTERNS), n_envs).astype(np.int32)
    poses = np.zeros((n_envs, 12), np.float32)
    for k in range(n_scenes):
        idx = np.flatnonzero(env_scene == k)
        if len(idx):
            h, b = samplers[k]
            poses[idx] = terrain_poses(h, b, len(idx), seed * 7919 + k)
    patterns = [lidar_pattern(ne, lo, hi, na) for ne, lo, hi, na in UNEVEN_PATTERNS]
    return UnevenWorld(scenes, env_scene, env_pattern, poses, patterns,
                       [p[3] for p in UNEVEN_PATTERNS])


# --------------------------------------------------------------------------
# Gaussian scenes (inputs of the Gaussian-to-occupancy conversion)
#
# Layout: means float32 [n, 3]; quats float32 [n, 4] as (w, x, y, z), not
# necessarily unit length; scales float32 [n, 3] (linear, > 0); opacity
# float32 [n] in [0, 1].  Trained 3DGS assets are not available, so seeded
# Gaussians with their structure stand in: flat discs lying on surfaces,
# plus a few low-opacity floaters in free space.

def random_gaussians(rng: np.random.Generator, n: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                     s_lo: float = 0.02, s_hi: float = 0.2, a_lo: float = 0.05, a_hi: float = 1.0):
    """n Gaussians: means uniform in [lo, hi], quaternions with normal
    components (arbitrary length), scales log-uniform in [s_lo, s_hi],
    opacity uniform in [a_lo, a_hi]."""
    means = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    quats = rng.normal(size=(n, 4)).astype(np.float32)
    scales = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), (n, 3))).astype(np.float32)
    opac = rng.uniform(a_lo, a_hi, n).astype(np.float32)
    return means, quats, scales, opac


def _quat_mul(a, b):
    """Hamilton product of (w, x, y, z) quaternion arrays."""
    aw, ax, ay, az = a[:, 0], a[:, 1], a[:, 2], a[:, 3]
    bw, bx, by, bz = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=1)


def splat_scene(seed: int = 1, n: int = 1_000_000, h_mesh: float = 0.035,
                floaters: float = 0.03, tan_scale: float = 0.02):
    """3DGS-like Gaussians on the indoor scene (room + 200 primitives,
    marching cubes at ``h_mesh``): points sampled uniformly by area on the
    surface, the disc normal (smallest scale) along the surface normal with a
    random twist, tangential scales log-normal around ``tan_scale`` metres,
    normal scale 20..60 % of the smaller tangential one; opacity mostly high.
    A ``floaters`` fraction lies in free space: near-isotropic, 1..10 cm,
    opacity 0.01..0.2.  Returns (means, quats, scales, opacity, room box)."""
    sdf, v, t = indoor_mesh(seed, h_mesh)
    rng = np.random.default_rng(1000 + seed)
    n_float = int(round(n * floaters))
    n_surf = n - n_float
    a = v[t[:, 0]].astype(np.float64)
    b = v[t[:, 1]].astype(np.float64)
    c = v[t[:, 2]].astype(np.float64)
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    ok = area > 0
    cdf = np.cumsum(np.where(ok, area, 0.0))
    pick = np.searchsorted(cdf, rng.uniform(0, cdf[-1], n_surf), side="right")
    pick = np.minimum(pick, len(area) - 1)
    r1 = np.sqrt(rng.uniform(size=n_surf))
    r2 = rng.uniform(size=n_surf)
    pts = ((1 - r1)[:, None] * a[pick] + (r1 * (1 - r2))[:, None] * b[pick]
           + (r1 * r2)[:, None] * c[pick])
    nrm = cr[pick] / np.linalg.norm(cr[pick], axis=1, keepdims=True)
    # rotation taking +z to the normal, then a random twist about it
    qa = np.stack([1 + nrm[:, 2], -nrm[:, 1], nrm[:, 0], np.zeros(n_surf)], axis=1)
    flip = qa[:, 0] < 1e-9
    qa[flip] = (0.0, 1.0, 0.0, 0.0)
    qa /= np.linalg.norm(qa, axis=1, keepdims=True)
    phi = rng.uniform(0, 2 * math.pi, n_surf)
    qt = np.stack([np.cos(phi / 2), np.zeros(n_surf), np.zeros(n_surf), np.sin(phi / 2)], axis=1)
    q_surf = _quat_mul(qa, qt)
    st = np.exp(rng.normal(math.log(tan_scale), 0.4, (n_surf, 2)))
    sn = np.minimum(st[:, 0], st[:, 1]) * rng.uniform(0.2, 0.6, n_surf)
    s_surf = np.stack([st[:, 0], st[:, 1], sn], axis=1)
    hi_op = rng.uniform(size=n_surf) < 0.7
    a_surf = np.where(hi_op, rng.uniform(0.6, 1.0, n_surf), rng.uniform(0.05, 0.6, n_surf))
    lo, hi = np.asarray(sdf.room[:3]), np.asarray(sdf.room[3:])
    m_fl = rng.uniform(lo, hi, (n_float, 3))
    q_fl = rng.normal(size=(n_float, 4))
    base = np.exp(rng.uniform(math.log(0.01), math.log(0.1), n_float))
    s_fl = base[:, None] * rng.uniform(0.7, 1.3, (n_float, 3))
    a_fl = rng.uniform(0.01, 0.2, n_float)
    means = np.concatenate([pts, m_fl]).astype(np.float32)
    quats = np.concatenate([q_surf, q_fl]).astype(np.float32)
    scales = np.concatenate([s_surf, s_fl]).astype(np.float32)
    opac = np.concatenate([a_surf, a_fl]).astype(np.float32)
    perm = rng.permutation(n)
    return (np.ascontiguousarray(means[perm]), np.ascontiguousarray(quats[perm]),
            np.ascontiguousarray(scales[perm]), np.ascontiguousarray(opac[perm]),
            np.asarray(sdf.room, dtype=np.float64))
