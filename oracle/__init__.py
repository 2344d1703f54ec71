"""FP64 CPU oracle for batched LiDAR ray casting -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and the two share no
code.  The arithmetic lives in ``oracle.c`` (plain C, FP64); this module only
compiles it with gcc and marshals numpy arrays through ctypes.

What the oracle computes is the nearest-intersection definition of FGGS-LiDAR
Sec. IV-C written out as the naive O(N_rays * N_tris) loop; see the header of
``oracle.c`` for the readings taken where the paper is silent.

Every function here is pinned by tests in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")

FLAG_EDGE_NEAR = 1
FLAG_AMBIGUOUS = 2
EDGE_EPS_RAD = 1e-6


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so with gcc (no fast-math, no FMA)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
             "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
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
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_make_rays.argtypes = [P, I64, P, I64, P, P]
        lib.oracle_make_rays.restype = None
        lib.oracle_tri_test.argtypes = [P, P, P, P, P, P]
        lib.oracle_tri_test.restype = ctypes.c_int
        lib.oracle_edge_angle.argtypes = [P, P, P, P]
        lib.oracle_edge_angle.restype = D
        lib.oracle_raycast.argtypes = [P, I64, P, I64, P, P, I64, P, I64, D, D,
                                       P, P, ctypes.c_int]
        lib.oracle_raycast.restype = ctypes.c_int
        lib.oracle_raycast_checked.argtypes = [P, I64, P, I64, P, P, I64, P, I64,
                                               D, D, D, P, P, P, P, P, ctypes.c_int]
        lib.oracle_raycast_checked.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(a, shape_tail):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.shape[-len(shape_tail):] == shape_tail, a.shape
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def make_rays(poses, dirs):
    """FP64 rays of Sec. IV-C: o = t_e, d = normalize(R_e b_j); [E*B, 3] each."""
    poses = _f32(poses, (12,)).reshape(-1, 12)
    dirs = _f32(dirs, (3,)).reshape(-1, 3)
    n = poses.shape[0] * dirs.shape[0]
    o = np.empty((n, 3), np.float64)
    d = np.empty((n, 3), np.float64)
    _load().oracle_make_rays(_ptr(poses), poses.shape[0], _ptr(dirs), dirs.shape[0],
                             _ptr(o), _ptr(d))
    return o, d


def tri_test(o, d, v0, v1, v2):
    """FP64 watertight test of one ray against one triangle: t or None."""
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    v = [np.ascontiguousarray(x, np.float32) for x in (v0, v1, v2)]
    t = np.zeros(1, np.float64)
    hit = _load().oracle_tri_test(_ptr(o), _ptr(d), _ptr(v[0]), _ptr(v[1]), _ptr(v[2]), _ptr(t))
    return float(t[0]) if hit else None


def edge_angle(o, d, a, b) -> float:
    """Angular distance (rad) from unit d to the arc of edge (a, b) seen from o."""
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    return float(_load().oracle_edge_angle(_ptr(o), _ptr(d), _ptr(a), _ptr(b)))


def raycast(verts, tris, poses, dirs, t_min, t_max, ray_idx=None, threads=None,
            checked=False, eps_rad=EDGE_EPS_RAD):
    """Closest hit of every (env, beam) ray, or of the flattened indices in
    ``ray_idx`` (e * n_beams + b).

    Returns ``(t, id)`` -- FP64 range (+inf on a miss) and triangle id (-1 on
    a miss) -- or, with ``checked=True``, ``(t, id, flags, second_t,
    min_edge_angle)`` where flags holds FLAG_EDGE_NEAR / FLAG_AMBIGUOUS.
    """
    verts = _f32(verts, (3,)).reshape(-1, 3)
    tris = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
    poses = _f32(poses, (12,)).reshape(-1, 12)
    dirs = _f32(dirs, (3,)).reshape(-1, 3)
    if tris.size and (tris.min() < 0 or tris.max() >= verts.shape[0]):
        raise ValueError("triangle index out of range")
    n_beams = dirs.shape[0]
    if ray_idx is None:
        idx_p = None
        n = poses.shape[0] * n_beams
    else:
        ray_idx = np.ascontiguousarray(ray_idx, np.int64)
        if ray_idx.size and (ray_idx.min() < 0 or ray_idx.max() >= poses.shape[0] * n_beams):
            raise ValueError("ray index out of range")
        idx_p = _ptr(ray_idx)
        n = ray_idx.shape[0]
    threads = threads or default_threads()
    t = np.empty(n, np.float64)
    ids = np.empty(n, np.int32)
    lib = _load()
    if not checked:
        lib.oracle_raycast(_ptr(verts), verts.shape[0], _ptr(tris), tris.shape[0],
                           _ptr(poses), _ptr(dirs), n_beams, idx_p, n,
                           float(t_min), float(t_max), _ptr(t), _ptr(ids), threads)
        return t, ids
    flags = np.empty(n, np.int32)
    second = np.empty(n, np.float64)
    mina = np.empty(n, np.float64)
    lib.oracle_raycast_checked(_ptr(verts), verts.shape[0], _ptr(tris), tris.shape[0],
                               _ptr(poses), _ptr(dirs), n_beams, idx_p, n,
                               float(t_min), float(t_max), float(eps_rad),
                               _ptr(t), _ptr(ids), _ptr(flags), _ptr(second), _ptr(mina),
                               threads)
    return t, ids, flags, second, mina
