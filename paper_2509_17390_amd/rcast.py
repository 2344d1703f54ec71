"""Thin ctypes binding of librcast (include/rcast.h).

Argument marshalling only: every step of the ray-casting path runs in the
HIP library.  PyTorch supplies device memory and the current stream.  If
the library has not been built, every entry point raises -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "librcast.so")

RC_OK = 0
RC_PENDING = 1
RC_E_INVAL = -1
RC_E_NOMEM = -2
RC_E_NOTFOUND = -3
RC_E_BUSY = -4
RC_E_DEVICE = -5
RC_E_STATE = -6

RC_NODE_FP32 = 0
RC_NODE_Q8 = 1

RC_DBG_MORTON = 1
RC_DBG_SORTED = 2
RC_DBG_TOPOLOGY = 3
RC_DBG_NODES = 4
RC_DBG_TRIS = 5
RC_DBG_Q8NODES = 6

RC_GDBG_BOXES = 1
RC_GDBG_SORTED = 2
RC_GDBG_TOPOLOGY = 3
RC_GDBG_RECORDS = 4

# every symbol include/rcast.h declares
EXPORTED = [
    "rc_last_error", "rc_version", "rc_create", "rc_destroy", "rc_scene_upload",
    "rc_lbvh_build", "rc_scene_release", "rc_pattern_upload", "rc_raycast_batch",
    "rc_raycast_batch_noalloc",
    "rc_raycast_bruteforce", "rc_raycast_stats", "rc_scene_get_info",
    "rc_scene_debug_copy", "rc_device_bytes", "rc_set_tuning", "rc_get_tuning",
    "rc_autotune", "rc_graph_create", "rc_graph_launch", "rc_graph_destroy",
    "rc_serve_start", "rc_serve_stop", "rc_serve_submit", "rc_serve_poll", "rc_serve_release",
    "rc_serve_copy", "rc_serve_get_stats", "rc_gauss_upload", "rc_gauss_build",
    "rc_gauss_release", "rc_voxelize", "rc_voxelize_counts", "rc_gauss_debug_copy",
    "rc_tsdf", "rc_marching_cubes", "rc_marching_cubes_step", "rc_marching_cubes_table",
    "rc_nearest",
    "rc_chamfer_fscore", "rc_taubin_smooth", "rc_decimate", "rc_decimate_qem",
    "rc_remove_small_components",
    "rc_calib_gather", "rc_calib_valu", "rc_tuning_cache_load", "rc_tuning_cache_save",
]

RC_DEVICE_MOCK = -1


class RcastError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rcast error {status}: {msg}")
        self.status = status


class rc_build_opts(ctypes.Structure):
    _fields_ = [("morton_bits", ctypes.c_int32), ("node_format", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class rc_job(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("pattern", ctypes.c_int32),
                ("n_envs", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("poses_3x4", ctypes.c_void_p), ("t_min", ctypes.c_float),
                ("t_max", ctypes.c_float), ("out_offset", ctypes.c_int64)]


class rc_scene_info(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int64), ("n_tris", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("n_q8_nodes", ctypes.c_int64),
                ("depth", ctypes.c_int32),
                ("node_format", ctypes.c_int32), ("morton_bits", ctypes.c_int32),
                ("has_bvh", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("scene_lo", ctypes.c_float * 3), ("scene_hi", ctypes.c_float * 3)]


class rc_tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("stack_lds", ctypes.c_int32),
                ("refill_min", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tile_az", ctypes.c_int32), ("tile_el", ctypes.c_int32),
                ("chunk_max", ctypes.c_int32), ("waves_cap", ctypes.c_int32),
                ("group_waves", ctypes.c_int32), ("leaf_batch", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rc_request(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("pattern", ctypes.c_int32),
                ("n_envs", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("poses_3x4", ctypes.c_void_p), ("t_min", ctypes.c_float),
                ("t_max", ctypes.c_float)]


class rc_serve_opts(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("max_batch_rays_m", ctypes.c_int32), ("mock_ns_per_ray", ctypes.c_int32),
                ("mock_fail_scene", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("max_wait_ms", ctypes.c_int32), ("mock_launch_delay_us", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


class rc_serve_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "submitted", "completed", "failed", "rejected", "cancelled", "launches",
        "max_batch_requests", "bytes_in_use", "peak_bytes", "out_capacity_bytes", "pending",
        "inflight", "peak_inflight")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class rc_gauss_opts(ctypes.Structure):
    _fields_ = [("cutoff_sigma", ctypes.c_float), ("morton_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class rc_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float),
                ("dims", ctypes.c_int32 * 3), ("tile", ctypes.c_int32),
                ("theta", ctypes.c_float), ("reserved", ctypes.c_int32 * 3)]


class rc_tsdf_opts(ctypes.Structure):
    _fields_ = [("sigma_smooth", ctypes.c_float), ("tau", ctypes.c_float),
                ("band", ctypes.c_float), ("threshold_mode", ctypes.c_int32),
                ("quantile", ctypes.c_float), ("reserved", ctypes.c_int32 * 3)]


class rc_fidelity(ctypes.Structure):
    _fields_ = [("chamfer", ctypes.c_double), ("mean_pg", ctypes.c_double),
                ("mean_gp", ctypes.c_double), ("precision", ctypes.c_double),
                ("recall", ctypes.c_double), ("fscore", ctypes.c_double),
                ("n_p", ctypes.c_int64), ("n_g", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """Load librcast.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2509_17390_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    S = ctypes.c_int
    sig = {
        "rc_last_error": ([], ctypes.c_char_p),
        "rc_version": ([], I32),
        "rc_create": ([ctypes.c_int, U64, ctypes.POINTER(P)], S),
        "rc_destroy": ([P], None),
        "rc_scene_upload": ([P, P, I64, P, I64, ctypes.c_int, P, ctypes.POINTER(I32)], S),
        "rc_lbvh_build": ([P, I32, ctypes.POINTER(rc_build_opts), P], S),
        "rc_scene_release": ([P, I32], S),
        "rc_pattern_upload": ([P, P, I32, I32, ctypes.POINTER(I32)], S),
        "rc_raycast_batch": ([P, ctypes.POINTER(rc_job), I32, P, P, P], S),
        "rc_raycast_batch_noalloc": ([P, ctypes.POINTER(rc_job), I32, P, P, P], S),
        "rc_raycast_bruteforce": ([P, ctypes.POINTER(rc_job), I32, P, P, P], S),
        "rc_raycast_stats": ([P, ctypes.POINTER(rc_job), I32, P, P, P, P, P], S),
        "rc_scene_get_info": ([P, I32, ctypes.POINTER(rc_scene_info)], S),
        "rc_scene_debug_copy": ([P, I32, I32, P, U64], S),
        "rc_device_bytes": ([P], U64),
        "rc_set_tuning": ([P, ctypes.POINTER(rc_tuning)], S),
        "rc_get_tuning": ([P, ctypes.POINTER(rc_tuning)], S),
        "rc_autotune": ([P, ctypes.POINTER(rc_job), I32, P, P, P, I32, ctypes.POINTER(rc_tuning),
                         ctypes.POINTER(ctypes.c_float)], S),
        "rc_graph_create": ([P, ctypes.POINTER(rc_job), I32, P, P, ctypes.POINTER(P)], S),
        "rc_graph_launch": ([P, P], S),
        "rc_graph_destroy": ([P], None),
        "rc_serve_start": ([P, ctypes.POINTER(rc_serve_opts)], S),
        "rc_serve_stop": ([P], S),
        "rc_serve_submit": ([P, ctypes.POINTER(rc_request), ctypes.POINTER(U64)], S),
        "rc_serve_poll": ([P, U64, I64, ctypes.POINTER(P), ctypes.POINTER(P),
                           ctypes.POINTER(ctypes.c_double)], S),
        "rc_serve_release": ([P, U64], S),
        "rc_serve_copy": ([P, U64, P, P, ctypes.c_int], S),
        "rc_serve_get_stats": ([P, ctypes.POINTER(rc_serve_stats)], S),
        "rc_gauss_upload": ([P, P, P, P, P, I64, ctypes.c_int, P, ctypes.POINTER(I32)], S),
        "rc_gauss_build": ([P, I32, ctypes.POINTER(rc_gauss_opts), P], S),
        "rc_gauss_release": ([P, I32], S),
        "rc_voxelize": ([P, I32, ctypes.POINTER(rc_grid), P, P, P, P], S),
        "rc_voxelize_counts": ([P, I32, ctypes.POINTER(rc_grid), P, P], S),
        "rc_gauss_debug_copy": ([P, I32, I32, P, U64], S),
        "rc_tsdf": ([P, ctypes.POINTER(rc_grid), P, ctypes.POINTER(rc_tsdf_opts), P, P, P], S),
        "rc_marching_cubes": ([P, ctypes.POINTER(rc_grid), P, ctypes.c_float, P, P, P, I64, I64,
                               ctypes.POINTER(I64), ctypes.POINTER(I64), P], S),
        "rc_marching_cubes_step": ([P, ctypes.POINTER(rc_grid), P, ctypes.c_float, I32, P, P, P,
                                    I64, I64, ctypes.POINTER(I64), ctypes.POINTER(I64), P], S),
        "rc_marching_cubes_table": ([P, P], S),
        "rc_nearest": ([P, P, I64, P, I64, P, P, P], S),
        "rc_taubin_smooth": ([P, P, I64, P, I64, ctypes.c_float, ctypes.c_float, I32, P], S),
        "rc_decimate": ([P, P, I64, P, I64, ctypes.c_float, P, P, ctypes.POINTER(I64),
                         ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_float), P], S),
        "rc_decimate_qem": ([P, P, I64, P, I64, ctypes.c_float, I32, P, P, ctypes.POINTER(I64),
                             ctypes.POINTER(I64), ctypes.POINTER(I32), P], S),
        "rc_remove_small_components": ([P, P, I64, P, I64, I64, P, P, ctypes.POINTER(I64),
                                        ctypes.POINTER(I64), P], S),
        "rc_chamfer_fscore": ([P, P, I64, P, I64, ctypes.c_float, ctypes.POINTER(rc_fidelity),
                               P], S),
        "rc_tuning_cache_load": ([P, ctypes.c_char_p], S),
        "rc_tuning_cache_save": ([P, ctypes.c_char_p], S),
        "rc_calib_gather": ([P, U64, I64, I32, P, P], S),
        "rc_calib_valu": ([I64, I32, I32, P, P], S),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def last_error() -> str:
    """Text of the last error the library reported on this thread."""
    msg = load().rc_last_error()
    return msg.decode() if msg else ""


def _check(status: int):
    if status != RC_OK:
        msg = load().rc_last_error()
        raise RcastError(status, msg.decode() if msg else "")


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(x) -> int:
    """Device pointer of a torch tensor (or host pointer of a numpy array)."""
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return int(x.data_ptr())


@dataclasses.dataclass
class Job:
    scene: int
    pattern: int
    poses: object            # torch float32 cuda tensor [n_envs, 12]
    t_min: float
    t_max: float
    out_offset: int = 0

    @property
    def n_envs(self) -> int:
        return int(self.poses.shape[0])


class Context:
    """A librcast context on one device."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.rc_create(int(device), int(budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device
        self._n_beams = {}

    def close(self):
        if getattr(self, "_h", None):
            load().rc_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass

    # -- scenes ---------------------------------------------------------------
    def upload_scene(self, verts, tris, stream=None) -> int:
        """verts [nv,3] float32, tris [nt,3] int32: numpy (host) or torch cuda."""
        on_dev = not isinstance(verts, np.ndarray)
        if on_dev:
            assert verts.is_cuda and tris.is_cuda and verts.is_contiguous() and tris.is_contiguous()
            nv, nt = int(verts.shape[0]), int(tris.shape[0])
            vp, tp = _ptr(verts), _ptr(tris)
            sp = _stream_ptr(stream)
        else:
            verts = np.ascontiguousarray(verts, np.float32).reshape(-1, 3)
            tris = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
            nv, nt = verts.shape[0], tris.shape[0]
            vp, tp = verts.ctypes.data, tris.ctypes.data
            sp = 0
        out = ctypes.c_int32()
        _check(load().rc_scene_upload(self._h, vp, nv, tp, nt, int(on_dev), sp, ctypes.byref(out)))
        return out.value

    def _sp(self, stream) -> int:
        return 0 if self.device == RC_DEVICE_MOCK else _stream_ptr(stream)

    def build(self, scene: int, morton_bits: int = 10, node_format: int = RC_NODE_FP32,
              stream=None):
        o = rc_build_opts(morton_bits, node_format)
        _check(load().rc_lbvh_build(self._h, scene, ctypes.byref(o), self._sp(stream)))

    def release_scene(self, scene: int):
        _check(load().rc_scene_release(self._h, scene))

    def scene_info(self, scene: int) -> rc_scene_info:
        info = rc_scene_info()
        _check(load().rc_scene_get_info(self._h, scene, ctypes.byref(info)))
        return info

    def debug_copy(self, scene: int, what: int) -> np.ndarray:
        info = self.scene_info(scene)
        nt, ni = info.n_tris, info.n_nodes
        if what == RC_DBG_MORTON or what == RC_DBG_SORTED:
            a = np.empty(nt, np.uint32)
        elif what == RC_DBG_TOPOLOGY:
            a = np.empty((ni, 3), np.int32)
        elif what == RC_DBG_NODES or what == RC_DBG_Q8NODES:
            a = np.empty((ni, 16), np.float32)
        elif what == RC_DBG_TRIS:
            a = np.empty((nt, 12), np.float32)
        else:
            raise ValueError(what)
        _check(load().rc_scene_debug_copy(self._h, scene, what, a.ctypes.data, a.nbytes))
        return a

    def device_bytes(self) -> int:
        return int(load().rc_device_bytes(self._h))

    def get_tuning(self) -> dict:
        t = rc_tuning()
        _check(load().rc_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Update traversal tuning fields (see rc_tuning); reset() restores defaults."""
        cur = self.get_tuning()
        cur.update(kw)
        t = rc_tuning(**cur)
        _check(load().rc_set_tuning(self._h, ctypes.byref(t)))

    def reset_tuning(self):
        _check(load().rc_set_tuning(self._h, None))

    # -- Gaussian-to-occupancy conversion -------------------------------------
    def upload_gaussians(self, means, quats, scales, opacity, stream=None) -> int:
        """means [n,3], quats [n,4] (w,x,y,z), scales [n,3], opacity [n], float32:
        numpy (host) or torch cuda tensors."""
        arrs = [means, quats, scales, opacity]
        on_dev = not isinstance(means, np.ndarray)
        if on_dev:
            for a in arrs:
                assert a.is_cuda and a.is_contiguous()
            n = int(means.shape[0])
            ptrs = [_ptr(a) for a in arrs]
            sp = _stream_ptr(stream)
        else:
            widths = (3, 4, 3, 1)
            arrs = [np.ascontiguousarray(a, np.float32).reshape(-1, w) for a, w in zip(arrs, widths)]
            n = arrs[0].shape[0]
            ptrs = [a.ctypes.data for a in arrs]
            sp = 0
        out = ctypes.c_int32()
        _check(load().rc_gauss_upload(self._h, *ptrs, n, int(on_dev), sp, ctypes.byref(out)))
        self._gauss_n = getattr(self, "_gauss_n", {})
        self._gauss_n[out.value] = n
        return out.value

    def build_gaussians(self, gset: int, cutoff_sigma: float = 3.0, morton_bits: int = 10,
                        stream=None):
        o = rc_gauss_opts(float(cutoff_sigma), int(morton_bits))
        _check(load().rc_gauss_build(self._h, gset, ctypes.byref(o), _stream_ptr(stream)))

    def release_gaussians(self, gset: int):
        _check(load().rc_gauss_release(self._h, gset))

    @staticmethod
    def grid(origin, spacing: float, dims, theta: float, tile: int = 8) -> rc_grid:
        g = rc_grid()
        for a in range(3):
            g.origin[a] = float(origin[a])
            g.dims[a] = int(dims[a])
        g.spacing = float(spacing)
        g.tile = int(tile)
        g.theta = float(theta)
        return g

    def voxelize(self, gset: int, grid: rc_grid, out_density=None, out_occ=None, out_surf=None,
                 stream=None):
        """Device outputs (torch cuda tensors, [nz, ny, nx]): float32 density,
        uint8 occupancy, uint8 surface mask; any may be None."""
        p = [0 if t is None else _ptr(t) for t in (out_density, out_occ, out_surf)]
        _check(load().rc_voxelize(self._h, gset, ctypes.byref(grid), *p, _stream_ptr(stream)))

    def voxelize_counts(self, gset: int, grid: rc_grid, out_counts, stream=None):
        _check(load().rc_voxelize_counts(self._h, gset, ctypes.byref(grid), _ptr(out_counts),
                                         _stream_ptr(stream)))

    def gauss_debug_copy(self, gset: int, what: int) -> np.ndarray:
        n = self._gauss_n[gset]
        if what == RC_GDBG_BOXES:
            a = np.empty((n, 6), np.float32)
        elif what == RC_GDBG_SORTED:
            a = np.empty(n, np.uint32)
        elif what == RC_GDBG_TOPOLOGY:
            a = np.empty((max(n - 1, 0), 3), np.int32)
        elif what == RC_GDBG_RECORDS:
            a = np.empty((n, 16), np.float32)
        else:
            raise ValueError(what)
        _check(load().rc_gauss_debug_copy(self._h, gset, what, a.ctypes.data, a.nbytes))
        return a

    def tsdf(self, grid: rc_grid, surf, out_phi, sigma_smooth: float, tau: float, band: float,
             out_vtilde=None, stream=None, quantile=None):
        """Narrow-band TSDF of a device uint8 surface mask into device float32
        out_phi (both [nz, ny, nx]); synchronous.  With quantile = q the
        re-threshold is V' >= Quantile_q(V') (tau unused)."""
        o = rc_tsdf_opts(float(sigma_smooth), float(tau), float(band),
                         0 if quantile is None else 1,
                         0.0 if quantile is None else float(quantile))
        _check(load().rc_tsdf(self._h, ctypes.byref(grid), _ptr(surf), ctypes.byref(o),
                              _ptr(out_phi), 0 if out_vtilde is None else _ptr(out_vtilde),
                              _stream_ptr(stream)))

    def marching_cubes(self, grid: rc_grid, phi, iso: float = 0.0, stream=None,
                       normals: bool = False, step: int = 1):
        """Mesh of a device float32 field: (verts [nv, 3] float32, tris [nt, 3]
        int32) as torch cuda tensors; with normals=True also the unit vertex
        normals [nv, 3] float32 from the gradient of phi; step = mc_step
        (every step-th lattice point, rc_marching_cubes_step)."""
        import torch
        nv, nt = ctypes.c_int64(), ctypes.c_int64()
        lib = load()
        sp = _stream_ptr(stream)
        dev = phi.device

        def fill(cv, ct):
            verts = torch.empty((cv, 3), dtype=torch.float32, device=dev)
            tris = torch.empty((ct, 3), dtype=torch.int32, device=dev)
            nrm = torch.empty((cv, 3), dtype=torch.float32, device=dev) if normals else None
            st = lib.rc_marching_cubes_step(self._h, ctypes.byref(grid), _ptr(phi), float(iso),
                                            int(step), _ptr(verts), _ptr(tris),
                                            _ptr(nrm) if normals else None, cv, ct,
                                            ctypes.byref(nv), ctypes.byref(nt), sp)
            out = (verts[:nv.value], tris[:nt.value])
            return st, (out + (nrm[:nv.value],) if normals else out)

        cap_v, cap_t = getattr(self, "_mc_cap", (0, 0))
        if cap_v and cap_t:
            # the previous mesh's size (+10 %) as capacity: one pass if it fits
            st, out = fill(cap_v, cap_t)
            if st == RC_OK:
                return out
            if st != RC_E_NOMEM:
                _check(st)
        else:
            _check(lib.rc_marching_cubes_step(self._h, ctypes.byref(grid), _ptr(phi),
                                              float(iso), int(step), None, None, None, 0, 0,
                                              ctypes.byref(nv), ctypes.byref(nt), sp))
        self._mc_cap = (max(1, int(nv.value * 1.1) + 16), max(1, int(nt.value * 1.1) + 16))
        st, out = fill(max(nv.value, 1), max(nt.value, 1))
        _check(st)
        return out

    # -- mesh optimisation -------------------------------------------------------
    def taubin(self, verts, tris, lam: float = 0.5, mu: float = -0.53, iterations: int = 10,
               stream=None):
        """Taubin smoothing in place of a device float32 [nv, 3] vertex tensor."""
        assert verts.is_cuda and verts.is_contiguous() and tris.is_cuda and tris.is_contiguous()
        _check(load().rc_taubin_smooth(self._h, _ptr(verts), int(verts.shape[0]), _ptr(tris),
                                       int(tris.shape[0]), float(lam), float(mu),
                                       int(iterations), _stream_ptr(stream)))

    def decimate(self, verts, tris, ratio: float = 0.1, stream=None):
        """Quadric-error decimation of a device mesh: (verts, tris, cell size)."""
        import torch
        nv, nt = int(verts.shape[0]), int(tris.shape[0])
        ov = torch.empty((nv, 3), dtype=torch.float32, device=verts.device)
        ot_ = torch.empty((nt, 3), dtype=torch.int32, device=verts.device)
        n_v, n_t, cell = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_float()
        _check(load().rc_decimate(self._h, _ptr(verts), nv, _ptr(tris), nt, float(ratio),
                                  _ptr(ov), _ptr(ot_), ctypes.byref(n_v), ctypes.byref(n_t),
                                  ctypes.byref(cell), _stream_ptr(stream)))
        return ov[:n_v.value], ot_[:n_t.value], cell.value

    def decimate_qem(self, verts, tris, ratio: float = 0.1, rounds: int = 3, stream=None):
        """Quadric-error decimation by rounds of parallel edge contraction of a
        device mesh: (verts, tris, contraction steps)."""
        import torch
        nv, nt = int(verts.shape[0]), int(tris.shape[0])
        ov = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=verts.device)
        ot_ = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=verts.device)
        n_v, n_t, n_s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(load().rc_decimate_qem(self._h, _ptr(verts), nv, _ptr(tris), nt, float(ratio),
                                      int(rounds), _ptr(ov), _ptr(ot_), ctypes.byref(n_v),
                                      ctypes.byref(n_t), ctypes.byref(n_s), _stream_ptr(stream)))
        return ov[:n_v.value], ot_[:n_t.value], n_s.value

    def remove_small_components(self, verts, tris, min_faces: int, stream=None):
        """Drop the components of fewer than min_faces triangles of a device
        mesh: (verts, tris) as torch cuda tensors."""
        import torch
        nv, nt = int(verts.shape[0]), int(tris.shape[0])
        ov = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=verts.device)
        ot_ = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=verts.device)
        n_v, n_t = ctypes.c_int64(), ctypes.c_int64()
        _check(load().rc_remove_small_components(
            self._h, _ptr(verts) if nv else None, nv, _ptr(tris) if nt else None, nt,
            int(min_faces), _ptr(ov), _ptr(ot_), ctypes.byref(n_v), ctypes.byref(n_t),
            _stream_ptr(stream)))
        return ov[:n_v.value], ot_[:n_t.value]

    # -- point-cloud fidelity --------------------------------------------------
    def nearest(self, ref, query, stream=None):
        """Nearest reference point of every query (device float32 [n, 3]
        tensors): (distances float64, indices int32) as torch cuda tensors."""
        import torch
        n_q = int(query.shape[0])
        d = torch.empty(max(n_q, 1), dtype=torch.float64, device=query.device)
        i = torch.empty(max(n_q, 1), dtype=torch.int32, device=query.device)
        _check(load().rc_nearest(self._h, _ptr(ref) if ref.shape[0] else None, int(ref.shape[0]),
                                 _ptr(query) if n_q else None, n_q, _ptr(d), _ptr(i),
                                 _stream_ptr(stream)))
        return d[:n_q], i[:n_q]

    def chamfer_fscore(self, P, G, tau: float = 0.05, stream=None) -> dict:
        """CD and F-score of device float32 clouds P, G ([n, 3] tensors)."""
        out = rc_fidelity()
        _check(load().rc_chamfer_fscore(self._h, _ptr(P), int(P.shape[0]), _ptr(G),
                                        int(G.shape[0]), float(tau), ctypes.byref(out),
                                        _stream_ptr(stream)))
        return out.as_dict()

    # -- patterns ------------------------------------------------------------
    def upload_pattern(self, dirs, n_az: int = 0) -> int:
        d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
        out = ctypes.c_int32()
        _check(load().rc_pattern_upload(self._h, d.ctypes.data, d.shape[0], int(n_az),
                                        ctypes.byref(out)))
        self._n_beams[out.value] = d.shape[0]
        return out.value

    def n_beams(self, pattern: int) -> int:
        return self._n_beams[pattern]

    # -- ray casting ---------------------------------------------------------
    @staticmethod
    def _jobs(jobs: Sequence[Job]):
        arr = (rc_job * max(1, len(jobs)))()
        for i, j in enumerate(jobs):
            assert j.poses.is_cuda and j.poses.is_contiguous()
            arr[i] = rc_job(int(j.scene), int(j.pattern), j.n_envs, 0, _ptr(j.poses),
                            float(j.t_min), float(j.t_max), int(j.out_offset))
        return arr

    def raycast(self, jobs: Sequence[Job], out_range, out_hit, stream=None, mode: str = "bvh",
                out_nodes=None, out_tris=None):
        arr = self._jobs(jobs)
        lib = load()
        sp = _stream_ptr(stream)
        if mode == "bvh":
            _check(lib.rc_raycast_batch(self._h, arr, len(jobs), _ptr(out_range), _ptr(out_hit), sp))
        elif mode == "noalloc":
            _check(lib.rc_raycast_batch_noalloc(self._h, arr, len(jobs), _ptr(out_range),
                                                _ptr(out_hit), sp))
        elif mode == "brute":
            _check(lib.rc_raycast_bruteforce(self._h, arr, len(jobs), _ptr(out_range),
                                             _ptr(out_hit), sp))
        elif mode == "stats":
            _check(lib.rc_raycast_stats(self._h, arr, len(jobs), _ptr(out_range), _ptr(out_hit),
                                        _ptr(out_nodes), _ptr(out_tris), sp))
        else:
            raise ValueError(mode)

    def autotune(self, jobs: Sequence[Job], out_range, out_hit, reps: int = 2, stream=None):
        """Time the candidate launch shapes on this batch; keep and return the
        fastest (dict) and its time in ms."""
        arr = self._jobs(jobs)
        best = rc_tuning()
        ms = ctypes.c_float()
        _check(load().rc_autotune(self._h, arr, len(jobs), _ptr(out_range), _ptr(out_hit),
                                  _stream_ptr(stream), int(reps), ctypes.byref(best),
                                  ctypes.byref(ms)))
        return best.as_dict(), float(ms.value)

    def tuning_cache_load(self, path: str):
        """Load persisted autotuner results (a missing file is an empty cache)
        and make autotune() consult and extend them; autotune() then reports
        ms = -1 for a batch found in the cache."""
        _check(load().rc_tuning_cache_load(self._h, os.fsencode(path)))

    def tuning_cache_save(self, path: str):
        _check(load().rc_tuning_cache_save(self._h, os.fsencode(path)))

    def graph(self, jobs: Sequence[Job], out_range, out_hit) -> "Graph":
        return Graph(self, jobs, out_range, out_hit)

    # -- serving -------------------------------------------------------------
    def serve_start(self, arena_bytes: int = 0, max_inflight: int = 0, max_batch_rays_m: int = 0,
                    mock_ns_per_ray: int = 0, mock_fail_scene: int = 0, policy: int = 0,
                    max_wait_ms: int = 0, mock_launch_delay_us: int = 0):
        o = rc_serve_opts(arena_bytes, max_inflight, max_batch_rays_m, mock_ns_per_ray,
                          mock_fail_scene, policy, max_wait_ms, mock_launch_delay_us)
        _check(load().rc_serve_start(self._h, ctypes.byref(o)))

    def serve_stop(self):
        _check(load().rc_serve_stop(self._h))

    def submit(self, scene: int, pattern: int, poses, t_min: float, t_max: float) -> int:
        """Queue a request; poses are host float32 [n_envs, 12] (copied)."""
        p = np.ascontiguousarray(poses, np.float32).reshape(-1, 12)
        rq = rc_request(int(scene), int(pattern), p.shape[0], 0, p.ctypes.data, float(t_min),
                        float(t_max))
        t = ctypes.c_uint64()
        _check(load().rc_serve_submit(self._h, ctypes.byref(rq), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, timeout_us: int = 0):
        """(status, latency_ms); status RC_OK, RC_PENDING or an error code
        (its text: ``last_error()`` on the same thread)."""
        r, h = ctypes.c_void_p(), ctypes.c_void_p()
        lat = ctypes.c_double()
        st = load().rc_serve_poll(self._h, int(ticket), int(timeout_us), ctypes.byref(r),
                                  ctypes.byref(h), ctypes.byref(lat))
        return st, float(lat.value)

    def fetch(self, ticket: int, n_rays: int):
        """Copy a finished ticket's results to host numpy arrays."""
        rng = np.empty(n_rays, np.float32)
        hit = np.empty(n_rays, np.int32)
        _check(load().rc_serve_copy(self._h, int(ticket), rng.ctypes.data, hit.ctypes.data, 1))
        return rng, hit

    def fetch_into(self, ticket: int, out_range, out_hit):
        """Copy a finished ticket's results into device tensors."""
        _check(load().rc_serve_copy(self._h, int(ticket), _ptr(out_range), _ptr(out_hit), 0))

    def release(self, ticket: int):
        _check(load().rc_serve_release(self._h, int(ticket)))

    def serve_stats(self) -> dict:
        st = rc_serve_stats()
        _check(load().rc_serve_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def total_rays(self, jobs: Sequence[Job]) -> int:
        return max((j.out_offset + j.n_envs * self.n_beams(j.pattern) for j in jobs), default=0)

    def cast(self, jobs: Sequence[Job], mode: str = "bvh", stream=None):
        """Allocate outputs, cast, and return (range, hit) torch tensors."""
        import torch
        n = self.total_rays(jobs)
        dev = torch.device("cuda", self.device)
        rng = torch.empty(n, dtype=torch.float32, device=dev)
        hit = torch.empty(n, dtype=torch.int32, device=dev)
        if mode == "stats":
            nodes = torch.empty(n, dtype=torch.int32, device=dev)
            tris = torch.empty(n, dtype=torch.int32, device=dev)
            self.raycast(jobs, rng, hit, stream, mode, nodes, tris)
            return rng, hit, nodes, tris
        self.raycast(jobs, rng, hit, stream, mode)
        return rng, hit


class Graph:
    """A batch captured once (rc_graph_create) and replayed with launch()."""

    def __init__(self, ctx: Context, jobs: Sequence[Job], out_range, out_hit):
        self._ctx = ctx
        self._keep = (list(jobs), out_range, out_hit)   # keep buffers alive
        h = ctypes.c_void_p()
        _check(load().rc_graph_create(ctx._h, Context._jobs(jobs), len(jobs), _ptr(out_range),
                                      _ptr(out_hit), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load().rc_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().rc_graph_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass


def marching_cubes_table():
    """The library's marching-cubes case table: (count uint8 [256], tris int8
    [256, 15])."""
    count = np.zeros(256, np.uint8)
    tris = np.zeros((256, 15), np.int8)
    _check(load().rc_marching_cubes_table(count.ctypes.data, tris.ctypes.data))
    return count, tris
