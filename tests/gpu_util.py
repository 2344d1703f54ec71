"""Helpers shared by the GPU tests: run a scene through librcast and compare
with the FP64 oracle under the parity bar.

Parity bar (per ray that the oracle's checker does not flag as edge-near --
within 1e-6 rad of a relevant triangle edge -- or ambiguous -- a second
surface within tol of the best hit, or a hit within tol of t_min / t_max):
  * hit/miss agreement on every such ray,
  * hit ids bit-exact,
  * |range_gpu - t_oracle| <= 1e-4 m + 1e-6 * t_oracle.
Flagged rays have several correct answers; for every one of them the GPU
answer must be one of those answers:
  * never beyond the oracle's nearest hit: range <= t* + 1e-3 + 1e-5 t*
    (a ray that slipped through a shared edge of the near surface and hit a
    triangle behind it fails here);
  * a miss where the oracle hits only on an edge-near ray, or when t* lies
    within tol of t_min or t_max (the FP32 distance may fall just outside);
  * a reported triangle really is hit by the ray near the reported range
    (or, for an edge-near ray that passed the neighbouring triangle, the
    range agrees with t*), inside [t_min - tol, t_max + tol].
"""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2509_17390_amd import Context, Job

TOL_ABS = 1e-4
TOL_REL = 1e-6


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def cast_scene(ctx: Context, verts, tris, poses, dirs, t_min, t_max, mode="bvh", n_az=0,
               build=True, morton_bits=10):
    """Upload, build, cast; returns numpy (range, hit) and the handles."""
    import torch
    scene = ctx.upload_scene(verts, tris)
    if build:
        ctx.build(scene, morton_bits=morton_bits)
    pat = ctx.upload_pattern(dirs, n_az)
    job = Job(scene, pat, cuda(poses), t_min, t_max, 0)
    out = ctx.cast([job], mode=mode)
    torch.cuda.synchronize()
    res = tuple(o.cpu().numpy() for o in out)
    return res, scene, pat


def oracle_checked(verts, tris, poses, dirs, t_min, t_max, ray_idx=None, threads=None):
    """The oracle's answer and checker flags for the rays in ray_idx (or all),
    for several compare_with_oracle calls on the same rays."""
    return oracle.raycast(verts, tris, poses, dirs, t_min, t_max, ray_idx=ray_idx,
                          threads=threads, checked=True)


def compare_with_oracle(verts, tris, poses, dirs, t_min, t_max, g_range, g_hit, ray_idx=None,
                        threads=None, min_checked_frac=0.97, oracle_out=None):
    """Check GPU results (for the rays in ray_idx, or all) against the oracle
    (computed here, or given as oracle_out from oracle_checked on the same
    rays).  Returns a dict of counts."""
    if oracle_out is None:
        oracle_out = oracle_checked(verts, tris, poses, dirs, t_min, t_max, ray_idx, threads)
    t, ids, flags, second, _ = oracle_out
    if ray_idx is not None:
        g_range = g_range[ray_idx]
        g_hit = g_hit[ray_idx]
    clean = flags == 0
    n = len(t)
    o_hit = ids >= 0
    g_is_hit = g_hit >= 0
    bad_hm = clean & (o_hit != g_is_hit)
    bad_id = clean & o_hit & (g_hit != ids)
    tol = TOL_ABS + TOL_REL * np.where(o_hit, t, 0.0)
    err = np.where(o_hit & g_is_hit, np.abs(g_range.astype(np.float64) - np.where(o_hit, t, 0.0)),
                   0.0)
    bad_rng = clean & o_hit & (g_hit == ids) & ~(err <= tol)
    stats = {"rays": n, "clean": int(clean.sum()), "edge_near": int((flags & 1).sum()),
             "ambiguous": int((flags & 2).sum()), "hits": int(o_hit.sum()),
             "bad_hitmiss": int(bad_hm.sum()), "bad_id": int(bad_id.sum()),
             "bad_range": int(bad_rng.sum()),
             "max_range_err": float(err[clean & o_hit].max()) if (clean & o_hit).any() else 0.0}
    if bad_hm.any() or bad_id.any() or bad_rng.any():
        k = np.flatnonzero(bad_hm | bad_id | bad_rng)[:10]
        detail = [(int(i), float(t[i]), int(ids[i]), float(g_range[i]), int(g_hit[i]))
                  for i in k]
        raise AssertionError(f"parity failure {stats}; first (ray, t, id, gpu_t, gpu_id): {detail}")
    assert clean.sum() >= min_checked_frac * n, stats
    check_flagged(verts, tris, poses, dirs, t_min, t_max, ray_idx, t, ids, flags, g_range, g_hit)
    stats["flagged_checked"] = int((~clean).sum())
    return stats


def _wide(x):
    return 1e-3 + 1e-5 * np.abs(x)


def check_flagged(verts, tris, poses, dirs, t_min, t_max, ray_idx, t, ids, flags, g_range,
                  g_hit):
    """Validity of the GPU answer on every ray the checker flags (see the
    module docstring).  Arrays are per checked ray; ray_idx maps them to
    flattened (env, beam) indices (None: identity)."""
    flagged = flags != 0
    o_hit = ids >= 0
    g_is_hit = g_hit >= 0
    # never beyond the nearest surface
    far = flagged & o_hit & g_is_hit & (g_range.astype(np.float64) > t + _wide(t))
    assert not far.any(), ("flagged ray beyond the nearest hit",
                           [(int(i), float(t[i]), float(g_range[i]), int(g_hit[i]))
                            for i in np.flatnonzero(far)[:10]])
    # a miss only where the oracle's hit is edge-near or at the range limits
    tol = TOL_ABS + TOL_REL * np.where(o_hit, np.abs(t), 0.0)
    # (a miss carries t = +inf, and t_max may be +inf: no inf - inf)
    t_fin = np.where(o_hit, t, 0.0)
    fin_max = np.isfinite(t_max)
    near_max = fin_max & (np.abs(t_fin - np.where(fin_max, t_max, 0.0)) <= tol)
    at_limit = o_hit & ((np.abs(t_fin - t_min) <= tol) | near_max)
    lost = flagged & o_hit & ~g_is_hit & ((flags & oracle.FLAG_EDGE_NEAR) == 0) & ~at_limit
    assert not lost.any(), ("flagged ray missed where the oracle hits",
                            [(int(i), float(t[i]), int(flags[i])) for i in np.flatnonzero(lost)[:10]])
    # every reported hit is a real hit near its range, inside the interval
    sel = np.flatnonzero(flagged & g_is_hit)
    if len(sel) == 0:
        return
    gr = g_range[sel].astype(np.float64)
    lim_lo = t_min - _wide(t_min)
    lim_hi = t_max + _wide(t_max) if np.isfinite(t_max) else np.inf
    assert np.all((gr >= lim_lo) & (gr <= lim_hi)), "flagged hit outside [t_min, t_max]"
    o, d = _rays_for(poses, dirs, ray_idx, sel)
    for r, i in enumerate(sel):
        tri = tris[g_hit[i]]
        tt = oracle.tri_test(o[r], d[r], verts[tri[0]], verts[tri[1]], verts[tri[2]])
        near = tt is not None and abs(tt - g_range[i]) <= _wide(tt)
        if not near:
            # an edge-near ray may have passed the neighbouring triangle in
            # FP64; its range must still agree with the oracle's
            assert (flags[i] & oracle.FLAG_EDGE_NEAR) and o_hit[i] and \
                abs(g_range[i] - t[i]) <= _wide(t[i]), (int(i), tt, float(g_range[i]), float(t[i]))


def _rays_for(poses, dirs, ray_idx, sel):
    nb = len(dirs)
    g = np.asarray(sel) if ray_idx is None else np.asarray(ray_idx)[sel]
    o, d = oracle.make_rays(poses, dirs) if len(poses) * nb <= 2_000_000 else (None, None)
    if o is not None:
        return o[g], d[g]
    oo, dd = [], []
    for gi in g:
        a, b = oracle.make_rays(poses[gi // nb][None], dirs[gi % nb][None])
        oo.append(a[0])
        dd.append(b[0])
    return np.array(oo), np.array(dd)
