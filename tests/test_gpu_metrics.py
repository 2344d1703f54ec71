"""Exact nearest neighbours and the fidelity metrics on the GPU vs the oracle
(oracle/metrics.py): FGGS-LiDAR Sec. V, symmetric Chamfer distance and
F-score at a threshold.

Parity bar: nearest distances within 1e-12 relative (both sides FP64 from the
same float32 points; only the summation order of the three squares may
differ), the reported index a true nearest point (the lowest index on exact
ties, checked by brute force on small sets), CD within 1e-12 relative, and
precision / recall counts exact (no distance lies within 1e-12 of tau in
these inputs, which the test asserts).
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from oracle import metrics as om
from paper_2509_17390_amd import Context, Job
from paper_2509_17390_amd import rcast

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def gpu_nearest(ctx, ref, q):
    import torch
    d, i = ctx.nearest(cuda(ref), cuda(q))
    torch.cuda.synchronize()
    return d.cpu().numpy(), i.cpu().numpy()


@pytest.mark.parametrize("n_ref,n_q", [(1, 50), (2, 50), (3, 7), (1000, 3000), (20000, 5000)])
def test_nearest_matches_the_oracle(ctx, n_ref, n_q):
    rng = np.random.default_rng(n_ref + n_q)
    ref = rng.uniform(-2, 2, (n_ref, 3)).astype(np.float32)
    q = rng.uniform(-2.5, 2.5, (n_q, 3)).astype(np.float32)
    d, i = gpu_nearest(ctx, ref, q)
    do, _ = om.nearest(ref, q)
    np.testing.assert_allclose(d, do, rtol=1e-12, atol=0)
    di = np.linalg.norm(ref[i].astype(np.float64) - q.astype(np.float64), axis=1)
    np.testing.assert_allclose(di, do, rtol=1e-12, atol=0)


def test_ties_go_to_the_lowest_index(ctx):
    rng = np.random.default_rng(4)
    base = rng.uniform(0, 1, (300, 3)).astype(np.float32)
    ref = np.concatenate([base, base, base[::-1]])        # every point three times
    q = np.concatenate([base[:100], rng.uniform(0, 1, (200, 3)).astype(np.float32)])
    d, i = gpu_nearest(ctx, ref, q)
    for k in range(len(q)):
        dd = ((ref.astype(np.float64) - q[k].astype(np.float64)) ** 2).sum(axis=1)
        m = dd.min()
        assert i[k] == np.nonzero(dd == m)[0].min()


def test_empty_reference(ctx):
    d, i = gpu_nearest(ctx, np.zeros((0, 3), np.float32),
                       np.ones((5, 3), np.float32))
    assert np.all(np.isinf(d)) and np.all(i == -1)


def check_metrics(ctx, P, G, tau):
    got = ctx.chamfer_fscore(cuda(P), cuda(G), tau)
    cd, mpg, mgp, p, r, f = om.chamfer_fscore(P, G, tau)
    dpg, _ = om.nearest(G, P)
    dgp, _ = om.nearest(P, G)
    t = float(np.float32(tau))
    assert not np.any(np.abs(dpg - t) <= 1e-12 * t) and not np.any(np.abs(dgp - t) <= 1e-12 * t)
    assert got["chamfer"] == pytest.approx(cd, rel=1e-12)
    assert got["mean_pg"] == pytest.approx(mpg, rel=1e-12)
    assert got["mean_gp"] == pytest.approx(mgp, rel=1e-12)
    assert got["precision"] == p and got["recall"] == r
    assert got["fscore"] == pytest.approx(f, rel=1e-15)
    log(f"n_p {len(P)} n_g {len(G)}: CD {got['chamfer']:.6g} F {got['fscore']:.4f}")
    return got


def test_metrics_random_clouds(ctx):
    rng = np.random.default_rng(7)
    G = rng.uniform(0, 3, (30000, 3)).astype(np.float32)
    P = (G[:20000] + rng.normal(0, 0.02, (20000, 3))).astype(np.float32)
    check_metrics(ctx, P, G, 0.05)


def lidar(ctx, verts, tris, poses, dirs, n_az):
    import torch
    scene = ctx.upload_scene(verts, tris)
    ctx.build(scene)
    pat = ctx.upload_pattern(dirs, n_az)
    r, h = ctx.cast([Job(scene, pat, cuda(poses), 0.1, 120.0)])
    torch.cuda.synchronize()
    ctx.release_scene(scene)
    return om.lidar_points(poses, dirs, r.cpu().numpy(), h.cpu().numpy()).astype(np.float32)


def test_metrics_of_lidar_scans(ctx):
    """Scans of the room-with-sphere scene against scans of the same scene
    with the sphere moved by 1 cm: most points coincide, the sphere's differ."""
    s0 = synth.room_sphere_scene(0)
    v1 = s0.verts.copy()
    on_sphere = np.arange(len(v1)) >= 8                    # the room has 8 vertices
    v1[on_sphere] += np.float32(0.01)
    G = lidar(ctx, s0.verts, s0.tris, s0.poses, s0.dirs, s0.n_az)
    P = lidar(ctx, v1, s0.tris, s0.poses, s0.dirs, s0.n_az)
    got = check_metrics(ctx, P, G, 0.05)
    assert got["chamfer"] < 0.05


def test_metric_errors(ctx):
    import torch
    P = torch.zeros((3, 3), dtype=torch.float32, device="cuda")
    E = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(rcast.RcastError) as e:
        ctx.chamfer_fscore(P, E, 0.05)
    assert e.value.status == rcast.RC_E_INVAL
    with pytest.raises(rcast.RcastError) as e:
        ctx.chamfer_fscore(P, P, -1.0)
    assert e.value.status == rcast.RC_E_INVAL
