"""Pins of the fidelity-metric oracle (oracle/metrics.py): FGGS-LiDAR Sec. V,
symmetric Chamfer distance and F-score at a distance threshold."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import metrics as om


def grid_points(n=6, step=0.2):
    g = np.arange(n) * step
    return np.array(list(itertools.product(g, g, g)), dtype=np.float32)


def test_identical_clouds():
    P = grid_points()
    cd, mpg, mgp, p, r, f = om.chamfer_fscore(P, P, 0.05)
    assert cd == 0 and p == 1 and r == 1 and f == 1


def test_rigid_offset_closed_form():
    """Offset s below half the spacing: every nearest neighbour is the
    point's own copy, so every distance is |s|."""
    G = grid_points()
    s = np.array([0.03, -0.04, 0.0])                  # |s| = 0.05 (up to rounding)
    P = (G.astype(np.float64) + s).astype(np.float32)
    d = np.linalg.norm(P.astype(np.float64) - G.astype(np.float64), axis=1)
    cd, mpg, mgp, p, r, f = om.chamfer_fscore(P, G, 0.06)
    assert cd == pytest.approx(d.mean(), rel=1e-12)
    assert p == 1 and r == 1 and f == 1
    cd, mpg, mgp, p, r, f = om.chamfer_fscore(P, G, 0.04)
    assert p == 0 and r == 0 and f == 0


def test_threshold_is_inclusive():
    G = np.array([[0.0, 0.0, 0.0]], np.float32)
    P = np.array([[0.5, 0.0, 0.0], [0.0, 0.75, 0.0]], np.float32)
    _, _, _, p, r, f = om.chamfer_fscore(P, G, 0.5)
    assert p == 0.5 and r == 1.0 and f == pytest.approx(2 * 0.5 / 1.5)


def test_nearest_brute_force():
    rng = np.random.default_rng(1)
    ref = rng.uniform(-1, 1, (300, 3)).astype(np.float32)
    q = rng.uniform(-1.2, 1.2, (200, 3)).astype(np.float32)
    d, i = om.nearest(ref, q)
    for k in range(len(q)):
        best = min(math.dist(q[k].astype(float), r.astype(float)) for r in ref)
        assert d[k] == pytest.approx(best, rel=1e-12)
        assert math.dist(q[k].astype(float), ref[i[k]].astype(float)) == pytest.approx(best, rel=1e-12)


def test_subset_and_asymmetry():
    rng = np.random.default_rng(2)
    G = rng.uniform(0, 1, (400, 3)).astype(np.float32)
    P = G[:100]
    cd, mpg, mgp, p, r, f = om.chamfer_fscore(P, G, 0.05)
    assert mpg == 0 and p == 1
    dgp = np.array([min(np.linalg.norm(g.astype(float) - x.astype(float)) for x in P) for g in G])
    assert mgp == pytest.approx(dgp.mean(), rel=1e-12)
    assert r == pytest.approx(np.mean(dgp <= np.float32(0.05)))
    assert cd == pytest.approx(0.5 * mgp)


def test_lidar_points_lie_on_the_room_walls():
    """Rays from inside the empty box room: every point lies on a wall,
    ceiling or floor plane (closed form of a box room)."""
    verts, tris = synth.box_room()
    pose = synth.yaw_pose((3.0, 4.0, 1.5), 0.3)
    dirs = synth.lidar_pattern(8, -30.0, 30.0, 90)
    poses = pose[None]
    # exact first hits of the closed box along each ray (slab formula)
    R = pose.reshape(3, 4)[:, :3].astype(np.float64)
    o = pose.reshape(3, 4)[:, 3].astype(np.float64)
    d = dirs.astype(np.float64) @ R.T
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lo, hi = np.array(synth.ROOM_LO), np.array(synth.ROOM_HI)
    with np.errstate(divide="ignore"):
        t = np.min(np.maximum((lo - o) / d, (hi - o) / d), axis=1)
    pts = om.lidar_points(poses, dirs, t, np.zeros(len(dirs), np.int32))
    on = np.min(np.abs(np.concatenate([pts - lo, pts - hi], axis=1)), axis=1)
    assert np.all(on < 1e-9)
    assert len(pts) == len(dirs)
