"""Pins for the FP64 oracle, independent of the oracle's own formulas.

Each test checks the oracle against something the geometry or the
mathematics fixes: hand-derived values, closed forms (plane, box room,
sphere within tessellation error), exact rational arithmetic on random
triangle soups, watertightness of closed meshes and special cases.
The definition under test is FGGS-LiDAR Sec. IV-C (ray model and the
nearest-intersection equation).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
IDENT = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)


def pose_at(o, R=None):
    p = IDENT.copy()
    p[[3, 7, 11]] = o
    if R is not None:
        p[[0, 1, 2, 4, 5, 6, 8, 9, 10]] = np.asarray(R, np.float32).ravel()
    return p


def cast1(verts, tris, o, d, t_min=0.0, t_max=1e30):
    t, i = oracle.raycast(verts, tris, pose_at(o)[None], np.asarray(d, np.float32)[None],
                          t_min, t_max)
    return float(t[0]), int(i[0])


# --------------------------------------------------------------------------
def test_golden_box_room_axis_rays():
    v, t = synth.box_room()
    rows = np.loadtxt(os.path.join(GOLDEN, "box_room_axis_rays.txt"))
    for ox, oy, oz, dx, dy, dz, te, ie in rows:
        tt, ii = cast1(v, t, (ox, oy, oz), (dx, dy, dz))
        assert ii == int(ie)
        assert tt == te


def test_ray_generation_yaw_and_translation():
    # a yaw pose rotates every beam's azimuth by +yaw and keeps its elevation;
    # the origin is the translation column.  A transposed R would rotate by
    # -yaw, a wrong column would move the origin.
    dirs = synth.lidar_pattern(7, -30.0, 30.0, 36)
    el = np.radians(np.linspace(-30.0, 30.0, 7)).repeat(36)
    az = np.tile(np.arange(36) * 2 * np.pi / 36, 7)
    for yaw in (0.0, 0.7, -2.1):
        pos = (1.5, -2.25, 0.75)
        o, d = oracle.make_rays(synth.yaw_pose(pos, yaw)[None], dirs)
        exp = np.stack([np.cos(el) * np.cos(az + yaw), np.cos(el) * np.sin(az + yaw),
                        np.sin(el)], -1)
        assert np.abs(d - exp).max() < 1e-6
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
        assert np.all(o == np.float32(pos))


def test_ray_generation_pitch():
    # pitching the sensor by p about +y tilts a forward beam to elevation -p
    o, d = oracle.make_rays(synth.rpy_pose((0, 0, 0), 0.0, 0.3, 0.0)[None],
                            np.array([[1, 0, 0]], np.float32))
    assert np.allclose(d[0], [math.cos(0.3), 0.0, -math.sin(0.3)], atol=1e-7)


# --------------------------------------------------------------------------
def test_plane_closed_form():
    # 2 km quad at z=0; a downward beam of elevation el from height h hits at
    # range h / sin(-el), at horizontal bearing az + yaw.
    v, t = synth.plane_quad(1000.0, 0.0)
    dirs = synth.lidar_pattern(12, -60.0, -5.0, 90)
    el = np.radians(np.linspace(-60.0, -5.0, 12)).repeat(90)
    az = np.tile(np.arange(90) * 2 * np.pi / 90, 12)
    rng = np.random.default_rng(3)
    for _ in range(4):
        h = rng.uniform(0.5, 20.0)
        pos = (rng.uniform(-50, 50), rng.uniform(-50, 50), h)
        yaw = rng.uniform(0, 2 * np.pi)
        pose = synth.yaw_pose(pos, yaw)
        tt, ii, fl, _, _ = oracle.raycast(v, t, pose[None], dirs, 0.0, 1e4, checked=True)
        h32 = float(np.float32(h))
        exp_t = h32 / np.sin(-el)
        assert np.all(np.abs(tt - exp_t) <= 2e-6 * exp_t)
        px = np.float32(pos[0]) + exp_t * np.cos(el) * np.cos(az + yaw)
        py = np.float32(pos[1]) + exp_t * np.cos(el) * np.sin(az + yaw)
        exp_id = np.where(py < px, 0, 1)
        clear = np.abs(py - px) > 1e-3 * exp_t
        assert clear.sum() > 0.9 * len(clear)
        assert np.all(ii[clear] == exp_id[clear])
        assert np.all(fl[clear] & oracle.FLAG_EDGE_NEAR == 0)
    # upward beams miss
    up = synth.lidar_pattern(3, 5.0, 30.0, 16)
    tt, ii = oracle.raycast(v, t, synth.yaw_pose((0, 0, 2), 0.0)[None], up, 0.0, 1e4)
    assert np.all(ii == -1) and np.all(np.isinf(tt))


def _room_face_ids(o, d, lo, hi):
    """Closed form for the box room: exit distance and face/triangle id."""
    with np.errstate(divide="ignore"):
        t1 = (lo - o) / d
        t2 = (hi - o) / d
    tx = np.maximum(t1, t2)
    ax = np.argmin(tx, axis=1)
    t = tx[np.arange(len(o)), ax]
    side = (d[np.arange(len(o)), ax] > 0).astype(int)
    f = 2 * ax + side
    p = o + t[:, None] * d
    a, b = (ax + 1) % 3, (ax + 2) % 3
    n = np.arange(len(o))
    ua = (p[n, a] - lo[a]) / (hi[a] - lo[a])
    ub = (p[n, b] - lo[b]) / (hi[b] - lo[b])
    ids = np.where(ub <= ua, 2 * f, 2 * f + 1)
    margin = np.minimum.reduce([np.abs(ua - ub), ua, 1 - ua, ub, 1 - ub])
    return t, ids, margin


def test_box_room_closed_form():
    v, tr = synth.box_room()
    lo, hi = np.array(synth.ROOM_LO), np.array(synth.ROOM_HI)
    rng = np.random.default_rng(11)
    dirs = synth.lidar_pattern(24, -85.0, 85.0, 48)
    for k in range(5):
        pos = rng.uniform(lo + 0.2, hi - 0.2)
        pose = synth.rpy_pose(pos, *rng.uniform(-np.pi, np.pi, 3))
        tt, ii, fl, _, mina = oracle.raycast(v, tr, pose[None], dirs, 0.0, 100.0, checked=True)
        o, d = oracle.make_rays(pose[None], dirs)
        te, ie, margin = _room_face_ids(o, d, lo, hi)
        assert np.all(ii >= 0)                       # closed room: every ray hits
        assert np.all(np.abs(tt - te) <= 1e-12 * te)
        clear = margin > 1e-4
        assert np.all(ii[clear] == ie[clear])
        assert np.all(fl[clear] & oracle.FLAG_EDGE_NEAR == 0)


def test_sphere_within_tessellation():
    # vertices lie on the sphere, so the mesh lies between the sphere and the
    # concentric sphere through the nearest face plane (radius r_in): a ray
    # entering the inner ball hits the mesh between the two entry distances;
    # a ray missing the outer ball misses the mesh.
    c = np.array([0.3, -0.2, 0.1])
    r = 1.0
    v, t = synth.uv_sphere(c, r, 64, 32)
    assert len(t) == 3968
    P = v.astype(np.float64)[t]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    r_in = np.abs(np.einsum("ij,ij->i", n, P[:, 0] - c)).min()
    assert 0.99 < r_in < 1.0
    dirs = synth.lidar_pattern(40, -40.0, 40.0, 90)
    rng = np.random.default_rng(5)
    for _ in range(3):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pos = c + 3.0 * u
        yaw = math.atan2(-u[1], -u[0])
        pose = synth.yaw_pose(pos, yaw)
        tt, ii = oracle.raycast(v, t, pose[None], dirs, 0.0, 100.0)
        o, d = oracle.make_rays(pose[None], dirs)
        oc = c - o
        tca = np.einsum("ij,ij->i", oc, d)
        d2 = np.einsum("ij,ij->i", oc, oc) - tca ** 2
        slack = 1e-6
        inner = (d2 < (r_in - slack) ** 2) & (tca > 0)   # ray points at the ball
        outer_miss = d2 > (r + slack) ** 2
        assert inner.sum() > 100 and outer_miss.sum() > 100
        t_out = tca - np.sqrt(np.maximum((r + slack) ** 2 - d2, 0))
        t_in = tca - np.sqrt(np.maximum((r_in - slack) ** 2 - d2, 0))
        assert np.all(ii[inner] >= 0)
        assert np.all(tt[inner] >= t_out[inner]) and np.all(tt[inner] <= t_in[inner])
        assert np.all(ii[outer_miss] == -1)


# --------------------------------------------------------------------------
def test_inside_closed_room_sphere_all_hit():
    s = synth.room_sphere_scene(0)
    tt, ii = oracle.raycast(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max)
    assert np.all(ii >= 0)
    assert (ii >= 12).sum() > 0  # some beams see the sphere
    assert np.all(tt <= math.sqrt(10 ** 2 + 8 ** 2 + 3 ** 2))


def test_inside_closed_indoor_mesh_all_hit():
    # coarse marching-cubes mesh of the indoor field: closed, so every ray
    # cast from free space inside it hits
    sdf = synth.indoor_sdf(5, n_prims=30)
    v, t = synth.polygonise(sdf, 0.2)
    poses = synth.free_space_poses(sdf, 3, 9)
    dirs = synth.lidar_pattern(8, -60.0, 60.0, 64)
    tt, ii = oracle.raycast(v, t, poses, dirs, 0.0, 120.0)
    assert np.all(ii >= 0)


def test_watertight_through_vertices_and_edges():
    # rays aimed exactly at mesh vertices and shared edges never slip through
    v, t = synth.box_room()
    o = np.array([5.0, 4.0, 1.5])
    targets = [v[i].astype(np.float64) for i in range(8)]
    targets += [(v[a].astype(np.float64) + v[b]) / 2 for a, b, c in t]  # edge midpoints
    targets += [(v[a].astype(np.float64) + v[c]) / 2 for a, b, c in t]  # face diagonals
    dirs = np.array([(p - o) / np.linalg.norm(p - o) for p in targets], np.float32)
    tt, ii = oracle.raycast(v, t, pose_at(o)[None], dirs, 0.0, 100.0)
    assert np.all(ii >= 0)
    # from the centre of a UV sphere through every vertex (6 faces meet there)
    c = np.array([0.0, 0.0, 0.0])
    sv, st = synth.uv_sphere(c, 1.0, 64, 32)
    dirs = sv.astype(np.float64) - c
    dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    tt, ii = oracle.raycast(sv, st, pose_at(c)[None], dirs, 0.0, 10.0)
    assert np.all(ii >= 0)
    assert np.all(np.abs(tt - 1.0) < 1e-5)


# --------------------------------------------------------------------------
def _exact_cast(o, d, P, t_min, t_max):
    """Exact rational closest hit: same-sign test on triple products
    d . ((v_i - o) x (v_{i+1} - o)) and t from the plane equation."""
    o = [Fraction(float(x)) for x in o]
    d = [Fraction(float(x)) for x in d]

    def sub(a, b):
        return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]

    def cross(a, b):
        return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]

    def dot(a, b):
        return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]
    best, bid, min_margin = None, -1, float("inf")
    for k, tri in enumerate(P):
        V = [[Fraction(float(x)) for x in p] for p in tri]
        R = [sub(p, o) for p in V]
        s = [dot(d, cross(R[i], R[(i + 1) % 3])) for i in range(3)]
        if any(x < 0 for x in s) and any(x > 0 for x in s):
            continue
        n = cross(sub(V[1], V[0]), sub(V[2], V[0]))
        nd = dot(n, d)
        if nd == 0:
            continue
        tt = dot(n, sub(V[0], o)) / nd
        # angular margin of the ray to the triangle's edges
        for i in range(3):
            e = cross(R[i], R[(i + 1) % 3])
            en = math.sqrt(float(dot(e, e)))
            if en > 0:
                min_margin = min(min_margin, abs(float(s[i])) / en)
        if tt < t_min or tt > t_max:
            continue
        if best is None or tt < best:
            best, bid = tt, k
    return best, bid, min_margin


def test_exact_rational_random_soups():
    rng = np.random.default_rng(2024)
    for trial in range(6):
        n = [1, 3, 8, 16, 24, 32][trial]
        v, t = synth.random_soup(rng, n, 1.0)
        o = rng.uniform(-1.5, 1.5, size=3).astype(np.float32)
        dirs = rng.normal(size=(60, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        # aim half the rays at triangle interiors so hits are plentiful
        for j in range(30):
            k = rng.integers(n)
            w = rng.dirichlet([1, 1, 1])
            p = w @ v[t[k]].astype(np.float64)
            dirs[j] = (p - o) / np.linalg.norm(p - o)
        dirs = dirs.astype(np.float32)
        tt, ii = oracle.raycast(v, t, pose_at(o)[None], dirs, 0.0, 1e9)
        ro, rd = oracle.make_rays(pose_at(o)[None], dirs)
        P = v[t]
        checked = 0
        for j in range(len(dirs)):
            te, ie, margin = _exact_cast(ro[j], rd[j], P, 0.0, 1e9)
            if margin < 1e-9:
                continue  # ray grazes an edge: FP64 rounding may decide
            checked += 1
            assert ii[j] == ie, (trial, j)
            if ie >= 0:
                assert abs(tt[j] - float(te)) <= 1e-12 * max(1.0, float(te))
        assert checked >= 55


def test_special_cases():
    tri = np.array([[0, -1, -1], [0, 1, -1], [0, 0, 1]], np.float32)
    t0 = np.array([[0, 1, 2]], np.int32)
    o = (-5.0, 0.0, 0.0)
    # centroid hit at exact distance, and the back face is hit too (two-sided)
    c = tri.astype(np.float64).mean(0)
    d = (c - o) / np.linalg.norm(c - o)
    tt, ii = cast1(tri, t0, o, d)
    assert ii == 0 and abs(tt - np.linalg.norm(c - o)) < 1e-6
    tt, ii = cast1(tri, t0, (5.0, 0.0, 0.0), (-1, 0, 0))
    assert ii == 0 and tt == 5.0
    # behind the origin: miss
    assert cast1(tri, t0, o, (-1, 0, 0))[1] == -1
    # near miss just outside an edge (the bottom edge is at z=-1)
    assert cast1(tri, t0, (-5.0, 0.0, -1.001), (1, 0, 0))[1] == -1
    assert cast1(tri, t0, (-5.0, 0.0, -0.999), (1, 0, 0))[1] == 0
    # ray in the triangle's plane: det = 0, miss
    assert cast1(tri, t0, (0.0, -5.0, 0.0), (0, 1, 0))[1] == -1
    # degenerate (collinear) triangle is never hit
    deg = np.array([[0, -1, 0], [0, 0, 0], [0, 1, 0]], np.float32)
    assert cast1(deg, t0, (-5.0, 0.0, 0.0), (1, 0, 0))[1] == -1
    assert cast1(deg, t0, (-5.0, 0.0, 1e-3), (1, 0, -1e-4))[1] == -1
    # [t_min, t_max] is closed
    assert cast1(tri, t0, o, (1, 0, 0), 0.0, 5.0) == (5.0, 0)
    assert cast1(tri, t0, o, (1, 0, 0), 0.0, 4.999)[1] == -1
    assert cast1(tri, t0, o, (1, 0, 0), 5.0, 9.0) == (5.0, 0)
    assert cast1(tri, t0, o, (1, 0, 0), 5.001, 9.0)[1] == -1
    # exact tie: the lowest triangle id wins, whatever its position
    v = np.concatenate([tri, tri + np.float32([3, 0, 0]), tri])
    t3 = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)      # x=0, x=3, x=0
    assert cast1(v, t3, o, (1, 0, 0)) == (5.0, 0)
    t3b = np.array([[3, 4, 5], [6, 7, 8], [0, 1, 2]], np.int32)     # x=3, x=0, x=0
    assert cast1(v, t3b, o, (1, 0, 0)) == (5.0, 1)
    # nearest of several
    assert cast1(v, t3b, (10.0, 0, 0), (-1, 0, 0)) == (7.0, 0)


def test_tri_test_single():
    o = np.array([0.0, 0.0, 0.0])
    d = np.array([0.0, 0.0, 1.0])
    v0, v1, v2 = [1, -1, 2], [-1, -1, 2], [0, 1, 2]
    assert oracle.tri_test(o, d, v0, v1, v2) == 2.0
    assert oracle.tri_test(o, d, v0, v2, v1) == 2.0       # winding does not matter
    assert oracle.tri_test(o, -d, v0, v1, v2) == -2.0     # parameter is signed
    assert oracle.tri_test(o, d, [1, -1, 2], [2, -1, 2], [1.5, 1, 2]) is None


# --------------------------------------------------------------------------
def test_edge_angle_construction():
    # edge from a to b at distance 10 along +x; rotate the direction towards
    # the edge midpoint by theta out of the plane (o, a, b): angle = theta.
    o = np.zeros(3)
    a = np.array([10.0, -1.0, 0.0], np.float32)
    b = np.array([10.0, 1.0, 0.0], np.float32)
    for theta in (0.0, 3e-7, 1e-6, 2e-6, 1e-3):
        d = np.array([math.cos(theta), 0.0, math.sin(theta)])
        assert abs(oracle.edge_angle(o, d, a, b) - theta) < 1e-12
    # beyond endpoint b: angle to b
    d = np.array([10.0, 2.0, 0.0])
    d /= np.linalg.norm(d)
    bb = b.astype(np.float64) / np.linalg.norm(b.astype(np.float64))
    assert abs(oracle.edge_angle(o, d, a, b) - math.acos(np.dot(d, bb))) < 1e-9


def test_edge_near_flag():
    # a two-triangle quad split along the diagonal x=y: rays offset from the
    # diagonal by theta are edge-near iff theta <= 1e-6 rad
    v, t = synth.plane_quad(10.0, 0.0)
    o = np.array([0.0, 0.0, 5.0])
    p = np.array([2.0, 2.0, 0.0])
    base = (p - o) / np.linalg.norm(p - o)
    axis = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)   # perpendicular to the diagonal plane
    out = []
    for theta in (0.0, 4e-7, 3e-6, 1e-4):
        d = base * math.cos(theta) + axis * math.sin(theta)
        out.append(d)
    dirs = np.array(out, np.float32)
    tt, ii, fl, sec, mina = oracle.raycast(v, t, pose_at(o)[None], dirs, 0.0, 100.0,
                                           checked=True)
    assert list(fl & oracle.FLAG_EDGE_NEAR) == [1, 1, 0, 0]
    assert np.all(ii >= 0)


def test_ambiguous_flag():
    # two parallel squares 5e-5 m apart: the far one is within tol of the near
    # one, so the ray is ambiguous; at 1 m apart it is not
    v1, t1 = synth.plane_quad(5.0, 0.0)
    for gap, amb in ((5e-5, True), (1.0, False)):
        v2, t2 = synth.plane_quad(5.0, -gap)
        v, t = synth.concat_meshes((v1, t1), (v2, t2))
        d = np.array([[0.3, 0.1, -1.0]], np.float32)
        d /= np.linalg.norm(d)
        tt, ii, fl, sec, _ = oracle.raycast(v, t, pose_at((0.2, 0.7, 3.0))[None], d, 0.0, 100.0,
                                            checked=True)
        assert bool(fl[0] & oracle.FLAG_AMBIGUOUS) == amb
        assert ii[0] in (0, 1)
    # a hit within tol of t_max is ambiguous
    v, t = synth.plane_quad(5.0, 0.0)
    d = np.array([[0, 0, -1]], np.float32)
    _, ii, fl, _, _ = oracle.raycast(v, t, pose_at((0.1, 0.3, 3.0))[None], d, 0.0, 3.00005,
                                     checked=True)
    assert fl[0] & oracle.FLAG_AMBIGUOUS
    # an unbounded range (t_max = inf) has no upper end to be near: the same
    # hit is clean, at the same distance, as under a distant finite bound
    tt_inf, ii_inf, fl_inf, _, _ = oracle.raycast(v, t, pose_at((0.1, 0.3, 3.0))[None], d, 0.0,
                                                  np.inf, checked=True)
    tt_big, ii_big, fl_big, _, _ = oracle.raycast(v, t, pose_at((0.1, 0.3, 3.0))[None], d, 0.0,
                                                  1e9, checked=True)
    assert fl_inf[0] == fl_big[0] == 0
    assert ii_inf[0] == ii_big[0] >= 0 and abs(tt_inf[0] - 3.0) < 1e-12


def test_ray_index_sample_matches_full():
    s = synth.room_sphere_scene(1)
    t_all, i_all = oracle.raycast(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max)
    idx = np.random.default_rng(0).choice(s.n_rays, 300, replace=False)
    t_s, i_s = oracle.raycast(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, ray_idx=idx)
    assert np.array_equal(i_s, i_all[idx]) and np.array_equal(t_s, t_all[idx])


def test_thread_count_does_not_change_results():
    s = synth.room_sphere_scene(2)
    a = oracle.raycast(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, threads=1)
    b = oracle.raycast(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, threads=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_invalid_indices_rejected():
    v, t = synth.box_room()
    with pytest.raises(ValueError):
        oracle.raycast(v, t + 100, pose_at((1, 1, 1))[None], np.array([[1, 0, 0]], np.float32),
                       0.0, 10.0)


def test_non_unit_beam_vectors_are_normalised():
    # d_j is a unit direction (Sec. IV-C), so the range does not depend on the
    # length of the beam vector a caller passes
    v, t = synth.box_room()
    dirs = synth.lidar_pattern(5, -40.0, 40.0, 12)
    pose = synth.yaw_pose((3.0, 2.0, 1.0), 0.4)[None]
    t1, i1 = oracle.raycast(v, t, pose, dirs, 0.0, 100.0)
    t3, i3 = oracle.raycast(v, t, pose, dirs * np.float32(4.0), 0.0, 100.0)  # exact scaling
    assert np.array_equal(i1, i3)
    assert np.allclose(t1, t3, rtol=1e-12, atol=0)
