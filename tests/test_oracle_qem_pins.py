"""Pins of the quadric-error decimation oracle (oracle/qem.py) against what
the mathematics fixes: the plane quadric is the squared distance to the
plane, the minimiser solves the linear system, ratio 1 changes nothing,
protected boundaries and box corners stay exact, flat meshes stay flat,
closed meshes stay closed with Euler characteristic 2, the face target is
met, and each step contracts an independent set that holds the cheapest
eligible edge.  Planted mistakes in the oracle break these pins."""
import math

import numpy as np
import pytest

import synth
from oracle import mesh as om
from oracle import qem


def edge_counts(t):
    c = {}
    for f in np.asarray(t):
        for i in range(3):
            a, b = int(f[i]), int(f[(i + 1) % 3])
            e = (min(a, b), max(a, b))
            c[e] = c.get(e, 0) + 1
    return c


def closed_manifold_euler(v, t):
    c = edge_counts(t)
    assert all(n == 2 for n in c.values()), "not closed"
    used = len(np.unique(np.asarray(t).ravel()))
    return used - len(c) + len(t)


def test_plane_quadric_is_squared_distance():
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b, c = (tuple(rng.normal(size=3)) for _ in range(3))
        K = qem.plane_quadric(a, b, c)
        x = tuple(rng.normal(size=3) * 3)
        n = np.cross(np.subtract(b, a), np.subtract(c, a))
        dist = np.dot(n / np.linalg.norm(n), np.subtract(x, a))
        assert math.isclose(qem.quadric_cost(K, x), dist * dist, rel_tol=1e-9, abs_tol=1e-12)
    assert qem.plane_quadric((0, 0, 0), (1, 1, 1), (2, 2, 2)) == [0.0] * 10


def minimiser_errors(fn):
    """Largest relative deviation of fn from numpy's solve on random
    well-conditioned systems."""
    rng = np.random.default_rng(1)
    worst = 0.0
    for _ in range(50):
        M = rng.normal(size=(3, 3))
        A = M @ M.T + np.eye(3)
        bvec = rng.normal(size=3)
        Q = [A[0, 0], A[0, 1], A[0, 2], -bvec[0], A[1, 1], A[1, 2], -bvec[1], A[2, 2], -bvec[2],
             1.0]
        x = np.array(fn(Q))
        ref = np.linalg.solve(A, bvec)
        worst = max(worst, float(np.max(np.abs(x - ref)) / (1e-12 + np.max(np.abs(ref)))))
    return worst


def test_minimiser_solves_the_system():
    assert minimiser_errors(qem.minimiser) < 1e-9
    # rank 2 (a crease): no minimiser, the fallback keeps an endpoint
    Q = [1.0, 0, 0, 0, 1.0, 0, 0, 0.0, 0, 0]
    assert qem.minimiser(Q) is None


def test_planted_transposed_cofactor_is_caught():
    orig = qem.minimiser

    def wrong(Q):
        Qn = list(Q)
        Qn[1], Qn[2] = Q[2], Q[1]          # a01 and a02 exchanged
        return orig(Qn)
    assert minimiser_errors(wrong) > 1e-3


def test_round_targets():
    assert qem.round_targets(1000, 0.1, 3) == [465, 216, 101]   # 1000 * 0.1^(k/3), ceil
    assert qem.round_targets(1000, 1.0, 3) == [1000, 1000, 1000]


def test_ratio_one_is_identity():
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 12, 6)
    ov, ot = qem.decimate_qem(v, t, 1.0, 3)
    assert np.array_equal(ov, v) and np.array_equal(ot, t)


def test_repeated_index_faces_dropped_first():
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 8, 4)
    bad = np.array([[0, 0, 1], [2, 3, 2]], np.int32)
    ov, ot = qem.decimate_qem(v, np.concatenate([t, bad]), 1.0, 3)
    assert np.array_equal(ov, v) and np.array_equal(ot, t)


def test_flat_patch_stays_flat_and_keeps_its_boundary():
    v, t = synth.grid_patch(12, 1.0, 0.25)
    ov, ot = qem.decimate_qem(v, t, 0.3, 3)
    assert np.all(ov[:, 2] == np.float32(0.25))
    g = v[:, :2]
    frame = np.any((g == 0.0) | (g == 1.0), axis=1)
    keep = {tuple(p) for p in ov.tolist()}
    assert all(tuple(p) in keep for p in v[frame].tolist()), "boundary vertex moved or removed"
    assert len(ot) < len(t)
    # still one flat sheet covering the square: the projected area is 1
    a, b, c = (ov[ot[:, k]].astype(np.float64) for k in range(3))
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) -
                        (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    assert math.isclose(area.sum(), 1.0, rel_tol=1e-9)


def test_box_keeps_corners_faces_and_closure():
    lo, hi = (0.0, 0.0, 0.0), (2.0, 1.5, 1.0)
    v, t = synth.grid_box(lo, hi, 6)
    ov, ot = qem.decimate_qem(v, t, 0.1, 3)
    T = qem.round_targets(len(t), 0.1, 3)[-1]
    assert len(ot) in (T - 1, T)
    corners = {(x, y, z) for x in (0.0, 2.0) for y in (0.0, 1.5) for z in (0.0, 1.0)}
    assert corners <= {tuple(p) for p in ov.astype(np.float64).tolist()}
    # every vertex on the box surface, none outside
    o = ov.astype(np.float64)
    on_face = np.any(np.isclose(o, lo, atol=1e-12) | np.isclose(o, hi, atol=1e-12), axis=1)
    assert on_face.all() and np.all(o >= lo) and np.all(o <= hi)
    assert closed_manifold_euler(ov, ot) == 2
    # the enclosed volume is the box's (no corner cut, no face bent)
    a, b, c = (o[ot[:, k]] for k in range(3))
    vol = np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0
    assert math.isclose(vol, 3.0, rel_tol=1e-9)


def test_sphere_closed_target_met_and_near_surface():
    v, t = synth.uv_sphere((0.5, -0.25, 1.0), 1.0, 24, 12)
    ov, ot = qem.decimate_qem(v, t, 0.2, 3)
    T = qem.round_targets(len(t), 0.2, 3)[-1]
    assert len(ot) in (T - 1, T)
    assert closed_manifold_euler(ov, ot) == 2
    r = np.linalg.norm(ov.astype(np.float64) - (0.5, -0.25, 1.0), axis=1)
    assert r.min() > 0.98 and r.max() < 1.06


def test_each_step_is_an_independent_set_with_the_cheapest_edge():
    rng = np.random.default_rng(3)
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 16, 8)
    v = (v + rng.normal(scale=0.01, size=v.shape)).astype(np.float32)
    m = qem._Mesh(v, t)
    vf, nb, ec = m.incidence()
    Q = qem._quadrics(m, vf)
    cands, vf, nb = qem.candidates(m, Q, set())
    need = 40
    chosen = qem.select(cands, nb, need)
    eligible = sorted(cands.items(), key=lambda kv: kv[1][0])[:need]
    assert (chosen[0][0], chosen[0][1]) == eligible[0][0]
    ends = [(u, v) for u, v, _, _ in chosen]
    for i, (a, b) in enumerate(ends):
        for (c, d) in ends[i + 1:]:
            for p in (a, b):
                for q in (c, d):
                    assert p != q and q not in nb[p], "chosen edges touch"


def outward(v, t, center):
    o = v.astype(np.float64)
    a, b, c = (o[t[:, k]] for k in range(3))
    n = np.cross(b - a, c - a)
    return np.einsum("ij,ij->i", n, (a + b + c) / 3.0 - center)


def test_convex_mesh_keeps_every_face_outward():
    rng = np.random.default_rng(4)
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 20, 10)
    v = (v * (1.0 + rng.uniform(-0.01, 0.01, size=(len(v), 1)))).astype(np.float32)
    ov, ot = qem.decimate_qem(v, t, 0.1, 3)
    assert np.all(outward(ov, ot, (0, 0, 0)) > 0)


def hexagon_fan():
    """Flat fan: centre vertex 0 and a regular hexagon 1..6 of unit radius,
    six counter-clockwise faces (normals +z)."""
    ang = np.arange(6) * (np.pi / 3.0)
    v = np.concatenate([[[0.0, 0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1)])
    t = np.array([[0, 1 + k, 1 + (k + 1) % 6] for k in range(6)], np.int32)
    return v.astype(np.float32), t


def flips_at(flips_fn, x):
    v, t = hexagon_fan()
    m = qem._Mesh(v, t)
    vf, _, _ = m.incidence()
    return flips_fn(m, vf, 0, 1, x)


def test_flip_test_on_a_convex_fan():
    # contracting centre 0 with rim vertex 1: the four faces that keep one of
    # them stay counter-clockwise exactly when x lies strictly inside the
    # hexagon's kernel (the hexagon itself, less the two rim edges at
    # vertex 1, which the contraction removes); on or beyond the opposite
    # rim a face degenerates or turns over
    inside = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (-0.3, 0.4, 0.0), (0.2, -0.6, 0.0)]
    for x in inside:
        assert not flips_at(qem._flips, x), x
    v, _ = hexagon_fan()
    rim = tuple(v[4].astype(np.float64))        # onto rim vertex 4: faces 3-4 and 4-5 degenerate
    outside = [rim, (-1.5, 0.0, 0.0), (0.0, 2.0, 0.0)]
    for x in outside:
        assert flips_at(qem._flips, x), x


def test_planted_non_strict_flip_bound_is_caught(monkeypatch):
    orig_dot = qem.dot3
    calls = {"n": 0}

    def loose(m, vf, u, v, x):
        for k in sorted(set(vf[u]) | set(vf[v])):
            f = m.f[k]
            if u in f and v in f:
                continue
            old = [m.p[i] for i in f]
            new = [x if i in (u, v) else m.p[i] for i in f]
            n0 = qem.face_normal(*old)
            if orig_dot(n0, n0) > 0.0 and orig_dot(n0, qem.face_normal(*new)) < 0.0:
                return True
        return False
    v, _ = hexagon_fan()
    rim = tuple(v[4].astype(np.float64))
    assert flips_at(qem._flips, rim) and not flips_at(loose, rim)
    assert calls["n"] == 0


def test_planted_missing_link_condition_breaks_closure(monkeypatch):
    # decimating a closed mesh as far as it goes (ratio 0) keeps it closed
    # with Euler characteristic 2; without the link condition it collapses
    # away entirely
    def no_link(m, Q, protected):
        vf, nb, ec = m.incidence()
        out = {}
        for (u, v), cnt in sorted(ec.items()):
            if cnt != 2 or u in protected or v in protected:
                continue
            Qe = [Q[u][i] + Q[v][i] for i in range(10)]
            x, cost = qem.placement(Qe, m.p[u], m.p[v])
            if qem._flips(m, vf, u, v, x):
                continue
            out[(u, v)] = ((cost, u, v), x, Qe)
        return out, vf, nb
    for v, t in (synth.uv_sphere((0, 0, 0), 1.0, 8, 4), synth.grid_box((0, 0, 0), (1, 1, 1), 3)):
        ov, ot = qem.decimate_qem(v, t, 0.0, 3)
        assert len(ot) >= 2 and closed_manifold_euler(ov, ot) == 2
    monkeypatch.setattr(qem, "candidates", no_link)
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 8, 4)
    ov, ot = qem.decimate_qem(v, t, 0.0, 3)
    assert len(ot) == 0 or closed_manifold_euler(ov, ot) != 2


def _inv_xorshift(x, s):
    y = x
    for _ in range(32 // s + 1):
        y = x ^ (y >> s)
    return y & qem.MASK32


def test_tie_hash_is_a_bijection():
    # undo each step (xorshifts by iteration, odd multipliers by their
    # inverses mod 2^32): every key is distinct, so ties cannot occur
    i1 = pow(0x846CA68B, -1, 1 << 32)
    i2 = pow(0x7FEB352D, -1, 1 << 32)

    def inv(x):
        x = _inv_xorshift(x, 16)
        x = (x * i1) & qem.MASK32
        x = _inv_xorshift(x, 15)
        x = (x * i2) & qem.MASK32
        return _inv_xorshift(x, 16)
    rng = np.random.default_rng(4)
    for e in list(range(2000)) + [int(x) for x in rng.integers(0, 1 << 32, 2000)]:
        assert inv(qem.perm32(e)) == e
    assert len({qem.perm32(e) for e in range(1 << 16)}) == 1 << 16


def test_hashed_ties_contract_many_edges_per_step():
    # a flat marching-cubes wall region: costs tie at zero, and the hashed
    # order lets each step contract a good fraction of the eligible edges
    v, t = synth.grid_patch(16, 1.0, 0.25)
    trace = []
    qem.decimate_qem(v, t, 0.1, 3, trace=trace)
    assert trace[0][2] >= 15, trace[:3]
    assert len(trace) < 60
