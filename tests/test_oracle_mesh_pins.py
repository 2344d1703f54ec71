"""Pins of the mesh-optimisation oracle (oracle/mesh.py): Taubin smoothing of
FGGS-LiDAR Sec. IV-B ("Mesh optimization") with the defaults of Sec. V."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import mesh as omesh


def test_neighbours_of_small_meshes():
    tet = np.array([[0, 1, 2], [0, 3, 1], [1, 3, 2], [2, 3, 0]])
    nb, deg, bnd = omesh.neighbours(4, tet)
    assert list(deg) == [3, 3, 3, 3] and not bnd.any()
    assert list(nb[0]) == [1, 2, 3]
    nb, deg, bnd = omesh.neighbours(3, [[0, 1, 2]])
    assert bnd.all() and list(deg) == [2, 2, 2]
    nb, deg, bnd = omesh.neighbours(5, [[0, 1, 2], [2, 1, 3]])     # vertex 4 unused
    assert list(deg) == [2, 3, 3, 2, 0] and list(bnd) == [True, True, True, True, False]
    # a repeated index never makes a vertex its own neighbour
    nb, deg, bnd = omesh.neighbours(3, [[0, 0, 1], [0, 1, 2]])
    assert list(nb[0][:deg[0]]) == [1, 2] and deg[1] == 2


def grid_patch(n=9, jitter=0.0, seed=0):
    rng = np.random.default_rng(seed)
    xs, ys = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="xy")
    v = np.stack([xs.ravel(), ys.ravel(), np.zeros(n * n)], axis=1)
    v[:, 2] += jitter * rng.normal(size=n * n)
    t = []
    for j in range(n - 1):
        for i in range(n - 1):
            a, b, c, d = j * n + i, j * n + i + 1, (j + 1) * n + i, (j + 1) * n + i + 1
            t += [[a, b, d], [a, d, c]]
    return v.astype(np.float32), np.array(t, dtype=np.int32)


def test_boundary_stays_and_flat_patch_is_a_fixed_point_in_z():
    v, t = grid_patch(9, jitter=0.0)
    out = omesh.taubin(v, t, 0.5, -0.53, 5)
    _, _, bnd = omesh.neighbours(len(v), t)
    np.testing.assert_array_equal(out[bnd], v[bnd])
    assert np.all(out[:, 2] == 0)                 # a plane stays a plane


def test_noise_is_reduced_without_shrinking():
    """A noisy unit sphere: Taubin removes most of the radial noise and keeps
    the mean radius; plain Laplacian smoothing (mu = lambda) shrinks it."""
    v, t = synth.uv_sphere((0, 0, 0), 1.0, 48, 24)
    rng = np.random.default_rng(1)
    noisy = (v * (1 + 0.01 * rng.normal(size=(len(v), 1)))).astype(np.float32)
    r0 = np.linalg.norm(noisy.astype(np.float64), axis=1)
    out = omesh.taubin(noisy, t, 0.5, -0.53, 10)
    r1 = np.linalg.norm(out.astype(np.float64), axis=1)
    assert r1.std() < 0.5 * r0.std()
    assert abs(r1.mean() - r0.mean()) < 0.01
    lap = omesh.taubin(noisy, t, 0.5, 0.5, 10)
    assert np.linalg.norm(lap.astype(np.float64), axis=1).mean() < r1.mean() - 0.02


def test_matches_a_sparse_matrix_route():
    """The same steps as sparse matrices in FP64: x <- (I + f L) x with
    L = D^-1 A - I on moving rows and 0 on fixed rows; agreement to float32
    rounding."""
    v, t = grid_patch(12, jitter=0.3, seed=3)
    n = len(v)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    A = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    A.data[:] = 1.0                                   # distinct neighbours
    deg = np.asarray(A.sum(axis=1)).ravel()
    _, _, bnd = omesh.neighbours(n, t)
    move = ~bnd & (deg > 0)
    Dinv = sp.diags(np.where(move, 1.0 / np.maximum(deg, 1), 0.0))
    L = Dinv @ A - sp.diags(move.astype(float))
    x = v.astype(np.float64)
    for _ in range(4):
        for f in (0.5, -0.53):
            x = x + f * (L @ x)
    out = omesh.taubin(v, t, 0.5, -0.53, 4)
    np.testing.assert_allclose(out, x, rtol=0, atol=2e-5)


def test_fp64_definition_matches_the_sparse_matrix_route():
    """taubin_fp64 and the sparse-matrix form of the same steps, both FP64,
    agree to FP64 rounding."""
    v, t = grid_patch(12, jitter=0.3, seed=4)
    n = len(v)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    A = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    A.data[:] = 1.0
    deg = np.asarray(A.sum(axis=1)).ravel()
    _, _, bnd = omesh.neighbours(n, t)
    move = ~bnd & (deg > 0)
    L = sp.diags(np.where(move, 1.0 / np.maximum(deg, 1), 0.0)) @ A - sp.diags(move.astype(float))
    x = v.astype(np.float64)
    f_mu = float(np.float32(-0.53))
    for _ in range(5):
        for f in (0.5, f_mu):
            x = x + f * (L @ x)
    got, bound = omesh.taubin_fp64(v, t, 0.5, -0.53, 5)
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-12)
    assert np.all(bound[bnd] == 0) and np.all(bound[move] > 0)


@pytest.mark.parametrize("iterations", [1, 2, 10])
def test_float32_evaluation_within_the_fp64_bound(iterations):
    """The float32 evaluation stays inside the derived bound of the FP64
    definition on a noisy sphere away from the origin (high-valence poles
    included); at two iterations the bound is within 20x of the error."""
    v, t = synth.uv_sphere((3.0, -2.0, 1.0), 1.0, 48, 24)
    rng = np.random.default_rng(1)
    c = np.array([3.0, -2.0, 1.0])
    noisy = (c + (v - c) * (1 + 0.01 * rng.normal(size=(len(v), 1)))).astype(np.float32)
    o32 = omesh.taubin(noisy, t, 0.5, -0.53, iterations)
    x, bound = omesh.taubin_fp64(noisy, t, 0.5, -0.53, iterations)
    ratio = np.abs(o32 - x) / np.maximum(bound, 1e-300)
    assert ratio.max() <= 1.0
    if iterations <= 2:
        assert ratio.max() > 0.05


def test_planted_sign_error_breaks_the_fp64_bound():
    v, t = synth.uv_sphere((0.5, 0.2, -0.1), 1.0, 32, 16)
    rng = np.random.default_rng(2)
    noisy = (v * (1 + 0.01 * rng.normal(size=(len(v), 1)))).astype(np.float32)
    x, bound = omesh.taubin_fp64(noisy, t, 0.5, -0.53, 2)
    wrong = omesh.taubin(noisy, t, 0.5, 0.53, 2)           # mu with the wrong sign
    assert np.any(np.abs(wrong - x) > bound)


# ---- quadric-error decimation by vertex clustering ----------------------------

def box_mesh(n=12, size=(2.0, 1.5, 1.0)):
    """A closed box surface with sharp edges: each face an n x n grid of
    quads split in two, vertices shared along the edges."""
    index = {}
    verts = []

    def vid(p):
        key = tuple(round(x * 1e6) for x in p)
        if key not in index:
            index[key] = len(verts)
            verts.append(p)
        return index[key]

    tris = []
    for axis in range(3):
        u, w = (axis + 1) % 3, (axis + 2) % 3
        for side in (0, 1):
            g = [[None] * (n + 1) for _ in range(n + 1)]
            for i in range(n + 1):
                for j in range(n + 1):
                    p = [0.0, 0.0, 0.0]
                    p[axis] = side * size[axis]
                    p[u] = size[u] * i / n
                    p[w] = size[w] * j / n
                    g[i][j] = vid(tuple(p))
            for i in range(n):
                for j in range(n):
                    a_, b_, c_, d_ = g[i][j], g[i + 1][j], g[i + 1][j + 1], g[i][j + 1]
                    if side == 1:
                        tris += [[a_, b_, c_], [a_, c_, d_]]
                    else:
                        tris += [[a_, c_, b_], [a_, d_, c_]]
    return np.array(verts, np.float32), np.array(tris, np.int32)


def test_face_quadric_closed_form():
    v = np.array([[0, 0, 0.5], [2, 0, 0.5], [0, 3, 0.5]], np.float32)
    K = omesh.face_quadrics(v, [[0, 1, 2]])[0]
    # plane z = 0.5: p = (0, 0, 1, -0.5), area 3
    want = {(2, 2): 3.0, (2, 3): -1.5, (3, 3): 0.75}
    for k, ij in enumerate(omesh.UPPER):
        assert K[k] == pytest.approx(want.get(ij, 0.0), abs=1e-15)


def test_vertex_quadrics_brute_force():
    rng = np.random.default_rng(4)
    v = rng.uniform(0, 1, (30, 3)).astype(np.float32)
    t = rng.integers(0, 30, (60, 3))
    K = omesh.face_quadrics(v, t)
    Q = omesh.vertex_quadrics(30, t, K)
    for i in range(30):
        want = np.zeros(10)
        for j in range(len(t)):
            if i in set(t[j].tolist()):
                want = want + K[j]
        np.testing.assert_allclose(Q[i], want, rtol=1e-12, atol=1e-15)


def test_ratio_one_keeps_the_mesh():
    """Cells far smaller than the edges: every vertex is its own group and
    stays where it is (its quadric's minimiser or, on flat parts, its own
    position); only the numbering follows the cells."""
    v, t = box_mesh(8)
    dv, dt, c = omesh.decimate(v, t, 1.0)
    assert len(dt) == len(t) and len(dv) == len(v)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    np.testing.assert_allclose(key(dv.astype(np.float64)), key(v.astype(np.float64)), atol=1e-6)
    # the same triangles, renumbered
    tri_pts = lambda vv, tt: sorted(tuple(sorted(map(tuple, np.round(vv[x], 5).tolist()))) for x in tt)
    assert tri_pts(dv, dt) == tri_pts(v, t)


def test_box_corners_are_recovered_exactly():
    """Quadric minimisers of corner groups sit on the box corners (three
    planes meet there, the quadric has full rank); groups on one face or
    along an edge fall back to their mean, which stays inside the box and
    within a cell of its surface."""
    v, t = box_mesh(12)
    dv, dt, c = omesh.decimate(v, t, 0.1)
    assert len(dt) <= int(0.1 * len(t))
    lo, hi = v.min(axis=0).astype(np.float64), v.max(axis=0).astype(np.float64)
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])
    for cc in corners:
        assert np.min(np.linalg.norm(dv.astype(np.float64) - cc, axis=1)) < 1e-6
    d = dv.astype(np.float64)
    assert np.all(d >= lo - 1e-6) and np.all(d <= hi + 1e-6)
    off = np.min(np.abs(np.concatenate([d - lo, d - hi], axis=1)), axis=1)
    assert np.all(off <= c)


def test_boundary_vertices_are_protected():
    v, t = grid_patch(20, jitter=0.05, seed=5)
    dv, dt, c = omesh.decimate(v, t, 0.2)
    _, _, bnd = omesh.neighbours(len(v), t)
    kept = {tuple(p) for p in dv.tolist()}
    for p in v[bnd].tolist():
        assert tuple(p) in kept


def test_sphere_keeps_its_radius():
    from oracle import tsdf as ot
    n, h = 50, 0.06
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X, Y, Z = ((ix + 0.5) * h - 1.5, (iy + 0.5) * h - 1.5, (iz + 0.5) * h - 1.5)
    phi = (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - 1.0).astype(np.float32)
    v, t = ot.marching_cubes(phi, (-1.5, -1.5, -1.5), h, 0.0)
    dv, dt, c = omesh.decimate(v, t, 0.1)
    assert len(dt) <= int(0.1 * len(t)) and len(dt) > 0.05 * len(t)
    r = np.linalg.norm(dv.astype(np.float64), axis=1)
    assert np.all(np.abs(r - 1.0) < 0.01)


# ---- removal of tiny components (reading D5) -------------------------------

def _components_brute(nv, tris):
    """Triangle components by breadth-first search over 'shares a vertex',
    then each vertex's label = lowest vertex of its component (its own index
    when no triangle uses it)."""
    t = [tuple(int(x) for x in r) for r in np.asarray(tris).reshape(-1, 3)]
    by_vertex = {}
    for i, tri in enumerate(t):
        for v in tri:
            by_vertex.setdefault(v, []).append(i)
    comp = [-1] * len(t)
    labels = list(range(nv))
    for s in range(len(t)):
        if comp[s] >= 0:
            continue
        comp[s] = s
        queue, members = [s], [s]
        while queue:
            i = queue.pop()
            for v in t[i]:
                for j in by_vertex[v]:
                    if comp[j] < 0:
                        comp[j] = s
                        queue.append(j)
                        members.append(j)
        verts = {v for i in members for v in t[i]}
        low = min(verts)
        for v in verts:
            labels[v] = low
    sizes = {}
    for i in range(len(t)):
        sizes[comp[i]] = sizes.get(comp[i], 0) + 1
    return np.array(labels), [sizes[comp[i]] for i in range(len(t))]


@pytest.mark.parametrize("seed", range(6))
def test_components_match_breadth_first_search(seed):
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(5, 120))
    nt = int(rng.integers(1, 80))
    # sparse soups: many small components, some repeated corners
    tris = rng.integers(0, nv, size=(nt, 3))
    verts = rng.random((nv, 3)).astype(np.float32)
    labels, size_of = _components_brute(nv, tris)
    np.testing.assert_array_equal(omesh.component_labels(nv, tris), labels)
    for k in (0, 1, 2, 3, 5, 1000):
        keep = np.array(size_of) >= k
        used = np.zeros(nv, bool)
        used[tris[keep].ravel()] = True
        ids = np.cumsum(used) - 1
        v, t, _ = omesh.remove_small_components(verts, tris, k)
        np.testing.assert_array_equal(v, verts[used])
        np.testing.assert_array_equal(t, ids[tris[keep]])


def test_components_closed_form():
    """Two closed boxes (n = 3 and 2: 108 and 48 faces), a bow-tie (two
    triangles sharing one vertex: one component) and a lone triangle."""
    va, ta = box_mesh(3)
    vb, tb = box_mesh(2, (0.5, 0.5, 0.5))
    vb = vb + np.float32(5.0)
    tb = tb + len(va)
    o = len(va) + len(vb)
    vc = np.random.default_rng(0).random((8, 3)).astype(np.float32) + 9
    tc = np.array([[0, 1, 2], [2, 3, 4], [5, 6, 7]]) + o
    verts = np.concatenate([va, vb, vc])
    tris = np.concatenate([ta, tb, tc]).astype(np.int32)
    assert len(ta) == 108 and len(tb) == 48
    lab = omesh.component_labels(len(verts), tris)
    assert set(lab[:len(va)]) == {0} and set(lab[len(va):o]) == {len(va)}
    assert set(lab[o:o + 5]) == {o} and set(lab[o + 5:]) == {o + 5}
    for k, nt_kept, nv_kept in ((1, 159, len(verts)), (2, 158, len(verts) - 3),
                                (3, 156, len(va) + len(vb)), (48, 156, len(va) + len(vb)),
                                (49, 108, len(va)), (108, 108, len(va)), (109, 0, 0)):
        v, t, _ = omesh.remove_small_components(verts, tris, k)
        assert (len(t), len(v)) == (nt_kept, nv_kept), k
    # kept triangles in input order, renumbered onto the kept vertices
    v, t, _ = omesh.remove_small_components(verts, tris, 49)
    np.testing.assert_array_equal(t, ta)
    np.testing.assert_array_equal(v, va)


def test_components_drop_unreferenced_vertices_and_handle_empty_meshes():
    verts = np.arange(18, dtype=np.float32).reshape(6, 3)
    tris = np.array([[1, 3, 5]])
    v, t, lab = omesh.remove_small_components(verts, tris, 0)
    np.testing.assert_array_equal(v, verts[[1, 3, 5]])
    np.testing.assert_array_equal(t, [[0, 1, 2]])
    assert list(lab) == [0, 1, 2, 1, 4, 1]
    v, t, lab = omesh.remove_small_components(verts, np.zeros((0, 3), int), 1)
    assert v.shape == (0, 3) and t.shape == (0, 3) and list(lab) == list(range(6))
    v, t, lab = omesh.remove_small_components(np.zeros((0, 3)), np.zeros((0, 3), int), 1)
    assert v.shape == (0, 3) and t.shape == (0, 3) and len(lab) == 0
