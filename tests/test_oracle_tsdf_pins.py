"""Pins of the TSDF / marching-cubes oracle (oracle/tsdf.py), FGGS-LiDAR
Sec. IV-B: closed forms, invariants, independent library routes and brute
force."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import tsdf as ot


def test_single_corner_cases_cut_the_corner_facing_away():
    tab = ot.table()
    assert tab[0] == [] and tab[255] == []
    for k in range(8):
        tris = tab[1 << k]
        assert len(tris) == 1
        edges = set(tris[0])
        at_k = {i for i, (a, b, _) in enumerate(ot.EDGES) if k in (a, b)}
        assert edges == at_k
        # orientation: normal points away from the inside corner
        pts = []
        for e in tris[0]:
            a, b, _ = ot.EDGES[e]
            pts.append((np.array(ot.CORNERS[a]) + np.array(ot.CORNERS[b])) / 2.0)
        n = np.cross(pts[1] - pts[0], pts[2] - pts[0])
        assert n @ (np.mean(pts, axis=0) - np.array(ot.CORNERS[k])) > 0


def test_every_case_uses_each_crossed_edge_once():
    for c in range(256):
        ins = [(c >> k) & 1 for k in range(8)]
        crossed = sorted(i for i, (a, b, _) in enumerate(ot.EDGES) if ins[a] != ins[b])
        used = sorted(e for loop in ot.case_loops(c) for e in loop)
        assert used == crossed
        assert len(ot.table()[c]) == sum(len(l) - 2 for l in ot.case_loops(c))


def test_fans_never_lie_on_a_cube_face():
    for c in range(256):
        for tri in ot.table()[c]:
            # at least one pair of the triangle's edges shares no face, so the
            # triangle is not contained in a face
            common = ot.EDGE_FACES[tri[0]] & ot.EDGE_FACES[tri[1]] & ot.EDGE_FACES[tri[2]]
            assert not common, (c, tri)


def _edges_of(tris):
    d = {}
    for t in tris:
        for i in range(3):
            a, b = int(t[i]), int(t[(i + 1) % 3])
            d[(a, b)] = d.get((a, b), 0) + 1
    return d


def _closed_and_oriented(tris):
    d = _edges_of(tris)
    return all(v == 1 for v in d.values()) and all(d.get((b, a), 0) == 1 for (a, b) in d)


def test_sphere_mesh_closed_form():
    """phi = |x - c| - R: vertices within h^2 / R of the sphere, closed and
    consistently oriented (every directed edge once, its reverse once),
    Euler characteristic 2, enclosed volume 4/3 pi R^3 within the
    discretisation error."""
    h, R = 0.1, 1.3
    n = 34
    o = (-1.7, -1.7, -1.7)
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = o[0] + (ix + 0.5) * h
    Y = o[1] + (iy + 0.5) * h
    Z = o[2] + (iz + 0.5) * h
    c = np.array([0.013, -0.021, 0.034])
    phi = (np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - R).astype(np.float32)
    v, t = ot.marching_cubes(phi, o, h, 0.0)
    d = np.linalg.norm(v.astype(np.float64) - c, axis=1)
    assert np.max(np.abs(d - R)) < h * h / R
    assert _closed_and_oriented(t)
    E = len(_edges_of(t)) // 2
    assert len(v) - E + len(t) == 2
    a, b, cc = (v[t[:, k]].astype(np.float64) for k in range(3))
    vol = np.sum(np.einsum("ij,ij->i", a, np.cross(b, cc))) / 6.0
    assert vol == pytest.approx(4.0 / 3.0 * math.pi * R ** 3, rel=0.02)


def test_random_fields_give_closed_oriented_meshes():
    rng = np.random.default_rng(3)
    for trial in range(20):
        phi = rng.normal(size=(9, 10, 11)).astype(np.float32)
        phi[0, :, :] = phi[-1, :, :] = 1.0        # outside on the grid boundary
        phi[:, 0, :] = phi[:, -1, :] = 1.0
        phi[:, :, 0] = phi[:, :, -1] = 1.0
        v, t = ot.marching_cubes(phi, (0, 0, 0), 1.0, 0.0)
        assert _closed_and_oriented(t), trial
        a, b, cc = (v[t[:, k]].astype(np.float64) for k in range(3))
        assert np.sum(np.einsum("ij,ij->i", a, np.cross(b, cc))) > 0


def test_vertex_positions_closed_form():
    """Two-point field: the vertex lies at the linear zero crossing."""
    phi = np.array([[[-1.0, 3.0]]], dtype=np.float32).reshape(1, 1, 2)
    phi = np.broadcast_to(phi, (2, 2, 2)).copy()
    v, t = ot.marching_cubes(phi, (0, 0, 0), 0.5, 0.0)
    assert len(t) == 2 and len(v) == 4
    np.testing.assert_array_equal(v[:, 0], np.float32(0.25 + 0.25 * 0.5))
    # a corner exactly at iso is outside (inside is phi < iso): the vertex
    # sits on that corner (t = 1)
    phi0 = np.broadcast_to(np.array([-1.0, 0.0], np.float32).reshape(1, 1, 2), (2, 2, 2)).copy()
    v0, t0 = ot.marching_cubes(phi0, (0, 0, 0), 0.5, 0.0)
    assert len(t0) == 2
    np.testing.assert_array_equal(v0[:, 0], np.float32(0.75))


def test_binomial_smoothing_closed_forms():
    n = ot.binomial_steps(0.02, 0.02)          # sigma = 1 voxel -> n = 2, [1 4 6 4 1]
    assert n == 2
    surf = np.zeros((9, 9, 9), np.uint8)
    surf[4, 4, 4] = 1
    vt, acc = ot.denoise(surf, 0.02, 0.02, 0.0001)
    w = np.array([1, 4, 6, 4, 1])
    want = np.zeros((9, 9, 9), np.int64)
    want[2:7, 2:7, 2:7] = w[:, None, None] * w[None, :, None] * w[None, None, :]
    np.testing.assert_array_equal(acc, want)
    full = np.ones((12, 12, 12), np.uint8)
    _, acc = ot.denoise(full, 0.02, 0.02, 0.5)
    assert acc[6, 6, 6] == 2 ** 12 and acc[0, 6, 6] == 2 ** 12 * 11 // 16


def test_binomial_smoothing_matches_a_3d_convolution():
    rng = np.random.default_rng(5)
    surf = (rng.random((13, 14, 15)) < 0.2).astype(np.uint8)
    n = ot.binomial_steps(0.03, 0.02)
    w = np.array([math.comb(2 * n, n + k) for k in range(-n, n + 1)], dtype=np.float64)
    k3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    ref = ndimage.convolve(surf.astype(np.float64), k3, mode="constant", cval=0.0)
    _, acc = ot.denoise(surf, 0.03, 0.02, 0.5)
    np.testing.assert_array_equal(acc.astype(np.float64), ref)


def test_threshold_is_inclusive_and_exact():
    surf = np.ones((5, 5, 5), np.uint8)
    vt, acc = ot.denoise(surf, 0.02, 0.02, 1.0)
    assert vt[2, 2, 2] == 1 and acc[2, 2, 2] == 2 ** 12
    assert vt.sum() == 1


def test_flood_fill_cavities_and_tunnels():
    vt = np.zeros((11, 11, 11), np.uint8)
    vt[2:9, 2:9, 2:9] = 1
    vt[3:8, 3:8, 3:8] = 0                      # closed cavity
    o = ot.outside(vt)
    assert o[0, 0, 0] and o[1, 5, 5] and not o[5, 5, 5]
    vt2 = vt.copy()
    vt2[5, 5, 2] = 0                           # a tunnel through one wall
    o2 = ot.outside(vt2)
    assert o2[5, 5, 5]
    # brute force: iterate a 6-neighbour propagation from the frame
    for grid, want in ((vt, o), (vt2, o2)):
        free = np.pad(grid == 0, 1, constant_values=True)
        lab = np.zeros_like(free)
        lab[0, :, :] = lab[-1, :, :] = lab[:, 0, :] = lab[:, -1, :] = lab[:, :, 0] = lab[:, :, -1] = True
        while True:
            p = np.pad(lab, 1)
            nb = (p[:-2, 1:-1, 1:-1] | p[2:, 1:-1, 1:-1] | p[1:-1, :-2, 1:-1] | p[1:-1, 2:, 1:-1]
                  | p[1:-1, 1:-1, :-2] | p[1:-1, 1:-1, 2:])
            new = lab | (nb & free)
            if np.array_equal(new, lab):
                break
            lab = new
        np.testing.assert_array_equal(lab[1:-1, 1:-1, 1:-1], want)


def test_shells_are_taxicab_distances_to_the_boundary_set():
    rng = np.random.default_rng(9)
    vt = (rng.random((12, 13, 14)) < 0.05).astype(np.uint8)
    s0 = ot.boundary_set(vt)
    p = ot.shells(s0, 40)
    ref = ndimage.distance_transform_cdt(~s0, metric="taxicab")
    np.testing.assert_array_equal(p, ref)


def test_half_space_tsdf_closed_form():
    """Occupied for x >= 10 (a wall), h = 0.1, r = 0.35: S_0 is the two
    layers x = 9, 10; |phi| = 0.1 * (distance to them), clipped at r; the
    free side is outside (+), the wall side inside (-).  The smallest
    kernel ([1 2 1] / 4 per axis) keeps the wall at tau = 0.4: a wall corner
    on the grid boundary gets (3/4)^3 = 0.42, the free layer next to it 1/4."""
    surf = np.zeros((6, 7, 20), np.uint8)
    surf[:, :, 10:] = 1
    phi, vt, sgn, p = ot.tsdf(surf, 0.1, 0.0001, 0.4, 0.35)
    assert np.array_equal(vt, surf)
    # S_0 also holds the wall's voxels on the grid boundary (the frame is
    # free): inside the wall p is the distance to its nearest face
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(20), indexing="ij")
    wall_d = np.minimum.reduce([x - 10, 19 - x, y, 6 - y, z, 5 - z])
    dist = np.where(x <= 9, 9 - x, wall_d)
    want = np.clip(np.where(x <= 9, 1, -1) * (dist.astype(np.float32) * np.float32(0.1)),
                   -np.float32(0.35), np.float32(0.35)).astype(np.float32)
    np.testing.assert_array_equal(phi, want)
    assert np.array_equal(sgn == 1, x <= 9)


def _crossed_edges_brute(phi, iso=0.0):
    """(lattice point (x, y, z), axis) of every crossed edge, in the vertex
    numbering order (point z-major, then axis), by plain loops."""
    nz, ny, nx = phi.shape
    out = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for a, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    X, Y, Z = x + dx, y + dy, z + dz
                    if X >= nx or Y >= ny or Z >= nz:
                        continue
                    if (phi[z, y, x] < iso) != (phi[Z, Y, X] < iso):
                        out.append(((x, y, z), (X, Y, Z)))
    return out


def test_normals_match_numpy_gradient_interpolated_along_the_edge():
    """Random smooth field (boundary vertices included): the normal is the
    FP64 interpolation of numpy's gradient (central inside, one-sided on the
    grid's faces) at the edge's two lattice points, normalised."""
    rng = np.random.default_rng(11)
    for trial in range(4):
        base = rng.normal(size=(7, 8, 9))
        phi = ndimage.uniform_filter(base, 3).astype(np.float32) * 3.0
        v, t, nrm = ot.marching_cubes(phi, (0.1, -0.2, 0.3), 0.25, 0.0, normals=True)
        p64 = phi.astype(np.float64)
        gz, gy, gx = np.gradient(p64)
        edges = _crossed_edges_brute(phi)
        assert len(edges) == len(v) > 50
        for k, ((x, y, z), (X, Y, Z)) in enumerate(edges):
            fa, fb = p64[z, y, x], p64[Z, Y, X]
            tt = (0.0 - fa) / (fb - fa)
            ga = np.array([gx[z, y, x], gy[z, y, x], gz[z, y, x]])
            gb = np.array([gx[Z, Y, X], gy[Z, Y, X], gz[Z, Y, X]])
            n = (1.0 - tt) * ga + tt * gb
            n /= np.linalg.norm(n)
            np.testing.assert_allclose(nrm[k], n, atol=2e-5, err_msg=f"{trial} {k}")


def test_normals_of_a_linear_field_are_its_direction():
    """phi = a . x + b: every normal equals a / |a| (central and one-sided
    differences of a linear field agree)."""
    n = (6, 7, 8)
    iz, iy, ix = np.meshgrid(*(np.arange(k) for k in n), indexing="ij")
    a = np.array([0.3, -0.5, 0.8])
    phi = (a[0] * ix + a[1] * iy + a[2] * iz - 4.1).astype(np.float32)
    v, t, nrm = ot.marching_cubes(phi, (0, 0, 0), 1.0, 0.0, normals=True)
    assert len(v) > 20
    np.testing.assert_allclose(nrm, np.broadcast_to(a / np.linalg.norm(a), nrm.shape), atol=2e-6)


def test_sphere_normals_are_radial_and_agree_with_the_winding():
    """phi = |x - c| - R: vertex normals within 1 degree of the radius, and
    every vertex normal on the outward side of its incident triangles."""
    h, R, n = 0.1, 1.3, 34
    o = (-1.7, -1.7, -1.7)
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = np.array([0.013, -0.021, 0.034])
    X, Y, Z = (o[k] + (g + 0.5) * h - c[k] for k, g in enumerate((ix, iy, iz)))
    phi = (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - R).astype(np.float32)
    v, t, nrm = ot.marching_cubes(phi, o, h, 0.0, normals=True)
    r = v.astype(np.float64) - c
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    assert np.min(np.sum(r * nrm, axis=1)) > math.cos(math.radians(1.0))
    np.testing.assert_allclose(np.linalg.norm(nrm.astype(np.float64), axis=1), 1.0, atol=1e-6)
    a, b, cc = (v[t[:, k]].astype(np.float64) for k in range(3))
    fn = np.cross(b - a, cc - a)
    for k in range(3):
        assert np.all(np.sum(fn * nrm[t[:, k]], axis=1) > 0)


def test_normals_on_an_axis_of_size_one_and_at_a_flat_point():
    """One z layer: no cells, the x/y vertices still get normals with z = 0.
    A vertex where the interpolated gradient vanishes gets (0, 0, 0)."""
    phi = np.array([[[-1.0, 1.0], [-1.0, 1.0]]], dtype=np.float32)
    v, t, nrm = ot.marching_cubes(phi, (0, 0, 0), 1.0, 0.0, normals=True)
    assert len(t) == 0 and len(v) == 2
    np.testing.assert_array_equal(nrm, np.array([[1, 0, 0], [1, 0, 0]], np.float32))
    # x profile -1, 1, -1: on the first edge the gradients are 2 (one-sided)
    # and 0 (central); on the second 0 and -2
    phi2 = np.array([[[-1.0, 1.0, -1.0]]], dtype=np.float32)
    v2, _, n2 = ot.marching_cubes(phi2, (0, 0, 0), 1.0, 0.0, normals=True)
    np.testing.assert_array_equal(n2, np.array([[1, 0, 0], [-1, 0, 0]], np.float32))
    phi4 = np.array([[[1.0, -1.0, 1.0, -1.0, 1.0]]], dtype=np.float32)
    v4, _, n4 = ot.marching_cubes(phi4, (0, 0, 0), 1.0, 0.0, normals=True)
    # interior central differences are 0: the edge (1, 2) has g = (0, 0)
    # at both ends
    assert len(v4) == 4
    np.testing.assert_array_equal(n4[1], np.zeros(3, np.float32))
    np.testing.assert_array_equal(n4[0], np.array([-1, 0, 0], np.float32))


# ---------------------------------------------------------------------------
# The FP64 definitions of vertex positions and normals (T5, T6) and their
# float32 error bounds, which are the GPU tolerance.

def test_fp64_vertices_of_a_linear_field_lie_on_its_zero_set():
    """phi = a . x + b sampled at the lattice centres (rounded to float32):
    every FP64 vertex lies on the plane a . x + b = 0 up to the float32
    rounding of the two phi values of its edge; normals are a / |a|."""
    n = (7, 8, 9)
    h, o = 0.0625, np.array([0.3125, -0.28125, 1.875])    # exact in float32
    iz, iy, ix = np.meshgrid(*(np.arange(k) for k in n), indexing="ij")
    a = np.array([0.3, -0.5, 0.8])
    X = [o[k] + (g + 0.5) * h for k, g in enumerate((ix, iy, iz))]
    b = 1.95
    f64 = a[0] * X[0] + a[1] * X[1] + a[2] * X[2] - b
    phi = f64.astype(np.float32)
    x, nrm, ptol, ntol = ot.marching_cubes_fp64(phi, o, h, 0.0)
    assert len(x) > 40
    resid = np.abs(x @ a - b)
    # each phi carries u |phi| of rounding, i.e. |phi| u / |a . e_axis| of
    # position along the edge; |phi| <= |a|_1 h on a crossed edge
    assert np.all(resid <= 2 * 2.0 ** -24 * np.abs(a).sum() * h + 1e-12)
    np.testing.assert_allclose(nrm, np.broadcast_to(a / np.linalg.norm(a), nrm.shape), atol=1e-6)


def test_fp64_matches_the_closed_form_two_point_field():
    phi = np.broadcast_to(np.array([-1.0, 3.0], np.float32).reshape(1, 1, 2), (2, 2, 2)).copy()
    x, nrm, _, _ = ot.marching_cubes_fp64(phi, (0, 0, 0), 0.5, 0.0)
    np.testing.assert_array_equal(x[:, 0], 0.25 + 0.25 * 0.5)
    np.testing.assert_array_equal(nrm, np.tile([1.0, 0.0, 0.0], (4, 1)))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_float32_evaluation_lies_within_the_fp64_bounds(seed):
    """The float32 evaluation (one rounded operation at a time) differs from
    the FP64 definition by less than the derived bounds, on rough and smooth
    fields away from the origin; the bounds are not vacuous."""
    rng = np.random.default_rng(seed)
    base = rng.normal(size=(10, 12, 14))
    phi = (ndimage.uniform_filter(base, 3) * 3.0 if seed else base).astype(np.float32)
    o, h, iso = (17.3, -41.9, 5.02), 0.037, 0.05 * seed
    v32, t32, n32 = ot.marching_cubes(phi, o, h, iso, normals=True)
    x, nrm, ptol, ntol = ot.marching_cubes_fp64(phi, o, h, iso)
    assert len(v32) == len(x) > 100
    r_pos = np.abs(v32.astype(np.float64) - x) / ptol
    r_nrm = np.abs(n32.astype(np.float64) - nrm).max(axis=1) / ntol
    assert r_pos.max() <= 1.0 and r_nrm.max() <= 1.0
    assert r_pos.max() > 0.02 and r_nrm.max() > 1e-3


def test_planted_mistakes_break_the_fp64_bounds():
    """t measured from the wrong end, or a normal that drops the far
    gradient, is caught by the bounds."""
    rng = np.random.default_rng(5)
    phi = (ndimage.uniform_filter(rng.normal(size=(9, 10, 11)), 3) * 3.0).astype(np.float32)
    o, h = (0.2, 0.4, -0.3), 0.05
    v32, _, n32 = ot.marching_cubes(phi, o, h, 0.0, normals=True)
    x, nrm, ptol, ntol = ot.marching_cubes_fp64(phi, o, h, 0.0)
    c = np.floor((x - np.asarray(o)) / h - 0.5 + 1e-9) * h + np.asarray(o) + 0.5 * h
    wrong = c + (h - (x - c))          # t -> 1 - t on the moving axis
    moving = np.abs(x - c) > 1e-12
    assert np.any(np.abs(np.where(moving, wrong, x) - x) > ptol)
    # a normal from the near gradient only
    G = ot.lattice_gradient(phi).reshape(-1, 3).astype(np.float64)
    edges = _crossed_edges_brute(phi)
    nz, ny, nx = phi.shape
    near = np.array([G[(z * ny + y) * nx + xx] for (xx, y, z), _ in edges])
    near /= np.maximum(np.linalg.norm(near, axis=1, keepdims=True), 1e-300)
    assert np.any(np.abs(near - nrm).max(axis=1) > ntol)


# ---- quantile re-threshold (reading T2) and mc_step (reading T2b) ---------

def _random_mask(seed, shape=(9, 11, 13), p=0.3):
    return (np.random.default_rng(seed).random(shape) < p).astype(np.uint8)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quantile_threshold_matches_numpy_quantile(seed):
    # n = 1 step: sums <= 64, exact in float64, so numpy's linearly
    # interpolated quantile decides the same voxels
    from oracle import tsdf as ot
    surf = _random_mask(seed)
    _, acc = ot.denoise(surf, 0.02, 0.04, 0.0)
    rng = np.random.default_rng(seed + 10)
    for q in [0.0, 1.0, 0.5, 0.25, 0.9] + list(rng.random(20)):
        q32 = float(np.float32(q))
        vt, _ = ot.denoise_quantile(surf, 0.02, 0.04, q32)
        want = acc >= np.quantile(acc.astype(np.float64), q32)
        assert np.array_equal(vt.astype(bool), want), q32


def test_quantile_extremes():
    from oracle import tsdf as ot
    surf = _random_mask(3)
    vt0, acc = ot.denoise_quantile(surf, 0.02, 0.04, 0.0)
    assert vt0.all()
    vt1, _ = ot.denoise_quantile(surf, 0.02, 0.04, 1.0)
    assert np.array_equal(vt1.astype(bool), acc == acc.max())


def test_planted_quantile_lower_statistic_is_caught(monkeypatch):
    # taking x_k even when the position lies between order statistics
    from oracle import tsdf as ot
    surf = _random_mask(4)
    _, acc = ot.denoise(surf, 0.02, 0.04, 0.0)

    def wrong(a, q):
        flat = np.sort(np.asarray(a, dtype=np.int64).ravel())
        return int(flat[int(math.floor(float(np.float32(q)) * (flat.size - 1)))])
    monkeypatch.setattr(ot, "quantile_threshold", wrong)
    # positions half-way between two distinct order statistics
    flat = np.sort(acc.ravel())
    ks = np.nonzero(flat[1:] != flat[:-1])[0][:10]
    assert len(ks) > 3
    bad = 0
    for k in ks:
        q = float(np.float32((k + 0.5) / (flat.size - 1)))
        vt, _ = ot.denoise_quantile(surf, 0.02, 0.04, q)
        bad += not np.array_equal(vt.astype(bool),
                                  acc >= np.quantile(acc.astype(np.float64), q))
    assert bad == len(ks)


def _sampled(f, origin, h, dims, stride=1):
    """f at the centres of voxels (i, j, k) * stride of a grid (origin, h)."""
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return f(origin[0] + (x * stride + 0.5) * h, origin[1] + (y * stride + 0.5) * h,
             origin[2] + (z * stride + 0.5) * h).astype(np.float32)


@pytest.mark.parametrize("step", [1, 2, 3])
def test_mc_step_equals_the_field_sampled_on_the_coarse_lattice(step):
    # an independent route: the analytic field evaluated directly at the
    # coarse lattice points (not sliced out of the fine one)
    from oracle import tsdf as ot
    h = float(np.float32(0.05))
    o = (0.1, -0.2, 0.05)
    f = lambda x, y, z: np.sqrt((x - 0.6) ** 2 + (y - 0.4) ** 2 + (z - 0.5) ** 2) - 0.33
    fine = _sampled(f, o, h, (25, 22, 23))
    v, t = ot.marching_cubes_step(fine, o, h, step)
    hs = float(np.float32(np.float32(h) * np.float32(step)))
    dims = tuple((n - 1) // step + 1 for n in (25, 22, 23))
    # f evaluated at the fine centres (i step, ...) directly, and the plain
    # extraction of those samples on a grid whose centres are those points
    direct = _sampled(f, o, h, dims, stride=step)
    assert np.array_equal(direct, np.ascontiguousarray(fine[::step, ::step, ::step]))
    o2 = tuple(c - (step - 1) * h / 2.0 for c in o)
    v2, t2 = ot.marching_cubes(direct, o2, hs, 0.0)
    assert np.array_equal(t, t2)
    assert np.allclose(v, v2, atol=2e-7 * (1 + np.abs(v).max()))
    # vertices of the coarse mesh lie on the sphere within its cell size
    r = np.linalg.norm(v.astype(np.float64) - (0.6, 0.4, 0.5), axis=1)
    assert np.all(np.abs(r - 0.33) < 0.25 * hs), float(np.abs(r - 0.33).max())
    if step == 1:
        v1, t1 = ot.marching_cubes(fine, o, h, 0.0)
        assert np.array_equal(t, t1) and np.array_equal(v, v1)


@pytest.mark.parametrize("step", [2, 3, 4])
def test_mc_step_plane_vertices_on_the_plane(step):
    from oracle import tsdf as ot
    h = 0.03125
    f = lambda x, y, z: x - 0.4 + 0 * y + 0 * z
    fine = _sampled(f, (0.0, 0.0, 0.0), h, (33, 9, 10))
    v, t = ot.marching_cubes_step(fine, (0.0, 0.0, 0.0), h, step)
    assert len(t) > 0
    assert np.all(np.abs(v[:, 0] - 0.4) < 1e-6)
    # the coarse lattice spans the fine centres 0.5 h .. (8 // step * step + 0.5) h in y
    assert np.isclose(v[:, 1].min(), 0.5 * h) and np.isclose(v[:, 1].max(), (8 // step * step + 0.5) * h)
