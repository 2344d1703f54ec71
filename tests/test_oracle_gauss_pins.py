"""Pins of the Gaussian-to-occupancy oracle (oracle/gauss.py) against closed
forms, invariants, an independent library route and brute force, so that a
dropped term, a wrong sign, index or transposition fails one of them.

The Gaussian model is FGGS-LiDAR Sec. III-A; the culling set, density,
threshold and surface mask are Sec. IV-A ("Grid query and occupancy
evaluation")."""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import gauss as og
import synth


def one(mu, quat, scale, alpha):
    return (np.array([mu], np.float32), np.array([quat], np.float32),
            np.array([scale], np.float32), np.array([alpha], np.float32))


def centres(grid):
    nx, ny, nz = grid.dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    o = grid.origin.astype(np.float64)
    h = float(grid.h)
    return (o[0] + (ix + 0.5) * h, o[1] + (iy + 0.5) * h, o[2] + (iz + 0.5) * h)


def test_isotropic_gaussian_closed_form():
    """Sigma = s^2 I for any rotation: D = alpha^2 exp(-|v - mu|^2 / (2 s^2))
    wherever the tile meets the box mu +- k s, else 0."""
    s, a, k = 0.3, 0.8, 3.0
    mu = (1.03, 0.97, 1.11)
    q = (0.3, -0.5, 0.7, 0.2)        # not normalised on purpose
    grid = og.Grid((0, 0, 0), 0.1, (24, 20, 22), tile=4)
    D, counts = og.density(one(mu, q, (s, s, s), a), grid, k)
    X, Y, Z = centres(grid)
    m = np.array(mu, np.float32).astype(np.float64)
    r2 = (X - m[0]) ** 2 + (Y - m[1]) ** 2 + (Z - m[2]) ** 2
    want = np.float64(np.float32(a)) ** 2 * np.exp(-r2 / (2 * np.float64(np.float32(s)) ** 2))
    # tiles meeting [mu - 0.9, mu + 0.9]: tile t spans [0.4 t, 0.4 (t + 1)]
    lo = np.floor((m - 3 * s) / 0.4).astype(int)
    hi = np.floor((m + 3 * s) / 0.4).astype(int)
    inside = np.zeros_like(D, dtype=bool)
    nx, ny, nz = grid.dims
    for kz in range(nz):
        for jy in range(ny):
            for ix in range(nx):
                t = (ix // 4, jy // 4, kz // 4)
                inside[kz, jy, ix] = all(lo[a_] <= t[a_] <= hi[a_] for a_ in range(3))
    np.testing.assert_allclose(D[inside], want[inside], rtol=1e-13, atol=0)
    assert np.all(D[~inside] == 0)
    assert counts.sum() == np.prod(hi - lo + 1)


def _axis_gaussian_case(axis, theta, scales):
    """Gaussian rotated by +theta about a coordinate axis (right-hand rule):
    closed-form quadratic form from the rotated principal axes."""
    c, s = math.cos(theta), math.sin(theta)
    half = theta / 2
    quat = [math.cos(half), 0.0, 0.0, 0.0]
    quat[1 + axis] = math.sin(half)
    E = np.eye(3)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]     # the plane the rotation turns
    e = E.copy()
    # principal axis i goes to c e_i + s e_j, axis j to -s e_i + c e_j
    e[i] = c * E[i] + s * E[j]
    e[j] = -s * E[i] + c * E[j]
    return quat, e


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rotated_anisotropic_closed_form(axis):
    theta = math.radians(30.0)
    scales = (0.5, 0.2, 0.1)
    quat, e = _axis_gaussian_case(axis, theta, scales)
    mu = (1.6, 1.5, 1.4)
    grid = og.Grid((0, 0, 0), 0.1, (32, 30, 28), tile=8)
    k = 10.0    # every tile in range: the plain closed form holds everywhere
    D, counts = og.density(one(mu, quat, scales, 1.0), grid, k)
    X, Y, Z = centres(grid)
    m = np.array(mu, np.float32).astype(np.float64)
    d = np.stack([X - m[0], Y - m[1], Z - m[2]], axis=-1)
    s32 = np.array(scales, np.float32).astype(np.float64)
    qf = sum((d @ e[b]) ** 2 / s32[b] ** 2 for b in range(3))
    # the quaternion is rounded to float32 before use: allow that rotation error
    np.testing.assert_allclose(D, np.exp(-0.5 * qf), rtol=2e-6, atol=1e-12)
    assert np.all(counts == 1)


def test_rotation_matches_independent_library():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(200, 4)).astype(np.float32)
    R = og.rotation_matrices(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-14)


def test_box_is_the_tight_box_of_the_k_sigma_ellipsoid():
    rng = np.random.default_rng(4)
    n = 50
    mu = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    s = np.exp(rng.uniform(np.log(0.01), np.log(0.5), (n, 3))).astype(np.float32)
    k = 3.0
    boxes = og.gauss_boxes(mu, q, s, k)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for i in range(n):
        pts = mu[i].astype(np.float64) + k * (dirs * s[i].astype(np.float64)) @ R[i].T
        lo, hi = boxes[i, :3].astype(np.float64), boxes[i, 3:].astype(np.float64)
        tol = 1e-6 * (1 + np.abs(mu[i]))
        assert np.all(pts >= lo - tol) and np.all(pts <= hi + tol)
        half = 0.5 * (hi - lo)
        reach = np.max(np.abs(pts - mu[i].astype(np.float64)), axis=0)
        np.testing.assert_allclose(reach, half, rtol=2e-3)


def test_box_closed_form_for_a_planar_rotation():
    theta = math.radians(40.0)
    a, b, c = 0.5, 0.25, 0.125
    quat = (math.cos(theta / 2), 0, 0, math.sin(theta / 2))
    box = og.gauss_boxes(np.zeros((1, 3), np.float32), np.array([quat], np.float32),
                         np.array([[a, b, c]], np.float32), 3.0)[0]
    ex = 3 * math.sqrt(a * a * math.cos(theta) ** 2 + b * b * math.sin(theta) ** 2)
    ey = 3 * math.sqrt(a * a * math.sin(theta) ** 2 + b * b * math.cos(theta) ** 2)
    np.testing.assert_allclose(box, [-ex, -ey, -3 * c, ex, ey, 3 * c], rtol=1e-6)


def test_integral_of_density_is_the_gaussian_mass():
    """sum_v D(v) h^3 -> alpha^2 (2 pi)^(3/2) s_x s_y s_z (midpoint rule on a
    smooth, untruncated Gaussian: exponentially small error)."""
    s = (0.3, 0.2, 0.25)
    quat = (0.9, 0.1, -0.3, 0.2)
    alpha = 0.7
    h = 0.05
    grid = og.Grid((-2.0, -2.0, -2.0), h, (80, 80, 80), tile=8)
    D, _ = og.density(one((0.013, -0.021, 0.007), quat, s, alpha), grid, 8.0)
    s32 = np.array(s, np.float32).astype(np.float64)
    a32 = float(np.float32(alpha))
    mass = a32 ** 2 * (2 * math.pi) ** 1.5 * np.prod(s32)
    h32 = float(grid.h)     # the grid spacing is a float32 value
    assert abs(D.sum() * h32 ** 3 - mass) < 1e-11 * mass


def test_membership_uses_closed_tile_boxes():
    """Box [2, 4] on x (s = 0.25, k = 4: e = 1 exactly) with 1-m tiles
    [t, t+1]: tiles 1..4 touch it; moving mu up by one float32 step drops
    tile 1 (its box ends at 2 < 2 + ulp)."""
    grid = og.Grid((0, 0, 0), 0.125, (64, 8, 8), tile=8)
    s = (0.25, 0.25, 0.25)
    mu = (3.0, 0.5, 0.5)
    b = og.gauss_boxes(*one(mu, (1, 0, 0, 0), s, 1.0)[:3], 4.0)
    assert b[0, 0] == 2.0 and b[0, 3] == 4.0
    _, counts = og.density(one(mu, (1, 0, 0, 0), s, 1.0), grid, 4.0)
    assert list(counts[0, 0]) == [0, 1, 1, 1, 1, 0, 0, 0]
    mu2 = (float(np.nextafter(np.float32(3.0), np.float32(4.0))), 0.5, 0.5)
    _, counts2 = og.density(one(mu2, (1, 0, 0, 0), s, 1.0), grid, 4.0)
    assert list(counts2[0, 0]) == [0, 0, 1, 1, 1, 0, 0, 0]


def test_culling_is_per_tile_not_per_voxel():
    """A Gaussian whose box only clips a tile's corner still contributes to
    the tile's far voxels, with the unclipped value of w."""
    grid = og.Grid((0, 0, 0), 0.125, (8, 8, 8), tile=8)   # one 1-m tile
    s = (0.1, 0.1, 0.1)
    mu = (1.2, 1.2, 1.2)                                   # box [0.9, 1.5]^3
    D, counts = og.density(one(mu, (1, 0, 0, 0), s, 1.0), grid, 3.0)
    assert counts.sum() == 1
    v = 0.0625                                             # centre of voxel 0
    m = np.float64(np.float32(1.2))
    want = math.exp(-0.5 * 3 * (m - v) ** 2 / np.float64(np.float32(0.1)) ** 2)
    assert want > 0 and D[0, 0, 0] == pytest.approx(want, rel=1e-12)


def test_threshold_is_strict():
    """alpha = 0.5 at a voxel centre: D = 0.25 exactly there; theta = 0.25."""
    grid = og.Grid((0, 0, 0), 0.5, (3, 3, 3), tile=8, theta=0.25)
    D, occ, surf, _ = og.voxelize(one((0.75, 0.75, 0.75), (1, 0, 0, 0),
                                      (0.01, 0.01, 0.01), 0.5), grid, 3.0)
    assert D[1, 1, 1] == 0.25
    assert occ.sum() == 0
    grid2 = og.Grid((0, 0, 0), 0.5, (3, 3, 3), tile=8, theta=0.2499)
    _, occ2, surf2, _ = og.voxelize(one((0.75, 0.75, 0.75), (1, 0, 0, 0),
                                        (0.01, 0.01, 0.01), 0.5), grid2, 3.0)
    assert occ2.sum() == 1 and occ2[1, 1, 1] == 1 and surf2[1, 1, 1] == 1


def test_surface_of_a_solid_cube_is_its_shell():
    occ = np.zeros((9, 9, 9), np.uint8)
    occ[2:7, 2:7, 2:7] = 1
    surf = og.surface(occ)
    assert surf.sum() == 5 ** 3 - 3 ** 3
    assert surf[4, 4, 4] == 0 and surf[2, 4, 4] == 1
    one_vox = np.zeros((3, 3, 3), np.uint8)
    one_vox[1, 1, 1] = 1
    assert og.surface(one_vox).sum() == 1


def test_surface_at_the_grid_boundary():
    """Reading G6: a fully occupied grid has only its boundary layer as
    surface."""
    occ = np.ones((5, 6, 7), np.uint8)
    surf = og.surface(occ)
    assert surf.sum() == 5 * 6 * 7 - 3 * 4 * 5
    assert surf[2, 3, 3] == 0 and surf[0, 3, 3] == 1 and surf[2, 3, 6] == 1


def test_surface_brute_force():
    rng = np.random.default_rng(7)
    occ = (rng.random((6, 7, 8)) < 0.7).astype(np.uint8)
    want = np.zeros_like(occ)
    nz, ny, nx = occ.shape
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if not occ[z, y, x]:
            continue
        full = True
        for dz, dy, dx in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            zz, yy, xx = z + dz, y + dy, x + dx
            if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx) or not occ[zz, yy, xx]:
                full = False
        want[z, y, x] = 0 if full else 1
    assert np.array_equal(og.surface(occ), want)


def test_density_brute_force_small():
    """Pure-Python loops over voxels and Gaussians, with Sigma^-1 from an
    independent route (scipy rotation, numpy inverse of R S S^T R^T) and the
    box test on the same float32 boxes."""
    rng = np.random.default_rng(11)
    n = 12
    mu = rng.uniform(0.2, 1.3, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    s = np.exp(rng.uniform(np.log(0.03), np.log(0.2), (n, 3))).astype(np.float32)
    al = rng.uniform(0.1, 1.0, n).astype(np.float32)
    grid = og.Grid((0.05, 0.0, 0.1), 0.1, (14, 13, 12), tile=4, theta=0.3)
    D, occ, surf, counts = og.voxelize((mu, q, s, al), grid, 3.0)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
    inv = [np.linalg.inv(R[i] @ np.diag(s[i].astype(np.float64) ** 2) @ R[i].T) for i in range(n)]
    boxes = og.gauss_boxes(mu, q, s, 3.0)
    nx, ny, nz = grid.dims
    o = grid.origin.astype(np.float64)
    h = float(grid.h)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        t = (x // 4, y // 4, z // 4)
        tb = grid.tile_box(t)
        v = np.array([o[0] + (x + 0.5) * h, o[1] + (y + 0.5) * h, o[2] + (z + 0.5) * h])
        acc = 0.0
        for i in range(n):
            if all(boxes[i, a] <= tb[3 + a] and boxes[i, 3 + a] >= tb[a] for a in range(3)):
                d = v - mu[i].astype(np.float64)
                acc += math.exp(-0.5 * float(d @ inv[i] @ d)) * float(al[i]) ** 2
        assert D[z, y, x] == pytest.approx(acc, rel=1e-10, abs=1e-300)
    assert occ.sum() > 0 and surf.sum() > 0


def test_density_at_matches_full_grid():
    rng = np.random.default_rng(12)
    n = 40
    params = (rng.uniform(0, 2, (n, 3)).astype(np.float32),
              rng.normal(size=(n, 4)).astype(np.float32),
              np.exp(rng.uniform(np.log(0.02), np.log(0.2), (n, 3))).astype(np.float32),
              rng.uniform(0.1, 1, n).astype(np.float32))
    grid = og.Grid((0, 0, 0), 0.1, (20, 19, 18), tile=8)
    D, counts, E = og.density(params, grid, 3.0, with_error=True)
    vox = np.stack([rng.integers(0, d, 300) for d in grid.dims], axis=1)
    Ds, Es, K = og.density_at(params, grid, vox, 3.0)
    np.testing.assert_array_equal(Ds, D[vox[:, 2], vox[:, 1], vox[:, 0]])
    np.testing.assert_array_equal(Es, E[vox[:, 2], vox[:, 1], vox[:, 0]])
    t = vox // 8
    np.testing.assert_array_equal(K, counts[t[:, 2], t[:, 1], t[:, 0]])
    assert np.all(E >= D)


# ---------------------------------------------------------------------------
# The error scale E(v) that sets the GPU density tolerance,
#   |D_fp32(v) - D(v)| <= 2^-24 (16 E(v) + 4 D(v)) + (K + 1) eps_abs,
# (eps_abs: the absolute granularity of the evaluation -- 2^-126 per term for
# float32 terms that underflow, 2^-31 for the GPU's fixed-point sum; K = the
# tile's culling-set size),
# pinned against an independent float32 evaluation of the density terms in
# tile-local coordinates (each tile's corner subtracted in FP64, then every
# operation in float32; the float32 terms summed exactly), on random cases
# that stress each part of E: ordinary, thin (the L / s part), and far-tail
# (a 6-sigma cutoff).  A planted mistake -- a dropped Gaussian, or E without
# its L / s part -- must break the bound.  (The constant and q parts are not
# separately necessary at these sizes: in a tail the q part and the L / s
# part are of the same size, since L >= |v - mu|, and the factor 16 covers
# the constant part's rounding of exp and alpha^2.)

def _density_f32(params, grid, k, drop_at=None):
    means, quats, scales, opac = params
    mu = np.asarray(means, np.float32).astype(np.float64)
    R32 = og.rotation_matrices(np.asarray(quats, np.float32)).astype(np.float32)
    s32 = np.asarray(scales, np.float32)
    al2 = np.asarray(opac, np.float32) * np.asarray(opac, np.float32)
    boxes = og.gauss_boxes(means, quats, scales, k)
    nx, ny, nz = grid.dims
    D = np.zeros((nz, ny, nx))
    h32 = np.float32(grid.h)
    tx, ty, tz = grid.tiles
    for kt in range(tz):
        for jt in range(ty):
            for it in range(tx):
                t = (it, jt, kt)
                mem = og.tile_members(boxes, grid.tile_box(t))
                if mem.size == 0:
                    continue
                (x0, x1), (y0, y1), (z0, z1) = grid.tile_voxels(t)
                corner = grid.origin.astype(np.float64) + np.array([x0, y0, z0]) * float(grid.h)
                iz, iy, ix = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1),
                                         indexing="ij")
                loc = np.stack([(ix - x0).ravel(), (iy - y0).ravel(), (iz - z0).ravel()], axis=1)
                v = (loc.astype(np.float32) + np.float32(0.5)) * h32          # [V, 3] f32
                m = (mu[mem] - corner).astype(np.float32)                    # [K, 3] f32
                d = v[:, None, :] - m[None, :, :]                           # f32
                Rk = R32[mem]
                u = (d[..., 0:1] * Rk[None, :, 0, :] + d[..., 1:2] * Rk[None, :, 1, :]) \
                    + d[..., 2:3] * Rk[None, :, 2, :]                       # (R^T d)_b, f32
                u = u / s32[mem][None]
                q = (u[..., 0] * u[..., 0] + u[..., 1] * u[..., 1]) + u[..., 2] * u[..., 2]
                terms = np.exp(np.float32(-0.5) * q) * al2[mem][None]       # f32
                assert terms.dtype == np.float32
                if drop_at is not None:
                    terms[:, np.argmax(terms.sum(axis=0))] = 0.0             # planted: one term lost
                D[z0:z1, y0:y1, x0:x1] = terms.astype(np.float64).sum(axis=1).reshape(iz.shape)
    return D


def _error_parts(params, grid, k):
    """E(v) split into its parts sum t, sum t q, sum t g (the oracle's own
    terms), for the planted checks."""
    means, quats, scales, opac = params
    mu = np.asarray(means, np.float32).astype(np.float64)
    sc = np.asarray(scales, np.float32).astype(np.float64)
    al = np.asarray(opac, np.float32).astype(np.float64)
    R = og.rotation_matrices(np.asarray(quats, np.float32))
    boxes = og.gauss_boxes(means, quats, scales, k)
    nx, ny, nz = grid.dims
    parts = np.zeros((3, nz, ny, nx))
    diag = math.sqrt(3.0) * grid.tile * float(grid.h)
    tx, ty, tz = grid.tiles
    for kt in range(tz):
        for jt in range(ty):
            for it in range(tx):
                t = (it, jt, kt)
                mem = og.tile_members(boxes, grid.tile_box(t))
                if mem.size == 0:
                    continue
                (x0, x1), (y0, y1), (z0, z1) = grid.tile_voxels(t)
                iz, iy, ix = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1),
                                         indexing="ij")
                pts = np.stack(grid.centres(ix.ravel(), iy.ravel(), iz.ravel()), axis=1)
                terms, u, q = og._terms(pts, mu[mem], R[mem], sc[mem], al[mem])
                L = diag + np.linalg.norm(pts[:, None, :] - mu[mem][None], axis=2)
                g = np.sum(np.abs(u) / sc[mem][None], axis=2) * L
                for j, part in enumerate((terms, terms * q, terms * g)):
                    parts[j, z0:z1, y0:y1, x0:x1] = part.sum(axis=1).reshape(iz.shape)
    return parts


CASES = {
    # name: (seed, n, scale range, cutoff, grid spacing)
    "ordinary": (31, 60, (0.02, 0.2), 3.0, 0.04),
    "thin": (32, 40, (0.0004, 0.004), 3.0, 0.05),
    "far_tail": (33, 30, (0.3, 0.6), 6.0, 0.01),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def f32_case(request):
    seed, n, (s_lo, s_hi), k, h = CASES[request.param]
    rng = np.random.default_rng(seed)
    params = synth.random_gaussians(rng, n, (0.2, 0.1, 0.3), (0.9, 0.8, 0.7), s_lo, s_hi)
    grid = og.Grid((0.13, 0.07, 0.21), h, (int(0.9 / h), int(0.8 / h), int(0.6 / h)), tile=8)
    D, _, E = og.density(params, grid, k, with_error=True)
    return request.param, params, grid, k, D, E


def test_error_scale_bounds_an_independent_float32_evaluation(f32_case):
    name, params, grid, k, D, E = f32_case
    D32 = _density_f32(params, grid, k)
    err = np.abs(D32 - D)
    bound = 2.0 ** -24 * (16 * E + 4 * D) + (_counts(params, grid, k) + 1) * 2.0 ** -126
    assert np.all(err <= bound), (name, float(np.max(err / np.maximum(bound, 1e-300))))
    assert (D > 0).mean() > 0.05           # the case has substance
    # the bound is not vacuous: the float32 error reaches a visible part of it
    assert float(np.max(err / np.maximum(bound, 1e-300))) > 0.01


def test_error_parts_sum_to_the_error_scale(f32_case):
    name, params, grid, k, D, E = f32_case
    parts = _error_parts(params, grid, k)
    np.testing.assert_allclose(parts.sum(axis=0), E, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(parts[0], D, rtol=1e-12, atol=1e-300)


def _counts(params, grid, k):
    """|C_tile| of every voxel's tile, [nz][ny][nx]."""
    boxes = og.gauss_boxes(params[0], params[1], params[2], k)
    c = og.tile_counts(boxes, grid)
    B = grid.tile
    nx, ny, nz = grid.dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return c[iz // B, iy // B, ix // B]


def test_planted_dropped_gaussian_breaks_the_bound(f32_case):
    name, params, grid, k, D, E = f32_case
    D32 = _density_f32(params, grid, k, drop_at=True)
    bound = 2.0 ** -24 * (16 * E + 4 * D) + (_counts(params, grid, k) + 1) * 2.0 ** -126
    assert np.any(np.abs(D32 - D) > bound)


@pytest.mark.parametrize("part,case", [(2, "thin")])
def test_planted_error_scale_without_a_part_breaks_the_bound(part, case):
    """Without its L / s part, the error scale no longer bounds the float32
    evaluation of thin Gaussians."""
    seed, n, (s_lo, s_hi), k, h = CASES[case]
    rng = np.random.default_rng(seed)
    params = synth.random_gaussians(rng, n, (0.2, 0.1, 0.3), (0.9, 0.8, 0.7), s_lo, s_hi)
    grid = og.Grid((0.13, 0.07, 0.21), h, (int(0.9 / h), int(0.8 / h), int(0.6 / h)), tile=8)
    D, _, E = og.density(params, grid, k, with_error=True)
    parts = _error_parts(params, grid, k)
    E_planted = E - parts[part]
    D32 = _density_f32(params, grid, k)
    slack = (_counts(params, grid, k) + 1) * 2.0 ** -126
    assert np.any(np.abs(D32 - D) > 2.0 ** -24 * (16 * E_planted + 4 * D) + slack)
