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
