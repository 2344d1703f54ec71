"""Taubin smoothing on the GPU vs the oracle (oracle/mesh.py), FGGS-LiDAR
Sec. IV-B "Mesh optimization".  Parity bar: vertex positions within the
per-vertex float32 error bound of the FP64 definition (oracle taubin_fp64),
checked after 2 iterations, where the bound is tight, and after the
requested count; and, as a second check, bit-exact with the oracle's float32
evaluation in the kernel's operation order."""
import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from oracle import mesh as omesh
from oracle import tsdf as ot
from paper_2509_17390_amd import Context
from paper_2509_17390_amd import rcast

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def check(ctx, v, t, lam=0.5, mu=-0.53, it=10, tag=""):
    import torch
    for n_it in sorted({min(2, it), it}):
        vd = cuda(v)
        ctx.taubin(vd, cuda(t), lam, mu, n_it)
        torch.cuda.synchronize()
        got = vd.cpu().numpy()
        x64, bound = omesh.taubin_fp64(v, t, lam, mu, n_it)
        ratio = np.abs(got.astype(np.float64) - x64) / np.maximum(bound, 1e-300)
        assert np.all((ratio <= 1.0) | (got.astype(np.float64) == x64)), float(ratio.max())
        want = omesh.taubin(v, t, lam, mu, n_it)
        np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    log(f"{tag}: {len(v)} vertices, {len(t)} triangles, {it} iterations, within the FP64 "
        f"bound and bit-exact")
    return got


def test_noisy_sphere(ctx):
    v, t = synth.uv_sphere((0.1, -0.2, 0.3), 1.0, 24, 16)   # poles: 24 triangles
    rng = np.random.default_rng(1)
    v = (v * (1 + 0.01 * rng.normal(size=(len(v), 1)))).astype(np.float32)
    check(ctx, v, t, tag="sphere")


def test_open_patch_keeps_its_boundary(ctx):
    rng = np.random.default_rng(2)
    n = 30
    xs, ys = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="xy")
    v = np.stack([xs.ravel(), ys.ravel(), 0.2 * rng.normal(size=n * n)], axis=1).astype(np.float32)
    t = []
    for j in range(n - 1):
        for i in range(n - 1):
            a, b, c, d = j * n + i, j * n + i + 1, (j + 1) * n + i, (j + 1) * n + i + 1
            t += [[a, b, d], [a, d, c]]
    t = np.array(t, np.int32)
    out = check(ctx, v, t, it=7, tag="patch")
    _, _, bnd = omesh.neighbours(len(v), t)
    assert np.array_equal(out[bnd], v[bnd])


def test_marching_cubes_mesh(ctx):
    n, h = 40, 0.05
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X, Y, Z = ((ix + 0.5) * h - 1, (iy + 0.5) * h - 1, (iz + 0.5) * h - 1)
    phi = (np.maximum(np.abs(X), np.maximum(np.abs(Y), np.abs(Z))) - 0.6).astype(np.float32)
    v, t = ot.marching_cubes(phi, (-1, -1, -1), h, 0.0)
    check(ctx, v, t, it=5, tag="marching-cubes cube")


def test_degenerate_and_isolated(ctx):
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.5], [5, 5, 5]], np.float32)
    t = np.array([[0, 1, 2], [1, 3, 2], [1, 1, 3]], np.int32)   # one repeated index
    check(ctx, v, t, it=3, tag="degenerate")
    check(ctx, v, t, it=0, tag="zero iterations")


def test_errors(ctx):
    import torch
    v = torch.zeros((3, 3), dtype=torch.float32, device="cuda")
    bad = torch.tensor([[0, 1, 3]], dtype=torch.int32, device="cuda")
    with pytest.raises(rcast.RcastError) as e:
        ctx.taubin(v, bad)
    assert e.value.status == rcast.RC_E_INVAL
    # valence above the limit: a fan of 70 triangles around vertex 0
    k = 70
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False)
    vf = np.concatenate([[[0, 0, 0]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1)]).astype(np.float32)
    tf = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    with pytest.raises(rcast.RcastError) as e:
        ctx.taubin(cuda(vf), cuda(tf))
    assert e.value.status == rcast.RC_E_INVAL


# ---- quadric-error decimation --------------------------------------------------

def check_decimate(ctx, v, t, ratio, tag=""):
    import torch
    dv, dt, cell = ctx.decimate(cuda(v), cuda(t), ratio)
    torch.cuda.synchronize()
    dv, dt = dv.cpu().numpy(), dt.cpu().numpy()
    ov, otr, oc = omesh.decimate(v, t, ratio)
    assert np.float32(oc) == np.float32(cell), (oc, cell)
    np.testing.assert_array_equal(dt, otr)
    np.testing.assert_array_equal(dv.view(np.uint32), ov.view(np.uint32))
    log(f"{tag}: {len(t)} -> {len(dt)} triangles, cell {cell:.4g}, bit-exact")
    return dv, dt


def mc_sphere(n=50, h=0.06):
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X, Y, Z = ((ix + 0.5) * h - 1.5, (iy + 0.5) * h - 1.5, (iz + 0.5) * h - 1.5)
    phi = (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - 1.0).astype(np.float32)
    return ot.marching_cubes(phi, (-1.5, -1.5, -1.5), h, 0.0)


@pytest.mark.parametrize("ratio", [0.1, 0.3, 1.0])
def test_decimate_sphere(ctx, ratio):
    v, t = mc_sphere()
    check_decimate(ctx, v, t, ratio, tag=f"sphere ratio {ratio}")


def test_decimate_open_patch(ctx):
    import sys
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_mesh_pins import box_mesh, grid_patch
    v, t = grid_patch(25, jitter=0.05, seed=5)
    check_decimate(ctx, v, t, 0.2, tag="patch")
    v, t = box_mesh(16)
    check_decimate(ctx, v, t, 0.1, tag="box")


def test_decimate_then_smooth_a_tsdf_mesh(ctx):
    rng = np.random.default_rng(3)
    surf = (rng.random((30, 32, 34)) < 0.08).astype(np.uint8)
    phi, vt, sgn, p = ot.tsdf(surf, 0.05, 0.05, 0.2, 0.15)
    v, t = ot.marching_cubes(phi, (0, 0, 0), 0.05, 0.0)
    dv, dt = check_decimate(ctx, v, t, 0.1, tag="tsdf mesh")
    check(ctx, dv, dt, it=10, tag="tsdf mesh smoothed")


def test_decimate_errors(ctx):
    import torch
    v = torch.zeros((3, 3), dtype=torch.float32, device="cuda")
    t = torch.tensor([[0, 1, 5]], dtype=torch.int32, device="cuda")
    with pytest.raises(rcast.RcastError) as e:
        ctx.decimate(v, t, 0.1)
    assert e.value.status == rcast.RC_E_INVAL
    t = torch.tensor([[0, 1, 2]], dtype=torch.int32, device="cuda")
    with pytest.raises(rcast.RcastError) as e:
        ctx.decimate(v, t, 0.0)
    assert e.value.status == rcast.RC_E_INVAL


# ---- removal of tiny components: bit-exact (integer labels, copies) --------

def check_components(ctx, v, t, min_faces, tag=""):
    import torch
    gv, gt = ctx.remove_small_components(cuda(v), cuda(np.ascontiguousarray(t, np.int32)),
                                         min_faces)
    torch.cuda.synchronize()
    gv, gt = gv.cpu().numpy(), gt.cpu().numpy()
    ov, otr, _ = omesh.remove_small_components(v, t, min_faces)
    assert gv.shape == ov.shape and gt.shape == otr.shape, (gv.shape, ov.shape, gt.shape, otr.shape)
    np.testing.assert_array_equal(gt, otr)
    np.testing.assert_array_equal(gv.view(np.uint32), ov.view(np.uint32))
    log(f"{tag}: min {min_faces}: {len(t)} -> {len(gt)} triangles, {len(v)} -> {len(gv)} vertices")
    return gv, gt


@pytest.mark.parametrize("seed", range(3))
def test_components_of_random_soups(ctx, seed):
    """Sparse random soups (many components, repeated corners, chains that
    cross many launches' worth of vertices), several thresholds."""
    rng = np.random.default_rng(seed)
    nv = 20000 + 777 * seed
    nt = 9000
    t = rng.integers(0, nv, size=(nt, 3)).astype(np.int32)
    # long chains: triangle k shares a vertex with triangle k + 1
    chain = np.arange(3000)
    t[:3000, 0] = 2 * chain
    t[:3000, 1] = 2 * chain + 2
    v = rng.random((nv, 3)).astype(np.float32)
    for k in (0, 1, 2, 3, 4, 50, 3000, 100000):
        check_components(ctx, v, t, k, tag=f"soup {seed}")


def test_components_of_a_decimated_blob_field(ctx):
    """30 balls of radii 4 to 44 cm (a union of sphere distance fields),
    marching cubes, decimation to 30 %: 24 components of 4 to 742 faces."""
    rng = np.random.default_rng(4)
    n, h = 48, 0.05
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    P = np.stack([(ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h], -1)
    phi = np.full((n, n, n), 1.0)
    for _ in range(30):
        c = rng.random(3) * n * h
        r = 0.04 + 0.4 * rng.random() ** 3
        phi = np.minimum(phi, np.linalg.norm(P - c, axis=-1) - r)
    phi = phi.astype(np.float32)
    v, t = ot.marching_cubes(phi, (0, 0, 0), h, 0.0)
    dv, dt, _ = omesh.decimate(v, t, 0.3)
    assert len(dt) > 1000
    for k in (1, 8, 32, 100, 742, 743):
        check_components(ctx, dv, dt, k, tag="blobs decimated")
    check_components(ctx, v, t, 200, tag="blobs raw")


def test_components_edge_cases(ctx):
    import torch
    v = np.arange(18, dtype=np.float32).reshape(6, 3)
    check_components(ctx, v, np.array([[1, 3, 5]]), 0, tag="unreferenced vertices")
    check_components(ctx, v, np.array([[2, 2, 2]]), 1, tag="degenerate triangle")
    check_components(ctx, v, np.array([[0, 1, 2], [3, 4, 5]]), 2, tag="all removed")
    # no triangles, and no mesh at all
    gv, gt = ctx.remove_small_components(cuda(v), torch.zeros((0, 3), dtype=torch.int32,
                                                               device="cuda"), 1)
    assert gv.shape == (0, 3) and gt.shape == (0, 3)
    gv, gt = ctx.remove_small_components(torch.zeros((0, 3), device="cuda"),
                                         torch.zeros((0, 3), dtype=torch.int32, device="cuda"), 1)
    assert gv.shape == (0, 3) and gt.shape == (0, 3)
    with pytest.raises(rcast.RcastError) as e:
        ctx.remove_small_components(cuda(v), cuda(np.array([[0, 1, 6]], np.int32)), 1)
    assert e.value.status == rcast.RC_E_INVAL
    with pytest.raises(rcast.RcastError) as e:
        ctx.remove_small_components(cuda(v), cuda(np.array([[0, -1, 2]], np.int32)), 1)
    assert e.value.status == rcast.RC_E_INVAL


def test_decimate_high_valence_vertices(ctx):
    """Vertices with more than 8 triangles take the boundary test's long
    path: UV-sphere poles (24 triangles), the hub of an open fan (20) and
    of a closed fan (40); a closed fan of 70 exceeds the limit of 64."""
    import torch
    v, t = synth.uv_sphere((0.1, -0.2, 0.3), 1.0, 24, 16)
    check_decimate(ctx, v, t, 0.5, tag="uv sphere")
    k = 20
    ang = np.linspace(0, 1.5 * np.pi, k + 1)
    vf = np.concatenate([[[0, 0, 0.1]], np.stack([np.cos(ang), np.sin(ang), 0.05 * ang], 1)])
    vf = vf.astype(np.float32)
    tf = np.array([[0, 1 + i, 2 + i] for i in range(k)], np.int32)
    check_decimate(ctx, vf, tf, 0.5, tag="open fan")
    def closed_fan(k):
        ang = np.linspace(0, 2 * np.pi, k, endpoint=False)
        vf = np.concatenate([[[0, 0, 0]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1)])
        tf = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
        return vf.astype(np.float32), tf
    check_decimate(ctx, *closed_fan(40), 0.5, tag="closed fan")
    vf, tf = closed_fan(70)
    with pytest.raises(rcast.RcastError) as e:
        ctx.decimate(cuda(vf), cuda(tf), 0.5)
    assert e.value.status == rcast.RC_E_INVAL
