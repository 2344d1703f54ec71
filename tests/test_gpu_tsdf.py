"""Denoising, flood-fill sign, narrow-band TSDF and marching cubes on the GPU
vs the oracle (oracle/tsdf.py), FGGS-LiDAR Sec. IV-B.

Parity bar.  V~ is decided on exact integer sums, the sign and shell
indices are integer and phi is one float32 product and a clip: bit-exact.
The mesh's topology (which edges carry vertices, the triangles, the
canonical numbering) comes from exact comparisons of the same float32 phi:
bit-exact.  Vertex positions and normals are compared with the FP64
definitions (oracle.tsdf.marching_cubes_fp64) within the derived float32
error bounds of each vertex; as a second check they also equal, bit for
bit, the oracle's float32 evaluation in the kernel's operation order
(t = (iso - phi_a) / (phi_b - phi_a), x = c_a + t h; w = 1 - t,
n = w g_a + t g_b, n / |n|).
"""
import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from oracle import gauss as og
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


def gpu_tsdf(ctx, surf, origin, h, sigma, tau, band):
    import torch
    nz, ny, nx = surf.shape
    g = ctx.grid(origin, h, (nx, ny, nz), 0.0)
    phi = torch.full((nz, ny, nx), 7.0, dtype=torch.float32, device="cuda")
    vt = torch.full((nz, ny, nx), 9, dtype=torch.uint8, device="cuda")
    ctx.tsdf(g, cuda(surf), phi, sigma, tau, band, out_vtilde=vt)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), vt.cpu().numpy(), g


def check_tsdf(ctx, surf, origin, h, sigma, tau, band, tag=""):
    phi_g, vt_g, g = gpu_tsdf(ctx, surf, origin, h, sigma, tau, band)
    phi, vt, sgn, p = ot.tsdf(surf, h, sigma, tau, band)
    np.testing.assert_array_equal(vt_g, vt)
    np.testing.assert_array_equal(phi_g.view(np.uint32), phi.view(np.uint32))
    log(f"{tag}: {surf.size} voxels, V~ {int(vt.sum())}, outside {int((sgn > 0).sum())}")
    return phi_g, g


def check_mc(ctx, phi, g, origin, h, iso, tag=""):
    """Mesh without normals, then with them: topology exact, positions and
    normals within the FP64 definitions' bounds, and equal to the float32
    evaluation bit for bit."""
    import torch
    vo, to, no = ot.marching_cubes(phi, origin, h, iso, normals=True)
    x64, n64, ptol, ntol = ot.marching_cubes_fp64(phi, origin, h, iso)
    for with_n in (False, True):
        out = ctx.marching_cubes(g, cuda(phi), iso, normals=with_n)
        torch.cuda.synchronize()
        v, t = out[0].cpu().numpy(), out[1].cpu().numpy()
        assert v.shape == vo.shape and t.shape == to.shape, (v.shape, vo.shape, t.shape, to.shape)
        np.testing.assert_array_equal(t, to)
        r_pos = np.abs(v.astype(np.float64) - x64) / ptol
        assert np.all(r_pos <= 1.0), float(r_pos.max())
        np.testing.assert_array_equal(v.view(np.uint32), vo.view(np.uint32))
        if with_n:
            n = out[2].cpu().numpy()
            r_n = np.abs(n.astype(np.float64) - n64).max(axis=1) / ntol
            assert np.all(r_n <= 1.0), float(r_n.max())
            np.testing.assert_array_equal(n.view(np.uint32), no.view(np.uint32))
    log(f"{tag}: {len(v)} vertices, {len(t)} triangles, positions and normals within bounds")
    return v, t


@pytest.mark.parametrize("seed", [0, 1])
def test_random_masks(ctx, seed):
    rng = np.random.default_rng(seed)
    surf = (rng.random((19, 23, 29)) < 0.15).astype(np.uint8)
    # smoothing of n = 2, 6, 1 and 3 steps (the tiled pass takes 1..3)
    for sigma, tau, band in ((0.02, 0.05, 0.06), (0.035, 0.2, 0.1), (0.01, 0.5, 0.02),
                             (0.025, 0.15, 0.08)):
        phi, g = check_tsdf(ctx, surf, (0.1, -0.2, 0.3), 0.02, sigma, tau, band,
                            tag=f"random {seed} sigma {sigma}")
        check_mc(ctx, phi, g, (0.1, -0.2, 0.3), 0.02, 0.0, tag=f"random {seed} mc")


def test_cavity_and_tunnel(ctx):
    surf = np.zeros((20, 21, 22), np.uint8)
    surf[3:17, 3:18, 3:19] = 1
    surf[4:16, 4:17, 4:18] = 0                        # closed shell
    phi, g = check_tsdf(ctx, surf, (0, 0, 0), 0.05, 0.001, 0.4, 0.2, tag="shell")
    assert phi[10, 10, 10] < 0                        # the cavity is not outside
    surf[10, 10, 3] = 0                               # a tunnel
    phi2, _ = check_tsdf(ctx, surf, (0, 0, 0), 0.05, 0.001, 0.4, 0.2, tag="tunnel")
    assert phi2[10, 10, 10] > 0


def test_gaussian_surface_to_mesh(ctx):
    """Surface mask from the Gaussian conversion of a region of the indoor
    scene, then TSDF and marching cubes."""
    import torch
    m, q, s, a, room = synth.splat_scene(1, 200000)
    lo = np.array([-0.1, 2.0, 0.9])
    grid = og.Grid(lo, 0.02, (44, 40, 36), tile=8, theta=0.2)
    hi = lo + 0.02 * np.array(grid.dims)
    boxes = og.gauss_boxes(m, q, s, 3.0)
    sel = np.all((boxes[:, :3] <= hi + 0.3) & (boxes[:, 3:] >= lo - 0.3), axis=1)
    gset = ctx.upload_gaussians(m[sel], q[sel], s[sel], a[sel])
    ctx.build_gaussians(gset)
    nx, ny, nz = grid.dims
    O = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    S = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    ctx.voxelize(gset, ctx.grid(lo, 0.02, grid.dims, 0.2), None, O, S)
    torch.cuda.synchronize()
    surf = S.cpu().numpy()
    ctx.release_gaussians(gset)
    phi, g = check_tsdf(ctx, surf, lo, 0.02, 0.02, 0.15, 0.06, tag="splat")
    v, t = check_mc(ctx, phi, g, lo, 0.02, 0.0, tag="splat mc")
    assert len(t) > 1000


def test_sphere_field_and_exact_iso(ctx):
    n = 31
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    h = 0.1
    X, Y, Z = (-1.5 + (ix + 0.5) * h, -1.5 + (iy + 0.5) * h, -1.5 + (iz + 0.5) * h)
    phi = (np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - 1.1).astype(np.float32)
    import torch
    g = ctx.grid((-1.5, -1.5, -1.5), h, (n, n, n), 0.0)
    for iso in (0.0, 0.05, -0.2):
        check_mc(ctx, phi, g, (-1.5, -1.5, -1.5), h, iso, tag=f"sphere iso {iso}")
    q = np.round(phi * 10).astype(np.float32) / 10   # many corners exactly at iso
    check_mc(ctx, q, g, (-1.5, -1.5, -1.5), h, 0.0, tag="sphere quantised")


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (1, 5, 7), (9, 1, 4)])
def test_tiny_grids(ctx, dims):
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    surf = (rng.random((nz, ny, nx)) < 0.5).astype(np.uint8)
    phi, g = check_tsdf(ctx, surf, (0, 0, 0), 0.1, 0.1, 0.3, 0.3, tag=f"tiny {dims}")
    check_mc(ctx, phi, g, (0, 0, 0), 0.1, 0.0, tag=f"tiny {dims} mc")


def test_constant_fields_have_no_mesh(ctx):
    import torch
    g = ctx.grid((0, 0, 0), 0.1, (10, 11, 12), 0.0)
    for val in (-1.0, 1.0, 0.0):
        phi = torch.full((12, 11, 10), val, dtype=torch.float32, device="cuda")
        v, t = ctx.marching_cubes(g, phi, 0.0)
        assert v.shape[0] == 0 and t.shape[0] == 0


def test_errors(ctx):
    import torch
    g = ctx.grid((0, 0, 0), 0.01, (8, 8, 8), 0.0)
    surf = torch.zeros((8, 8, 8), dtype=torch.uint8, device="cuda")
    phi = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    for sigma, tau, band in ((0.1, 0.5, 0.02), (0.01, 0.5, 3.0), (0.0, 0.5, 0.02),
                             (0.01, float("nan"), 0.02), (0.01, 0.5, -1.0)):
        with pytest.raises(rcast.RcastError) as e:
            ctx.tsdf(g, surf, phi, sigma, tau, band)
        assert e.value.status == rcast.RC_E_INVAL
    # capacity too small: sizes are still reported
    field = torch.ones((8, 8, 8), dtype=torch.float32, device="cuda")
    field[3:5, 3:5, 3:5] = -1.0
    import ctypes
    lib = rcast.load()
    nv, nt = ctypes.c_int64(), ctypes.c_int64()
    V = torch.empty((1, 3), dtype=torch.float32, device="cuda")
    T = torch.empty((1, 3), dtype=torch.int32, device="cuda")
    st = lib.rc_marching_cubes(ctx._h, ctypes.byref(g), field.data_ptr(), 0.0, V.data_ptr(),
                               T.data_ptr(), None, 1, 1, ctypes.byref(nv), ctypes.byref(nt),
                               torch.cuda.current_stream().cuda_stream)
    assert st == rcast.RC_E_NOMEM and nv.value > 1 and nt.value > 1
    st = lib.rc_marching_cubes(ctx._h, ctypes.byref(g), field.data_ptr(), 0.0, V.data_ptr(),
                               None, None, 1, 1, ctypes.byref(nv), ctypes.byref(nt),
                               torch.cuda.current_stream().cuda_stream)
    assert st == rcast.RC_E_INVAL


@pytest.mark.parametrize("dims", [(150, 40, 37), (128, 17, 33), (65, 70, 18), (70, 530, 12),
                                  (66, 12, 600)])
def test_wide_rows_and_long_columns(ctx, dims):
    """Rows of several 64-voxel words (ragged and exact) and columns of
    several 16-row segments, for the packed outside labelling, with both
    smoothing paths (n = 2 and n = 6), then marching cubes.  Columns of up
    to 32 segments take the one-kernel column pass, longer ones (530 rows
    along y, 600 along z) the three-kernel one."""
    nx, ny, nz = dims
    rng = np.random.default_rng(nx + ny + nz)
    surf = (rng.random((nz, ny, nx)) < 0.12).astype(np.uint8)
    # a closed box shell with one hole: its inside is reached only through it
    surf[4:nz - 4, 5:ny - 5, 6:nx - 6] = 1
    surf[5:nz - 5, 6:ny - 6, 7:nx - 7] = 0
    surf[nz // 2, ny // 2, 6] = 0
    for sigma, tau, band in ((0.02, 0.15, 0.06), (0.035, 0.2, 0.1)):
        phi, g = check_tsdf(ctx, surf, (0.05, 0.0, -0.1), 0.02, sigma, tau, band,
                            tag=f"wide {dims} sigma {sigma}")
    check_mc(ctx, phi, g, (0.05, 0.0, -0.1), 0.02, 0.0, tag=f"wide {dims} mc")


def test_unaligned_output_buffers(ctx):
    """The surface mask, phi and V~ as views one element into larger
    buffers (not 4- / 16-byte aligned): the library falls back to its
    element-wise paths and the results stay bit-exact."""
    import torch
    nz, ny, nx = 21, 26, 70
    rng = np.random.default_rng(5)
    surf = (rng.random((nz, ny, nx)) < 0.15).astype(np.uint8)
    g = ctx.grid((0.1, -0.2, 0.3), 0.02, (nx, ny, nz), 0.0)
    n = nx * ny * nz
    phi_buf = torch.full((n + 1,), 7.0, dtype=torch.float32, device="cuda")
    vt_buf = torch.full((n + 1,), 9, dtype=torch.uint8, device="cuda")
    phi = phi_buf[1:].view(nz, ny, nx)
    vt = vt_buf[1:].view(nz, ny, nx)
    assert phi.data_ptr() % 16 != 0 and vt.data_ptr() % 4 != 0
    surf_buf = torch.zeros((n + 1,), dtype=torch.uint8, device="cuda")
    surf_buf[1:] = cuda(surf).reshape(-1)
    surf_d = surf_buf[1:].view(nz, ny, nx)
    ctx.tsdf(g, surf_d, phi, 0.02, 0.15, 0.06, out_vtilde=vt)
    torch.cuda.synchronize()
    phi_o, vt_o, _, _ = ot.tsdf(surf, 0.02, 0.02, 0.15, 0.06)
    np.testing.assert_array_equal(vt.cpu().numpy(), vt_o)
    np.testing.assert_array_equal(phi.cpu().numpy().view(np.uint32), phi_o.view(np.uint32))
    # the elements before the views are untouched
    assert float(phi_buf[0]) == 7.0 and int(vt_buf[0]) == 9


# ---- quantile re-threshold and mc_step -------------------------------------

@pytest.mark.parametrize("q", [0.0, 0.35, 0.5, 0.93, 1.0])
def test_quantile_rethreshold(ctx, q):
    # V~ = [V' >= Quantile_q(V')] decided on the exact integer sums: V~ and
    # phi bit-exact with the oracle, on a ragged grid with a 2-step kernel
    import torch
    rng = np.random.default_rng(21)
    surf = (rng.random((13, 17, 29)) < 0.2).astype(np.uint8)
    h, sigma, band = 0.05, 0.05, 0.15
    nz, ny, nx = surf.shape
    g = ctx.grid((0.1, -0.3, 0.0), h, (nx, ny, nz), 0.0)
    phi = torch.full((nz, ny, nx), 7.0, dtype=torch.float32, device="cuda")
    vt = torch.full((nz, ny, nx), 9, dtype=torch.uint8, device="cuda")
    ctx.tsdf(g, cuda(surf), phi, sigma, 0.0, band, out_vtilde=vt, quantile=q)
    torch.cuda.synchronize()
    phi_o, vt_o, _, _ = ot.tsdf(surf, h, sigma, 0.0, band, quantile=q)
    np.testing.assert_array_equal(vt.cpu().numpy(), vt_o)
    np.testing.assert_array_equal(phi.cpu().numpy().view(np.uint32), phi_o.view(np.uint32))
    log(f"quantile {q}: V~ {int(vt_o.sum())} of {surf.size}")


def test_quantile_rethreshold_large_kernel(ctx):
    # 8-step kernel: sums up to 2^48, many distinct values
    import torch
    rng = np.random.default_rng(22)
    surf = (rng.random((20, 24, 30)) < 0.15).astype(np.uint8)
    h, sigma, band = 0.02, 0.04, 0.06
    nz, ny, nx = surf.shape
    g = ctx.grid((0.0, 0.0, 0.0), h, (nx, ny, nz), 0.0)
    phi = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
    vt = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    for q in (0.6, 0.85):
        ctx.tsdf(g, cuda(surf), phi, sigma, 0.0, band, out_vtilde=vt, quantile=q)
        torch.cuda.synchronize()
        phi_o, vt_o, _, _ = ot.tsdf(surf, h, sigma, 0.0, band, quantile=q)
        np.testing.assert_array_equal(vt.cpu().numpy(), vt_o)
        np.testing.assert_array_equal(phi.cpu().numpy().view(np.uint32), phi_o.view(np.uint32))


def test_quantile_rejects_bad_values(ctx):
    import torch
    surf = np.zeros((4, 4, 4), np.uint8)
    g = ctx.grid((0, 0, 0), 0.1, (4, 4, 4), 0.0)
    phi = torch.empty((4, 4, 4), dtype=torch.float32, device="cuda")
    for q in (-0.1, 1.5, float("nan")):
        with pytest.raises(rcast.RcastError) as e:
            ctx.tsdf(g, cuda(surf), phi, 0.1, 0.0, 0.2, quantile=q)
        assert e.value.status == rcast.RC_E_INVAL


@pytest.mark.parametrize("step", [1, 2, 3, 5])
def test_mc_step(ctx, step):
    # marching cubes on every step-th lattice point: topology, numbering and
    # float32 positions and normals bit-exact with the oracle's evaluation
    # on the coarse lattice, positions within the FP64 definition's bounds
    import torch
    rng = np.random.default_rng(30 + step)
    surf = (rng.random((26, 31, 37)) < 0.05).astype(np.uint8)
    origin, h = (0.25, -0.5, 0.125), 0.04
    phi, g = check_tsdf(ctx, surf, origin, h, 0.04, 0.1, 0.16, tag=f"mc_step {step} field")
    vo, to, no = ot.marching_cubes_step(phi, origin, h, step, 0.0, normals=True)
    hs = float(np.float32(np.float32(h) * np.float32(step)))
    o2 = tuple(float(np.float32(float(np.float32(o)) - (step - 1) * float(np.float32(h)) / 2.0))
               for o in origin)
    coarse = np.ascontiguousarray(phi[::step, ::step, ::step])
    x64, n64, ptol, ntol = ot.marching_cubes_fp64(coarse, o2, hs, 0.0)
    v, t, n = ctx.marching_cubes(g, cuda(phi), 0.0, normals=True, step=step)
    torch.cuda.synchronize()
    v, t, n = v.cpu().numpy(), t.cpu().numpy(), n.cpu().numpy()
    np.testing.assert_array_equal(t, to)
    np.testing.assert_array_equal(v.view(np.uint32), vo.view(np.uint32))
    np.testing.assert_array_equal(n.view(np.uint32), no.view(np.uint32))
    assert np.all(np.abs(v.astype(np.float64) - x64) <= ptol)
    log(f"mc_step {step}: {len(v)} vertices, {len(t)} triangles")


def test_mc_step_rejects_zero(ctx):
    surf = np.zeros((4, 4, 4), np.float32)
    g = ctx.grid((0, 0, 0), 0.1, (4, 4, 4), 0.0)
    with pytest.raises(rcast.RcastError) as e:
        ctx.marching_cubes(g, cuda(surf), 0.0, step=0)
    assert e.value.status == rcast.RC_E_INVAL


def test_marching_cubes_many_scan_tiles(ctx):
    # 9.2M lattice points: 9,000 scan tiles of 1,024 points, more than the
    # 8,192 tile totals one LDS chunk of the tile-offset scan holds, so the
    # scan carries its running totals across chunks; two spheres, compared
    # bit for bit with the oracle's float32 evaluation
    import torch
    nz, ny, nx = 96, 300, 320
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = (np.minimum(np.sqrt((x - 100.3) ** 2 + (y - 150.2) ** 2 + (z - 48.1) ** 2) - 40.7,
                      np.sqrt((x - 230.6) ** 2 + (y - 120.4) ** 2 + (z - 50.3) ** 2) - 35.2)
           * 0.01).astype(np.float32)
    g = ctx.grid((0.0, 0.0, 0.0), 0.01, (nx, ny, nz), 0.0)
    log(f"marching cubes on {phi.size} points")
    vg, tg, ng = ctx.marching_cubes(g, torch.from_numpy(phi).cuda(), 0.0, normals=True)
    torch.cuda.synchronize()
    vo, to, no = ot.marching_cubes(phi, (0.0, 0.0, 0.0), 0.01, 0.0, normals=True)
    assert len(to) > 100_000
    np.testing.assert_array_equal(tg.cpu().numpy(), to)
    np.testing.assert_array_equal(vg.cpu().numpy().view(np.uint32), vo.view(np.uint32))
    np.testing.assert_array_equal(ng.cpu().numpy().view(np.uint32), no.view(np.uint32))
