"""Gaussian-to-occupancy conversion on the GPU vs the FP64 oracle
(oracle/gauss.py): FGGS-LiDAR Sec. IV-A "Grid query and occupancy
evaluation" on the Gaussian model of Sec. III-A.

Parity bar:
  * Gaussian boxes: bit-exact (both sides evaluate them in FP64 in one fixed
    operation order and round to float32; membership in C_tile is decided on
    these float32 values).
  * |C_tile| per tile: bit-exact.
  * density: |D_gpu - D| <= 2^-24 (16 E + 4 D) + (K + 1) 2^-31 per voxel,
    with E the oracle's error scale sum_i t_i (1 + q_i + sum_b |u_ib| L_i /
    s_ib) and K = |C_tile|.  Derivation: an FP32 evaluation in tile-local
    voxel units perturbs the whitened coordinates u_b by at most about
    2^-24 * 6 L / s_b (L = the tile diagonal plus |v - mu|: rounding of
    the whitening matrix, of the tile-frame offset and of the products), so
    the exponent q moves by 2 sum_b |u_b| du_b and the term by that times
    ln 2 (with the constant log2(e)/2 folded in: < 6 * 2^-24 G), plus about
    1.5 q + 4 ulps for forming q, exp2 and the fixed-point step; each term
    also rounds to a multiple of 2^-31, and D is rounded to float32 once.
    That bound is 6 E + 2 D in units of 2^-24; the test allows twice that.
  * occupancy: bit-exact against [D_gpu > theta] (the decision is taken on
    the float32 D), and equal to the oracle's wherever |D - theta| exceeds
    the tolerance.
  * surface mask: bit-exact against the oracle's mask of the GPU occupancy.
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from oracle import gauss as og
from paper_2509_17390_amd import Context
from paper_2509_17390_amd import rcast

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24
U31 = 2.0 ** -31


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def run(ctx, params, grid: og.Grid, k=3.0, outputs=("d", "o", "s")):
    import torch
    g = ctx.upload_gaussians(*params)
    ctx.build_gaussians(g, cutoff_sigma=k)
    nx, ny, nz = grid.dims
    D = torch.full((nz, ny, nx), -1.0, dtype=torch.float32, device="cuda") if "d" in outputs else None
    O = torch.full((nz, ny, nx), 7, dtype=torch.uint8, device="cuda") if "o" in outputs else None
    S = torch.full((nz, ny, nx), 7, dtype=torch.uint8, device="cuda") if "s" in outputs else None
    rg = ctx.grid(grid.origin, float(grid.h), grid.dims, float(grid.theta), grid.tile)
    ctx.voxelize(g, rg, D, O, S)
    tx, ty, tz = grid.tiles
    C = torch.full((tz, ty, tx), -1, dtype=torch.int32, device="cuda")
    ctx.voxelize_counts(g, rg, C)
    torch.cuda.synchronize()
    out = {"set": g, "counts": C.cpu().numpy()}
    if D is not None:
        out["D"] = D.cpu().numpy()
    if O is not None:
        out["occ"] = O.cpu().numpy()
    if S is not None:
        out["surf"] = S.cpu().numpy()
    return out


def check(params, grid, res, k=3.0, tag=""):
    D, counts, E = og.density(params, grid, k, with_error=True)
    np.testing.assert_array_equal(res["counts"], counts)
    B = grid.tile
    nx, ny, nz = grid.dims
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    K = counts[iz // B, iy // B, ix // B].astype(np.float64)
    tol = U24 * (16 * E + 4 * D) + (K + 1) * U31
    err = np.abs(res["D"].astype(np.float64) - D)
    ratio = float(np.max(err / tol))
    log(f"{tag}: voxels {D.size}, max |C_tile| {counts.max()}, max err {err.max():.3g}, "
        f"max err/tol {ratio:.3f}")
    assert ratio <= 1.0
    theta = grid.theta
    np.testing.assert_array_equal(res["occ"], (res["D"] > theta).astype(np.uint8))
    clear = np.abs(D - float(theta)) > tol
    np.testing.assert_array_equal(res["occ"][clear], (D[clear] > float(theta)).astype(np.uint8))
    np.testing.assert_array_equal(res["surf"], og.surface(res["occ"]))
    return D


def test_boxes_bit_exact(ctx):
    rng = np.random.default_rng(1)
    params = synth.random_gaussians(rng, 20000, (-50, -50, -5), (50, 50, 5), 1e-3, 2.0)
    # extreme quaternions: near-zero components, huge and tiny norms
    params[1][:100] *= np.float32(1e-18)
    params[1][100:200] *= np.float32(1e18)
    params[1][200:300, 1:] = 0
    for k in (3.0, 2.5):
        g = ctx.upload_gaussians(*params)
        ctx.build_gaussians(g, cutoff_sigma=k)
        got = ctx.gauss_debug_copy(g, rcast.RC_GDBG_BOXES)
        want = og.gauss_boxes(*params[:3], k)
        np.testing.assert_array_equal(got, want)
        ctx.release_gaussians(g)


def test_records_match_the_model(ctx):
    rng = np.random.default_rng(2)
    params = synth.random_gaussians(rng, 3000, (0, 0, 0), (4, 4, 4))
    g = ctx.upload_gaussians(*params)
    ctx.build_gaussians(g)
    rec = ctx.gauss_debug_copy(g, rcast.RC_GDBG_RECORDS)
    order = ctx.gauss_debug_copy(g, rcast.RC_GDBG_SORTED)
    ids = rec[:, 13].view(np.int32)
    np.testing.assert_array_equal(ids, order.astype(np.int32))
    assert sorted(ids.tolist()) == list(range(3000))
    mu, q, s, a = (x[ids] for x in params)
    np.testing.assert_array_equal(rec[:, 0:3], mu)
    np.testing.assert_allclose(rec[:, 3], a.astype(np.float64) ** 2 * 2.0 ** 31, rtol=2 ** -23)
    R = og.rotation_matrices(q)
    c0 = math.sqrt(math.log2(math.e) / 2)
    M = c0 * np.transpose(R, (0, 2, 1)) / s.astype(np.float64)[:, :, None]
    np.testing.assert_allclose(rec[:, [4, 5, 6, 7, 8, 9, 10, 11, 12]].reshape(-1, 3, 3), M,
                               rtol=2 ** -22, atol=1e-30)
    ctx.release_gaussians(g)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_gaussians_ragged_grid(ctx, seed):
    rng = np.random.default_rng(10 + seed)
    params = synth.random_gaussians(rng, 600, (-0.3, -0.2, -0.1), (2.1, 1.6, 1.3), 0.02, 0.25)
    grid = og.Grid((0.013, -0.021, 0.007), 0.05, (37, 29, 23), tile=8, theta=0.4)
    log(f"random seed {seed}: 600 Gaussians, grid 37x29x23")
    res = run(ctx, params, grid)
    check(params, grid, res, tag=f"random seed {seed}")
    ctx.release_gaussians(res["set"])


def test_flat_surface_gaussians(ctx):
    """Disc-shaped Gaussians on surfaces (the structure of trained 3DGS
    assets), a region of the indoor scene near a wall."""
    m, q, s, a, room = synth.splat_scene(1, 200000)
    lo = np.array([-0.1, 2.0, 1.0])
    grid = og.Grid(lo, 0.02, (40, 36, 33), tile=8, theta=0.5)
    hi = lo + 0.02 * np.array(grid.dims)
    boxes = og.gauss_boxes(m, q, s, 3.0)
    sel = np.all((boxes[:, :3] <= hi + 0.3) & (boxes[:, 3:] >= lo - 0.3), axis=1)
    params = (m[sel], q[sel], s[sel], a[sel])
    log(f"splat region: {sel.sum()} Gaussians, grid 40x36x33")
    res = run(ctx, params, grid)
    D = check(params, grid, res, tag="splat region")
    assert res["occ"].sum() > 100 and res["surf"].sum() > 100
    ctx.release_gaussians(res["set"])


def test_dense_cluster_overflows_batches(ctx):
    """Thousands of Gaussians in one tile: the culling set runs through the
    LDS ring many times and the per-lane walks go deep."""
    rng = np.random.default_rng(5)
    params = synth.random_gaussians(rng, 3000, (0.1, 0.1, 0.1), (0.3, 0.3, 0.3), 0.01, 0.05)
    grid = og.Grid((0, 0, 0), 0.05, (12, 12, 12), tile=8, theta=1.0)
    res = run(ctx, params, grid)
    check(params, grid, res, tag="dense cluster")
    assert res["counts"].max() > 1000
    ctx.release_gaussians(res["set"])


def test_huge_gaussian_and_outside_ones(ctx):
    rng = np.random.default_rng(6)
    p = list(synth.random_gaussians(rng, 50, (5, 5, 5), (6, 6, 6), 0.01, 0.05))   # all outside
    big = synth.random_gaussians(rng, 1, (0.5, 0.5, 0.5), (0.6, 0.6, 0.6), 3.0, 4.0)
    params = tuple(np.concatenate([x, y]) for x, y in zip(p, big))
    grid = og.Grid((0, 0, 0), 0.1, (17, 9, 11), tile=8, theta=0.01)
    res = run(ctx, params, grid)
    check(params, grid, res, tag="huge + outside")
    assert np.all(res["counts"] == 1)
    ctx.release_gaussians(res["set"])


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_sets(ctx, n):
    rng = np.random.default_rng(20 + n)
    params = synth.random_gaussians(rng, n, (0.2, 0.2, 0.2), (0.5, 0.5, 0.5), 0.05, 0.2)
    grid = og.Grid((0, 0, 0), 0.07, (11, 10, 9), tile=8, theta=0.2)
    res = run(ctx, params, grid)
    check(params, grid, res, tag=f"n={n}")
    ctx.release_gaussians(res["set"])


def test_empty_set_and_single_voxel_grid(ctx):
    import torch
    empty = tuple(np.zeros((0, w), np.float32) for w in (3, 4, 3)) + (np.zeros(0, np.float32),)
    grid = og.Grid((0, 0, 0), 0.1, (9, 8, 17), tile=8, theta=0.0)
    res = run(ctx, empty, grid)
    assert np.all(res["D"] == 0) and np.all(res["occ"] == 0) and np.all(res["surf"] == 0)
    assert np.all(res["counts"] == 0)
    ctx.release_gaussians(res["set"])
    params = (np.array([[0.05, 0.05, 0.05]], np.float32), np.array([[1, 0, 0, 0]], np.float32),
              np.array([[0.1, 0.1, 0.1]], np.float32), np.array([0.9], np.float32))
    one = og.Grid((0, 0, 0), 0.1, (1, 1, 1), tile=8, theta=0.5)
    res = run(ctx, params, one)
    check(params, one, res, tag="1 voxel")
    assert res["occ"][0, 0, 0] == 1 and res["surf"][0, 0, 0] == 1
    ctx.release_gaussians(res["set"])


def test_cutoff_changes_the_culling_set(ctx):
    rng = np.random.default_rng(8)
    params = synth.random_gaussians(rng, 300, (0, 0, 0), (1.5, 1.5, 1.5), 0.02, 0.1)
    grid = og.Grid((0, 0, 0), 0.04, (40, 38, 36), tile=8, theta=0.3)
    for k in (1.5, 4.0):
        res = run(ctx, params, grid, k=k)
        check(params, grid, res, k=k, tag=f"k={k}")
        ctx.release_gaussians(res["set"])


def test_outputs_are_optional_and_deterministic(ctx):
    import torch
    rng = np.random.default_rng(9)
    params = synth.random_gaussians(rng, 2000, (0, 0, 0), (2, 2, 2), 0.02, 0.2)
    grid = og.Grid((0, 0, 0), 0.03, (70, 66, 65), tile=8, theta=0.5)
    full = run(ctx, params, grid)
    d_only = run(ctx, params, grid, outputs=("d",))
    o_only = run(ctx, params, grid, outputs=("o",))
    assert np.array_equal(full["D"].view(np.uint32), d_only["D"].view(np.uint32))
    assert np.array_equal(full["occ"], o_only["occ"])
    with pytest.raises(rcast.RcastError):
        rg = ctx.grid(grid.origin, float(grid.h), grid.dims, float(grid.theta))
        S = torch.zeros((65, 66, 70), dtype=torch.uint8, device="cuda")
        ctx.voxelize(full["set"], rg, None, None, S)
    for r in (full, d_only, o_only):
        ctx.release_gaussians(r["set"])


def test_invalid_inputs_are_rejected(ctx):
    rng = np.random.default_rng(3)
    good = synth.random_gaussians(rng, 10)
    bad_cases = []
    for arr, idx, val in [(0, (2, 1), np.nan), (1, (3,), 0.0), (2, (4, 2), 0.0),
                          (2, (5, 0), -1.0), (3, (6,), 1.5), (3, (7,), np.inf)]:
        p = [x.copy() for x in good]
        if arr == 1:
            p[1][idx[0]] = 0.0
        else:
            p[arr][idx] = val
        bad_cases.append(p)
    for p in bad_cases:
        with pytest.raises(rcast.RcastError) as e:
            ctx.upload_gaussians(*p)
        assert e.value.status == rcast.RC_E_INVAL
    g = ctx.upload_gaussians(*good)
    rg = ctx.grid((0, 0, 0), 0.1, (8, 8, 8), 0.5)
    import torch
    D = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(rcast.RcastError) as e:
        ctx.voxelize(g, rg, D)
    assert e.value.status == rcast.RC_E_STATE
    ctx.build_gaussians(g)
    for bad in [ctx.grid((0, 0, 0), 0.0, (8, 8, 8), 0.5), ctx.grid((0, 0, 0), 0.1, (8, 0, 8), 0.5),
                ctx.grid((0, 0, 0), 0.1, (8, 8, 8), 0.5, tile=4),
                ctx.grid((0, 0, 0), 0.1, (8, 8, 8), float("nan"))]:
        with pytest.raises(rcast.RcastError) as e:
            ctx.voxelize(g, bad, D)
        assert e.value.status == rcast.RC_E_INVAL
    with pytest.raises(rcast.RcastError) as e:
        ctx.build_gaussians(g, cutoff_sigma=-1.0)
    assert e.value.status == rcast.RC_E_INVAL
    ctx.release_gaussians(g)
