"""Quadric-error decimation by rounds of parallel edge contraction on the GPU
(rc_decimate_qem) against the oracle (oracle/qem.py), FGGS-LiDAR Sec. IV-B
"Mesh optimization" with the Sec. V defaults (ratio 0.1, three rounds,
boundary protected).  Parity bar: bit-exact -- equal float32 vertex bits,
equal face lists, equal step counts -- since both sides evaluate the same
FP64 operations in the same order and take every decision on the same
values."""
import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from oracle import qem
from paper_2509_17390_amd import Context
from paper_2509_17390_amd.rcast import RC_E_INVAL, RcastError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def check(ctx, v, t, ratio=0.1, rounds=3, tag=""):
    log(f"qem {tag}: {len(t)} faces, ratio {ratio}, rounds {rounds}")
    gv, gt, steps = ctx.decimate_qem(cuda(v), cuda(t), ratio, rounds)
    gv, gt = gv.cpu().numpy(), gt.cpu().numpy()
    trace = []
    ov, ot = qem.decimate_qem(v, t, ratio, rounds, trace=trace)
    assert gt.shape == ot.shape and np.array_equal(gt, ot), tag
    assert gv.shape == ov.shape and np.array_equal(gv.view(np.uint32), ov.view(np.uint32)), tag
    assert steps == len(trace), (steps, len(trace))
    return gv, gt


@pytest.mark.parametrize("ratio", [0.1, 0.3])
def test_uv_sphere(ctx, ratio):
    v, t = synth.uv_sphere((0.5, -0.25, 1.0), 1.0, 24, 12)
    check(ctx, v, t, ratio, 3, f"sphere {ratio}")


def test_noisy_sphere_many_rounds(ctx):
    rng = np.random.default_rng(11)
    v, t = synth.uv_sphere((0.0, 0.0, 0.0), 1.0, 40, 20)
    v = (v + rng.normal(scale=0.004, size=v.shape)).astype(np.float32)
    check(ctx, v, t, 0.1, 3, "noisy sphere")
    check(ctx, v, t, 0.25, 1, "noisy sphere, one round")
    check(ctx, v, t, 0.05, 5, "noisy sphere, five rounds")


def test_box_keeps_its_corners(ctx):
    gv, gt = check(ctx, *synth.grid_box((0.0, 0.0, 0.0), (2.0, 1.5, 1.0), 6), 0.1, 3, "box")
    corners = {(x, y, z) for x in (0.0, 2.0) for y in (0.0, 1.5) for z in (0.0, 1.0)}
    assert corners <= {tuple(p) for p in gv.astype(np.float64).tolist()}


def test_open_patch_keeps_its_boundary(ctx):
    v, t = synth.grid_patch(14, 1.0, 0.25)
    gv, _ = check(ctx, v, t, 0.3, 3, "patch")
    frame = np.any((v[:, :2] == 0.0) | (v[:, :2] == 1.0), axis=1)
    keep = {tuple(p) for p in gv.tolist()}
    assert all(tuple(p) in keep for p in v[frame].tolist())


def test_marching_cubes_mesh(ctx):
    sdf = synth.indoor_sdf(7, n_prims=4)
    v, t = synth.polygonise(sdf, 0.6)
    check(ctx, v, t, 0.1, 3, "marching cubes")


def test_ratio_one_repeated_corners_and_unused_vertices(ctx):
    v, t = synth.uv_sphere((0.0, 0.0, 0.0), 1.0, 10, 5)
    extra = np.array([[5.0, 5.0, 5.0]], np.float32)              # used by no face
    bad = np.array([[0, 0, 1], [2, 3, 2]], np.int32)             # repeated corners
    v2 = np.concatenate([v, extra])
    t2 = np.concatenate([t, bad])
    gv, gt = check(ctx, v2, t2, 1.0, 3, "identity")
    assert np.array_equal(gv, v) and np.array_equal(gt, t)
    check(ctx, v2, t2, 0.2, 3, "repeated corners")


def test_two_components_and_a_lone_triangle(ctx):
    a = synth.uv_sphere((0.0, 0.0, 0.0), 1.0, 16, 8)
    b = synth.grid_box((3.0, 0.0, 0.0), (4.0, 1.0, 1.0), 4)
    c = (np.array([[0, 5, 0], [1, 5, 0], [0, 6, 0]], np.float32), np.array([[0, 1, 2]], np.int32))
    v, t = synth.concat_meshes(a, b, c)
    check(ctx, v, t, 0.1, 3, "components")


def test_errors(ctx):
    v, t = synth.uv_sphere((0.0, 0.0, 0.0), 1.0, 8, 4)
    vd, td = cuda(v), cuda(t)
    for ratio, rounds in ((0.0, 3), (1.5, 3), (float("nan"), 3), (0.1, 0), (0.1, 65)):
        with pytest.raises(RcastError) as e:
            ctx.decimate_qem(vd, td, ratio, rounds)
        assert e.value.status == RC_E_INVAL
    bad = t.copy()
    bad[3, 1] = len(v)
    with pytest.raises(RcastError) as e:
        ctx.decimate_qem(vd, cuda(bad), 0.1, 3)
    assert e.value.status == RC_E_INVAL


def edge_counts(t):
    e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e[:, 0].astype(np.int64) << 32 | e[:, 1], return_counts=True)
    return cnt


@pytest.mark.parametrize("h", [0.1, 0.06])
def test_large_marching_cubes_mesh_properties(ctx, h):
    # 88k / 244k faces (the oracle's pure-Python steps would take hours):
    # what the definition guarantees at any size -- the round targets are
    # met to within one face, the mesh stays closed and manifold with the
    # same Euler characteristic, faces are proper triangles of used
    # vertices, and every vertex is finite
    sdf = synth.indoor_sdf(2, n_prims=40)
    v, t = synth.polygonise(sdf, h)
    c0 = edge_counts(t)
    assert np.all(c0 == 2)
    log(f"qem large: {len(t)} faces")
    gv, gt, steps = ctx.decimate_qem(cuda(v), cuda(t), 0.1, 3)
    gv, gt = gv.cpu().numpy(), gt.cpu().numpy()
    T = qem.round_targets(len(t), 0.1, 3)[-1]
    assert T - 1 <= len(gt) <= T
    c1 = edge_counts(gt)
    assert np.all(c1 == 2)
    eu0 = len(np.unique(t)) - len(c0) + len(t)
    eu1 = len(np.unique(gt)) - len(c1) + len(gt)
    assert eu0 == eu1
    assert len(np.unique(gt)) == len(gv)
    assert not np.any((gt[:, 0] == gt[:, 1]) | (gt[:, 1] == gt[:, 2]) | (gt[:, 0] == gt[:, 2]))
    assert np.all(np.isfinite(gv))
    # and the same call twice gives the same bits
    gv2, gt2, steps2 = ctx.decimate_qem(cuda(v), cuda(t), 0.1, 3)
    assert steps2 == steps and np.array_equal(gt2.cpu().numpy(), gt)
    assert np.array_equal(gv2.cpu().numpy().view(np.uint32), gv.view(np.uint32))
    log(f"qem large: {len(t)} -> {len(gt)} faces in {steps} steps")
