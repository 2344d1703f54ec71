"""GPU ray casting vs the FP64 oracle (parity bar in tests/gpu_util.py).

Covers the room + sphere scene in full, random triangle soups (1..1000
triangles, exhaustive), closed indoor meshes (coarse in full-ish samples,
the one-million-triangle mesh on a sampled subset of its 8 x 32,768 rays),
bit-exact agreement between the BVH kernel and the brute-force kernel,
multi-job batches, the instrumented traversal and edge cases.
"""
import numpy as np
import pytest

import synth
from gpu_util import cast_scene, compare_with_oracle, cuda, log, oracle_checked
from paper_2509_17390_amd import Context, Job, RcastError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_room_sphere_all_rays(ctx, seed):
    s = synth.room_sphere_scene(seed)
    log(f"room_sphere seed={seed} rays={s.n_rays}")
    (rng, hit), _, _ = cast_scene(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                  n_az=s.n_az)
    assert np.all(hit >= 0)  # closed room: every ray hits
    st = compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, rng, hit)
    log(str(st))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 255, 256, 257, 1000])
def test_random_soups(ctx, n):
    rng_ = np.random.default_rng(1000 + n)
    v, t = synth.random_soup(rng_, n, 1.0)
    poses = np.stack([synth.rpy_pose(rng_.uniform(-2, 2, 3), *rng_.uniform(-np.pi, np.pi, 3))
                      for _ in range(3)])
    dirs = synth.lidar_pattern(9, -60.0, 60.0, 71)   # 639 beams: ragged vs 64-lane waves
    log(f"soup n={n}")
    (r, h), _, _ = cast_scene(ctx, v, t, poses, dirs, 0.0, 50.0)
    compare_with_oracle(v, t, poses, dirs, 0.0, 50.0, r, h, min_checked_frac=0.9)
    (rb, hb), _, _ = cast_scene(ctx, v, t, poses, dirs, 0.0, 50.0, mode="brute")
    assert np.array_equal(h, hb) and np.array_equal(r.view(np.int32), rb.view(np.int32))


def test_bvh_equals_bruteforce_bitexact(ctx):
    sdf = synth.indoor_sdf(7, n_prims=60)
    v, t = synth.polygonise(sdf, 0.08)
    poses = synth.free_space_poses(sdf, 6, 3)
    dirs = synth.lidar_pattern(16, -30.0, 30.0, 256)
    log(f"bvh vs brute tris={len(t)}")
    (r, h), _, _ = cast_scene(ctx, v, t, poses, dirs, 0.1, 120.0)
    (rb, hb), _, _ = cast_scene(ctx, v, t, poses, dirs, 0.1, 120.0, mode="brute")
    assert np.all(h >= 0)
    same = (h == hb) & (r.view(np.int32) == rb.view(np.int32))
    assert same.all(), np.flatnonzero(~same)[:10]


def test_indoor_coarse_parity(ctx):
    sdf = synth.indoor_sdf(11, n_prims=200)
    v, t = synth.polygonise(sdf, 0.1)
    poses = synth.free_space_poses(sdf, 4, 5)
    dirs = synth.lidar_pattern(32, -16.0, 15.0, 256)
    log(f"indoor coarse tris={len(t)}")
    (r, h), _, _ = cast_scene(ctx, v, t, poses, dirs, 0.1, 120.0)
    assert np.all(h >= 0)
    idx = np.random.default_rng(0).choice(len(poses) * len(dirs), 6000, replace=False)
    st = compare_with_oracle(v, t, poses, dirs, 0.1, 120.0, r, h, ray_idx=np.sort(idx))
    log(str(st))


def test_indoor_1m_sampled_parity(ctx):
    # the one-million-triangle indoor mesh with 8 poses x 32 x 1024 beams, as
    # cast in one launch; the oracle checks a seeded sample of the rays
    s = synth.indoor_scene(seed=1, h=0.035, n_envs=8)
    log(f"indoor 1M tris={len(s.tris)} rays={s.n_rays}")
    (r, h), scene, _ = cast_scene(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                  n_az=s.n_az)
    assert np.all(h >= 0)  # closed mesh, poses in free space
    info = ctx.scene_info(scene)
    assert info.n_tris == len(s.tris) and 0 < info.depth <= 64
    idx = np.sort(np.random.default_rng(1).choice(s.n_rays, 1536, replace=False))
    st = compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, r, h, ray_idx=idx)
    log(str(st))


def test_multi_job_batch_matches_single_jobs(ctx):
    import torch
    a = synth.room_sphere_scene(5)
    sdf = synth.indoor_sdf(2, n_prims=40)
    bv, bt = synth.polygonise(sdf, 0.1)
    bposes = synth.free_space_poses(sdf, 5, 2)
    sa = ctx.upload_scene(a.verts, a.tris)
    sb = ctx.upload_scene(bv, bt)
    ctx.build(sa)
    ctx.build(sb)
    pa = ctx.upload_pattern(a.dirs, a.n_az)
    pb = ctx.upload_pattern(synth.lidar_pattern(32, -16, 15, 100), 100)
    ja = Job(sa, pa, cuda(np.repeat(a.poses, 3, 0)), a.t_min, a.t_max, 0)
    jb = Job(sb, pb, cuda(bposes), 0.1, 120.0, 3 * 5760 + 17)
    jc = Job(sb, pa, cuda(bposes[:2]), 0.5, 30.0, 3 * 5760 + 17 + 5 * 3200)
    log("multi-job batch")
    r_all, h_all = ctx.cast([ja, jb, jc])
    for j in (ja, jb, jc):
        n = j.n_envs * ctx.n_beams(j.pattern)
        r1, h1 = ctx.cast([Job(j.scene, j.pattern, j.poses, j.t_min, j.t_max, 0)])
        sl = slice(j.out_offset, j.out_offset + n)
        assert torch.equal(h_all[sl], h1) and torch.equal(r_all[sl].view(torch.int32),
                                                          r1.view(torch.int32))
    # the gap between job slices is left untouched
    torch.cuda.synchronize()


def test_stats_mode_matches_and_counts(ctx):
    s = synth.room_sphere_scene(0)
    (r, h), _, _ = cast_scene(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max)
    (r2, h2, nn, nt), _, _ = cast_scene(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                        mode="stats")
    assert np.array_equal(h, h2) and np.array_equal(r.view(np.int32), r2.view(np.int32))
    assert nn.min() >= 1 and nt.min() >= 1
    assert nn.mean() < 200 and nt.mean() < 100


def test_edge_cases(ctx):
    import torch
    # forward-facing fan: elevation -10..10 deg, azimuth -30..30 deg
    el, az = np.meshgrid(np.radians(np.linspace(-10, 10, 4)),
                         np.radians(np.linspace(-30, 30, 16)), indexing="ij")
    dirs = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)],
                    -1).reshape(-1, 3).astype(np.float32)
    pat = ctx.upload_pattern(dirs, 16)
    pose = cuda(synth.yaw_pose((0, 0, 0), 0.0)[None])
    # empty mesh: every ray misses
    s0 = ctx.upload_scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    ctx.build(s0)
    r, h = ctx.cast([Job(s0, pat, pose, 0.0, 10.0)])
    assert torch.all(h == -1) and torch.all(torch.isinf(r))
    # one triangle (no internal node)
    tri = np.array([[5, -50, -50], [5, 50, -50], [5, 0, 50]], np.float32)
    s1 = ctx.upload_scene(tri, np.array([[0, 1, 2]], np.int32))
    ctx.build(s1)
    r, h = ctx.cast([Job(s1, pat, pose, 0.0, 10.0)])
    assert torch.all(h == 0)
    # beam 0: elevation -10, azimuth -30 -> range 5 / (cos(el) cos(az))
    assert abs(float(r[0]) - 5.0 / (np.cos(np.radians(10)) * np.cos(np.radians(30)))) < 1e-4
    # zero environments: nothing written, no error
    r, h = ctx.cast([Job(s1, pat, cuda(np.zeros((0, 12), np.float32)), 0.0, 10.0)])
    assert r.numel() == 0
    # t range excludes the hit
    r, h = ctx.cast([Job(s1, pat, pose, 0.0, 4.0)])
    assert torch.all(h == -1)
    # invalid inputs
    with pytest.raises(RcastError) as e:
        ctx.upload_scene(tri, np.array([[0, 1, 3]], np.int32))
    assert e.value.status == -1
    bad = tri.copy()
    bad[1, 1] = np.nan
    with pytest.raises(RcastError):
        ctx.upload_scene(bad, np.array([[0, 1, 2]], np.int32))
    s2 = ctx.upload_scene(tri, np.array([[0, 1, 2]], np.int32))
    with pytest.raises(RcastError) as e:
        ctx.cast([Job(s2, pat, pose, 0.0, 10.0)])   # no BVH yet
    assert e.value.status == -6
    with pytest.raises(RcastError):
        ctx.cast([Job(s1, pat, pose, 5.0, 1.0)])
    with pytest.raises(RcastError):
        ctx.cast([Job(99, pat, pose, 0.0, 1.0)])
    for s in (s0, s1, s2):
        ctx.release_scene(s)
    with pytest.raises(RcastError):
        ctx.cast([Job(s1, pat, pose, 0.0, 10.0)])


def test_duplicate_and_degenerate_triangles(ctx):
    # equal Morton codes (stacked duplicates) and zero-area triangles
    v, t = synth.box_room()
    t2 = np.concatenate([t, t, t[::-1]]).astype(np.int32)
    deg = np.array([[0, 0, 1], [2, 2, 2]], np.int32)
    t2 = np.concatenate([deg, t2]).astype(np.int32)
    poses = np.stack([synth.yaw_pose((5, 4, 1.5), 0.3), synth.yaw_pose((1, 1, 1), 2.0)])
    dirs = synth.lidar_pattern(8, -80, 80, 64)
    (r, h), _, _ = cast_scene(ctx, v, t2, poses, dirs, 0.0, 100.0)
    assert np.all(h >= 2) and np.all(h < 2 + 12)   # lowest duplicate id wins
    # duplicates make every ray "ambiguous" to the checker, but the exact-tie
    # rule fixes the answer: ids must equal the oracle's away from edges
    import oracle
    t_o, i_o, fl, _, _ = oracle.raycast(v, t2, poses, dirs, 0.0, 100.0, checked=True)
    clear = (fl & oracle.FLAG_EDGE_NEAR) == 0
    assert clear.mean() > 0.95
    assert np.array_equal(h[clear], i_o[clear])
    assert np.all(np.abs(r[clear] - t_o[clear]) <= 1e-4 + 1e-6 * t_o[clear])


TUNINGS = [
    dict(persistent=0, stack_lds=8, refill_min=64, blocks_per_cu=0, tile_az=16, tile_el=4, chunk_max=4096, waves_cap=1),
    dict(persistent=0, stack_lds=0, refill_min=32, blocks_per_cu=0, tile_az=0, tile_el=0, chunk_max=1024, waves_cap=0),
    dict(persistent=0, stack_lds=16, refill_min=32, blocks_per_cu=0, tile_az=0, tile_el=0, chunk_max=1024, waves_cap=0),
    dict(persistent=1, stack_lds=8, refill_min=1, blocks_per_cu=0, tile_az=0, tile_el=0, chunk_max=1024, waves_cap=0),
    dict(persistent=1, stack_lds=16, refill_min=32, blocks_per_cu=1, tile_az=16, tile_el=4, chunk_max=1024, waves_cap=0),
    dict(persistent=1, stack_lds=24, refill_min=64, blocks_per_cu=2, tile_az=8, tile_el=8, chunk_max=1024, waves_cap=0),
    dict(persistent=1, stack_lds=16, refill_min=48, blocks_per_cu=0, tile_az=64, tile_el=1, chunk_max=1024, waves_cap=0),
    dict(persistent=0, stack_lds=0, refill_min=64, blocks_per_cu=0, tile_az=16, tile_el=4, chunk_max=4096, waves_cap=1, group_waves=4),
    dict(persistent=0, stack_lds=16, refill_min=64, blocks_per_cu=0, tile_az=0, tile_el=0, chunk_max=4096, waves_cap=0, group_waves=4),
    # queued leaf tests (Q8 trees only; plain trees ignore leaf_batch)
    dict(persistent=0, stack_lds=0, refill_min=64, blocks_per_cu=0, tile_az=16, tile_el=4, chunk_max=4096, waves_cap=1, group_waves=1, leaf_batch=64),
    dict(persistent=0, stack_lds=0, refill_min=64, blocks_per_cu=0, tile_az=16, tile_el=4, chunk_max=4096, waves_cap=1, group_waves=1, leaf_batch=1),
    dict(persistent=0, stack_lds=0, refill_min=64, blocks_per_cu=0, tile_az=8, tile_el=8, chunk_max=4096, waves_cap=0, group_waves=1, leaf_batch=17),
    dict(persistent=0, stack_lds=0, refill_min=64, blocks_per_cu=0, tile_az=0, tile_el=0, chunk_max=4096, waves_cap=1, group_waves=4, leaf_batch=32),
]


def _variant_sample(s, n=700, seed=11):
    idx = np.sort(np.random.default_rng(seed).choice(s.n_rays, n, replace=False))
    return idx, oracle_checked(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, idx)


def test_tuning_variants_bit_identical(ctx):
    # every launch shape (persistent or not, stack depth in LDS, refill
    # threshold, grid size, packet tile) must give bit-identical results,
    # and each one meets the oracle on the same sample of rays
    import torch
    s = synth.indoor_scene(seed=3, h=0.1, n_envs=6, n_az=256)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    poses = cuda(s.poses)
    job = [Job(scene, pat, poses, s.t_min, s.t_max)]
    idx, orc = _variant_sample(s)
    ref = None
    try:
        for tn in TUNINGS:
            log(f"tuning {tn}")
            ctx.set_tuning(**tn)
            r, h = ctx.cast(job)
            r2, h2, nn, nt = ctx.cast(job, mode="stats")
            torch.cuda.synchronize()
            assert torch.equal(h, h2) and torch.equal(r.view(torch.int32), r2.view(torch.int32))
            compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                r.cpu().numpy(), h.cpu().numpy(), ray_idx=idx, oracle_out=orc)
            if ref is None:
                ref = (r.clone(), h.clone())
                assert bool((h >= 0).all())
            else:
                assert torch.equal(h, ref[1])
                assert torch.equal(r.view(torch.int32), ref[0].view(torch.int32))
    finally:
        ctx.reset_tuning()


def test_tuning_rejects_bad_values(ctx):
    with pytest.raises(RcastError):
        ctx.set_tuning(persistent=1, stack_lds=5)
    with pytest.raises(RcastError):
        ctx.set_tuning(refill_min=0)
    with pytest.raises(RcastError):
        ctx.set_tuning(refill_min=65)
    with pytest.raises(RcastError):
        ctx.set_tuning(group_waves=2)
    default = Context(0)
    try:
        ctx.set_tuning(persistent=1, stack_lds=24, refill_min=7)
        ctx.reset_tuning()
        assert ctx.get_tuning() == default.get_tuning()
    finally:
        default.close()


def _cast_both(ctx, verts, tris, poses, dirs, t_min, t_max, n_az=0):
    import torch
    out = []
    for fmt in (0, 1):
        scene = ctx.upload_scene(verts, tris)
        ctx.build(scene, node_format=fmt)
        pat = ctx.upload_pattern(dirs, n_az)
        r, h = ctx.cast([Job(scene, pat, cuda(poses), t_min, t_max)])
        torch.cuda.synchronize()
        out.append((r.cpu().numpy(), h.cpu().numpy()))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_q8_equals_fp32_and_oracle_room_sphere(ctx, seed):
    s = synth.room_sphere_scene(seed)
    log(f"q8 room_sphere seed={seed}")
    (r32, h32), (rq, hq) = _cast_both(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                      s.n_az)
    assert np.array_equal(h32, hq) and np.array_equal(r32.view(np.int32), rq.view(np.int32))
    compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, rq, hq)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 257, 1000])
def test_q8_equals_fp32_soups(ctx, n):
    rng_ = np.random.default_rng(2000 + n)
    v, t = synth.random_soup(rng_, n, 1.0)
    poses = np.stack([synth.rpy_pose(rng_.uniform(-2, 2, 3), *rng_.uniform(-np.pi, np.pi, 3))
                      for _ in range(3)])
    dirs = synth.lidar_pattern(9, -60.0, 60.0, 71)
    log(f"q8 soup n={n}")
    (r32, h32), (rq, hq) = _cast_both(ctx, v, t, poses, dirs, 0.0, 50.0)
    assert np.array_equal(h32, hq) and np.array_equal(r32.view(np.int32), rq.view(np.int32))


@pytest.mark.parametrize("n_el,n_az", [(1, 1), (1, 97), (3, 1025), (7, 64)])
def test_odd_pattern_sizes(ctx, n_el, n_az):
    """Patterns whose sizes the packet tile does not divide (one beam, a
    prime count, rings of 1025) fall back to ring order; many environments
    per job exercise the ray index -> (environment, beam) map."""
    import torch
    s = synth.room_sphere_scene(1)
    dirs = synth.lidar_pattern(n_el, -20.0, 20.0, n_az) if n_el > 1 else \
        synth.lidar_pattern(1, 5.0, 5.0, n_az)
    rng_ = np.random.default_rng(n_el * 1000 + n_az)
    p0 = s.poses[0].reshape(3, 4)[:, 3]
    poses = np.stack([synth.yaw_pose(p0 + rng_.uniform(-0.1, 0.1, 3), rng_.uniform(0, 6.283))
                      for _ in range(37)])
    log(f"odd pattern {n_el}x{n_az}")
    res = []
    for fmt in (0, 1):
        scene = ctx.upload_scene(s.verts, s.tris)
        ctx.build(scene, node_format=fmt)
        pat = ctx.upload_pattern(dirs, n_az)
        r, h = ctx.cast([Job(scene, pat, cuda(poses), s.t_min, s.t_max)])
        torch.cuda.synchronize()
        res.append((r.cpu().numpy(), h.cpu().numpy()))
        ctx.release_scene(scene)
    (r32, h32), (rq, hq) = res
    assert np.array_equal(h32, hq) and np.array_equal(r32.view(np.int32), rq.view(np.int32))
    assert np.all(hq >= 0)
    compare_with_oracle(s.verts, s.tris, poses, dirs, s.t_min, s.t_max, rq, hq)


@pytest.mark.parametrize("fmt", [0, 1])
def test_far_from_origin(ctx, fmt):
    """The room + sphere scene and its sensor moved 10-25 km away from the
    world origin (coordinates rounded to FP32 there, as a user would hold
    them): the FP32 traversal must still meet the parity bar.  Differences
    v - o of nearby points are exact in FP32 (Sterbenz), so only the shear and
    the ray rounding err, both far inside the 1e-6 rad edge margin."""
    import torch
    s = synth.room_sphere_scene(2)
    off = np.array([1.2e4, -2.5e4, 3.0e3])
    v = (s.verts.astype(np.float64) + off).astype(np.float32)
    poses = s.poses.astype(np.float64).copy()
    poses[:, [3, 7, 11]] += off
    poses = poses.astype(np.float32)
    log(f"far from origin fmt={fmt}")
    scene = ctx.upload_scene(v, s.tris)
    ctx.build(scene, node_format=fmt)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    r, h = ctx.cast([Job(scene, pat, cuda(poses), s.t_min, s.t_max)])
    torch.cuda.synchronize()
    r, h = r.cpu().numpy(), h.cpu().numpy()
    assert np.all(h >= 0)   # still a closed room
    st = compare_with_oracle(v, s.tris, poses, s.dirs, s.t_min, s.t_max, r, h)
    log(str(st))
    ctx.release_scene(scene)


@pytest.mark.parametrize("closed", [True, False])
def test_unbounded_range(ctx, closed):
    """t_max = +inf: the interval is [t_min, inf).  Closed room: every ray
    hits, exactly as with a finite bound beyond the room.  Open soup: rays
    that miss everything must come back as misses (missed and empty child
    slots carry +inf, which an infinite bound must not admit)."""
    if closed:
        s = synth.room_sphere_scene(0)
        v, t, poses, dirs, n_az = s.verts, s.tris, s.poses, s.dirs, s.n_az
    else:
        rng_ = np.random.default_rng(77)
        v, t = synth.random_soup(rng_, 300, 1.0)
        poses = np.stack([synth.rpy_pose(rng_.uniform(-2, 2, 3), *rng_.uniform(-np.pi, np.pi, 3))
                          for _ in range(3)])
        dirs, n_az = synth.lidar_pattern(9, -60.0, 60.0, 71), 71
    log(f"unbounded range closed={closed}")
    (r32, h32), (rq, hq) = _cast_both(ctx, v, t, poses, dirs, 0.0, np.inf, n_az)
    assert np.array_equal(h32, hq) and np.array_equal(r32.view(np.int32), rq.view(np.int32))
    stats = compare_with_oracle(v, t, poses, dirs, 0.0, np.inf, rq, hq)
    if closed:
        assert stats["hits"] == stats["rays"]
        (rb, hb), _ = _cast_both(ctx, v, t, poses, dirs, 0.0, 1e6, n_az)
        assert np.array_equal(hb, hq) and np.array_equal(rb.view(np.int32), rq.view(np.int32))
    else:
        assert 0 < stats["hits"] < stats["rays"]
        assert np.all(np.isinf(rq[hq < 0]))


def test_q8_equals_fp32_indoor_1m(ctx):
    s = synth.indoor_scene(seed=1, h=0.035, n_envs=8)
    log(f"q8 indoor 1M tris={len(s.tris)}")
    (r32, h32), (rq, hq) = _cast_both(ctx, s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                      s.n_az)
    assert np.all(hq >= 0)
    same = (h32 == hq) & (r32.view(np.int32) == rq.view(np.int32))
    assert same.all(), np.flatnonzero(~same)[:10]
    idx = np.sort(np.random.default_rng(7).choice(s.n_rays, 1024, replace=False))
    st = compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, rq, hq,
                             ray_idx=idx)
    log(str(st))


def test_q8_tuning_variants_bit_identical(ctx):
    import torch
    s = synth.indoor_scene(seed=3, h=0.1, n_envs=6, n_az=256)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=1)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    job = [Job(scene, pat, cuda(s.poses), s.t_min, s.t_max)]
    idx, orc = _variant_sample(s, seed=12)
    ref = None
    try:
        for tn in TUNINGS:
            log(f"q8 tuning {tn}")
            ctx.set_tuning(**tn)
            r, h = ctx.cast(job)
            r2, h2, nn, nt = ctx.cast(job, mode="stats")
            torch.cuda.synchronize()
            assert torch.equal(h, h2) and torch.equal(r.view(torch.int32), r2.view(torch.int32))
            assert int(nn.min()) >= 1
            compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max,
                                r.cpu().numpy(), h.cpu().numpy(), ray_idx=idx, oracle_out=orc)
            if ref is None:
                ref = (r.clone(), h.clone())
            else:
                assert torch.equal(h, ref[1])
                assert torch.equal(r.view(torch.int32), ref[0].view(torch.int32))
    finally:
        ctx.reset_tuning()


@pytest.mark.parametrize("leaf_batch", [1, 32, 64])
def test_q8_leaf_batch_waves_across_scenes(ctx, leaf_batch):
    # queued leaf tests: a wave whose lanes belong to different jobs (other
    # scene, pattern, range) tests each queued pair against its own lane's
    # scene and ray; results equal each job cast alone with on-the-spot tests
    import torch
    a = synth.room_sphere_scene(6)
    sdf = synth.indoor_sdf(4, n_prims=30)
    bv, bt = synth.polygonise(sdf, 0.12)
    bposes = synth.free_space_poses(sdf, 3, 5)
    sa = ctx.upload_scene(a.verts, a.tris)
    sb = ctx.upload_scene(bv, bt)
    ctx.build(sa, node_format=1)
    ctx.build(sb, node_format=1)
    dirs = synth.lidar_pattern(7, -20, 10, 45)          # 315 beams: waves straddle jobs
    pat = ctx.upload_pattern(dirs, 45)
    jobs = [Job(sa, pat, cuda(a.poses), 0.0, 100.0, 0),
            Job(sb, pat, cuda(bposes), 0.1, 120.0, 315),
            Job(sa, pat, cuda(a.poses), 0.5, 4.0, 315 * 4),
            Job(sb, pat, cuda(bposes[:1]), 0.1, 2.5, 315 * 5)]
    try:
        singles = []
        for j in jobs:
            singles.append(ctx.cast([Job(j.scene, j.pattern, j.poses, j.t_min, j.t_max, 0)]))
        ctx.set_tuning(leaf_batch=leaf_batch, tile_az=0, tile_el=0)
        log(f"leaf_batch {leaf_batch}: straddling batch")
        r_all, h_all = ctx.cast(jobs)
        torch.cuda.synchronize()
        for j, (r1, h1) in zip(jobs, singles):
            n = j.n_envs * 315
            sl = slice(j.out_offset, j.out_offset + n)
            assert torch.equal(h_all[sl], h1) and torch.equal(r_all[sl].view(torch.int32),
                                                              r1.view(torch.int32))
        pb = bposes[:1]
        compare_with_oracle(bv, bt, pb, dirs, 0.1, 2.5, r_all[315 * 5:].cpu().numpy(),
                            h_all[315 * 5:].cpu().numpy())
    finally:
        ctx.reset_tuning()


def test_autotune_keeps_results_and_sets_tuning(ctx):
    import torch
    s = synth.indoor_scene(seed=4, h=0.1, n_envs=16, n_az=256)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=1)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    job = [Job(scene, pat, cuda(s.poses), s.t_min, s.t_max)]
    try:
        ref_r, ref_h = ctx.cast(job)
        r = torch.full_like(ref_r, -1.0)
        h = torch.full_like(ref_h, -7)
        log("autotune")
        best, ms = ctx.autotune(job, r, h, reps=1)
        torch.cuda.synchronize()
        assert ms > 0 and ctx.get_tuning() == best
        assert torch.equal(h, ref_h) and torch.equal(r.view(torch.int32), ref_r.view(torch.int32))
    finally:
        ctx.reset_tuning()


def test_autotune_cache_persists_across_contexts(tmp_path):
    # a context with a loaded (empty) cache tunes and stores the result; a
    # second context loading the saved file gets the same tuning without
    # launching (ms = -1, outputs untouched); a different batch size class
    # misses and is tuned again
    import torch
    s = synth.indoor_scene(seed=4, h=0.1, n_envs=16, n_az=256)
    path = str(tmp_path / "tuning.txt")
    got = []
    for k in range(2):
        c = Context(0)
        try:
            c.tuning_cache_load(path)
            scene = c.upload_scene(s.verts, s.tris)
            c.build(scene, node_format=1)
            pat = c.upload_pattern(s.dirs, s.n_az)
            job = [Job(scene, pat, cuda(s.poses), s.t_min, s.t_max)]
            n = len(s.poses) * len(s.dirs)
            r = torch.full((n,), -1.0, device="cuda")
            h = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            best, ms = c.autotune(job, r, h, reps=1)
            torch.cuda.synchronize()
            got.append((best, ms, bool((h == -7).all())))
            assert c.get_tuning() == best
            if k == 1:
                job1 = [Job(scene, pat, cuda(s.poses[:1]), s.t_min, s.t_max)]
                _, ms1 = c.autotune(job1, r, h, reps=1)
                assert ms1 > 0
            c.tuning_cache_save(path)
        finally:
            c.close()
    (b0, ms0, untouched0), (b1, ms1, untouched1) = got
    assert ms0 > 0 and not untouched0
    assert ms1 == -1.0 and untouched1 and b1 == b0
    lines = open(path).read().splitlines()
    assert lines[0] == "rcast-tuning-cache v2" and len(lines) == 3


@pytest.mark.parametrize("fmt,persistent", [(0, 0), (1, 0), (1, 1)])
def test_graph_replays_match_eager(ctx, fmt, persistent):
    # capture once, move the sensors between replays (eager torch work and a
    # sync in between), and check every replay against an eager launch
    import torch
    s = synth.indoor_scene(seed=6, h=0.1, n_envs=12, n_az=256)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=fmt)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    poses = cuda(s.poses)
    n = s.n_rays
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    h = torch.empty(n, dtype=torch.int32, device="cuda")
    try:
        if persistent:
            ctx.set_tuning(persistent=1, stack_lds=8, refill_min=48, blocks_per_cu=2,
                           chunk_max=1024, waves_cap=0)
        job = [Job(scene, pat, poses, s.t_min, s.t_max)]
        g = ctx.graph(job, r, h)
        sdf = s.meta["sdf"]
        for rep in range(4):
            newp = synth.free_space_poses(sdf, len(s.poses), 50 + rep)
            poses.copy_(torch.from_numpy(newp).cuda())
            torch.cuda.synchronize()
            log(f"graph replay {rep} fmt={fmt} persistent={persistent}")
            g.launch()
            torch.cuda.synchronize()
            er, eh = ctx.cast(job)
            torch.cuda.synchronize()
            assert torch.equal(h, eh) and torch.equal(r.view(torch.int32), er.view(torch.int32))
            assert bool((h >= 0).all())
        g.close()
    finally:
        ctx.reset_tuning()


def test_uneven_multi_scene_batch(ctx):
    # several resident terrains, environments bound to random scenes and to
    # three beam patterns, all in one launch: equal to each job cast alone,
    # and to the oracle on a sample of every job's rays
    import torch
    w = synth.uneven_world(seed=3, n_scenes=5, n_envs=20, tri_lo=20_000, tri_hi=150_000)
    sids = [ctx.upload_scene(v, t) for v, t in w.scenes]
    for k, sid in enumerate(sids):
        ctx.build(sid, node_format=k % 2)   # FP32 and Q8 scenes in one launch
    pids = [ctx.upload_pattern(d, na) for d, na in zip(w.patterns, w.n_az)]
    jobs, meta, off = [], [], 0
    for k in range(len(sids)):
        for pi in range(len(pids)):
            idx = np.flatnonzero((w.env_scene == k) & (w.env_pattern == pi))
            if len(idx):
                jobs.append(Job(sids[k], pids[pi], cuda(w.poses[idx]), w.t_min, w.t_max, off))
                meta.append((k, pi, idx))
                off += len(idx) * len(w.patterns[pi])
    log(f"uneven batch: {len(jobs)} jobs, {off} rays")
    r_all, h_all = ctx.cast(jobs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for j, (k, pi, idx) in zip(jobs, meta):
        n = len(idx) * len(w.patterns[pi])
        r1, h1 = ctx.cast([Job(j.scene, j.pattern, j.poses, j.t_min, j.t_max, 0)])
        sl = slice(j.out_offset, j.out_offset + n)
        assert torch.equal(h_all[sl], h1) and torch.equal(r_all[sl].view(torch.int32),
                                                          r1.view(torch.int32))
        v, t = w.scenes[k]
        sample = np.sort(rng.choice(n, min(n, 150), replace=False))
        compare_with_oracle(v, t, w.poses[idx], w.patterns[pi], w.t_min, w.t_max,
                            r1.cpu().numpy(), h1.cpu().numpy(), ray_idx=sample,
                            min_checked_frac=0.9)


def test_large_terrain_sampled_parity(ctx):
    # a 2.5M-triangle terrain (heightfield + boxes sunk into the ground, so
    # interpenetrating surfaces give ambiguous rays), 32 poses x 64 x 1024
    # beams in one launch, both node formats; the oracle checks a seeded
    # sample with its checker flags
    import torch
    v, t, height, boxes = synth.terrain_scene(77, 2_500_000)
    assert len(t) >= 2_000_000
    poses = synth.terrain_poses(height, boxes, 32, 78)
    dirs = synth.lidar_pattern(64, -25.0, 3.0, 1024)
    n_rays = len(poses) * len(dirs)
    log(f"terrain tris={len(t)} rays={n_rays}")
    scene = ctx.upload_scene(v, t)
    pat = ctx.upload_pattern(dirs, 1024)
    out = {}
    for fmt in (0, 1):
        ctx.build(scene, node_format=fmt)
        r, h = ctx.cast([Job(scene, pat, cuda(poses), 0.1, 120.0, 0)])
        torch.cuda.synchronize()
        out[fmt] = (r.cpu().numpy(), h.cpu().numpy())
    (r32, h32), (rq, hq) = out[0], out[1]
    assert np.array_equal(h32, hq) and np.array_equal(r32.view(np.int32), rq.view(np.int32))
    idx = np.sort(np.random.default_rng(5).choice(n_rays, 384, replace=False))
    st = compare_with_oracle(v, t, poses, dirs, 0.1, 120.0, rq, hq, ray_idx=idx,
                             min_checked_frac=0.9)
    log(str(st))


def test_indoor_2cm_sampled_parity(ctx):
    # the indoor mesh polygonised at 2 cm as written (3.39M triangles), 8
    # poses x 32 x 1024 beams, Q8 nodes; seeded oracle sample
    s = synth.indoor_scene(seed=1, h=0.02, n_envs=8)
    assert len(s.tris) > 3_000_000
    log(f"indoor 2 cm tris={len(s.tris)} rays={s.n_rays}")
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=1)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    r, h = ctx.cast([Job(scene, pat, cuda(s.poses), s.t_min, s.t_max, 0)])
    r, h = r.cpu().numpy(), h.cpu().numpy()
    assert np.all(h >= 0)   # closed mesh, poses in free space
    idx = np.sort(np.random.default_rng(9).choice(s.n_rays, 384, replace=False))
    st = compare_with_oracle(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, r, h,
                             ray_idx=idx)
    log(str(st))


def test_batch_larger_than_one_dispatch(ctx):
    # 3 jobs x 1.5e9 rays = 4.5e9 rays in one call: more work-items than one
    # dispatch can hold, so the library splits the launch; every ray must be
    # written.  A single triangle keeps the traversal trivial.
    import torch
    tri = np.array([[5, -50, -50], [5, 50, -50], [5, 0, 50]], np.float32)
    s1 = ctx.upload_scene(tri, np.array([[0, 1, 2]], np.int32))
    ctx.build(s1)
    nb = 1 << 15
    az = np.linspace(-0.5, 0.5, nb)
    dirs = np.stack([np.cos(az), np.sin(az), np.zeros(nb)], -1).astype(np.float32)
    pat = ctx.upload_pattern(dirs, nb)
    envs = 45_776          # x 32768 beams = 1.5e9 rays per job
    pose = cuda(np.repeat(synth.yaw_pose((0, 0, 0), 0.0)[None], envs, 0))
    per = envs * nb
    total = 3 * per
    assert total > 2 ** 32
    r = torch.full((total,), -1.0, dtype=torch.float32, device="cuda")
    h = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    jobs = [Job(s1, pat, pose, 0.0, 100.0, k * per) for k in range(3)]
    log(f"batch of {total} rays")
    ctx.raycast(jobs, r, h)
    torch.cuda.synchronize()
    assert bool((h == 0).all())
    exp = torch.from_numpy((5.0 / np.cos(az)).astype(np.float32)).cuda()
    last = r[-nb:]
    assert float((last - exp).abs().max()) < 1e-4
    del r, h
    torch.cuda.empty_cache()
    ctx.release_scene(s1)


def test_graph_keeps_its_scene_after_release(ctx):
    """A captured graph holds its scene: released after capture, the scene
    still serves every replay, and its memory returns when the graph goes."""
    import torch
    s = synth.indoor_scene(seed=8, h=0.1, n_envs=8, n_az=256)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=1)
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    poses = cuda(s.poses)
    job = [Job(scene, pat, poses, s.t_min, s.t_max)]
    ref_r, ref_h = ctx.cast(job)
    r = torch.empty_like(ref_r)
    h = torch.empty_like(ref_h)
    g = ctx.graph(job, r, h)
    torch.cuda.synchronize()
    held = ctx.device_bytes()
    ctx.release_scene(scene)
    assert ctx.device_bytes() == held          # still referenced by the graph
    with pytest.raises(RcastError):
        ctx.cast(job)
    for rep in range(3):
        r.fill_(-1.0)
        h.fill_(-7)
        torch.cuda.synchronize()
        log(f"graph replay after release {rep}")
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(h, ref_h) and torch.equal(r.view(torch.int32), ref_r.view(torch.int32))
    g.close()
    assert ctx.device_bytes() < held           # freed with the graph
