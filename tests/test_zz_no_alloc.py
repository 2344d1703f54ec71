"""rc_raycast_batch_noalloc -- the launch entry point that allocates
nothing -- against rc_raycast_batch, through the C ABI: bit-identical
outputs on two calls in a row on one stream (the second with a smaller
batch), with job tables that take several fill launches, in the grid and the
persistent launch shapes and in both node formats; more than 256 jobs are
refused; the context's device memory does not change."""
import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from paper_2509_17390_amd import Context, Job, RcastError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    ctx = Context(0)
    a = synth.indoor_scene(seed=5, h=0.1, n_envs=16, n_az=256)
    b = synth.room_sphere_scene(3)
    scenes = {}
    for fmt in (0, 1):
        sa = ctx.upload_scene(a.verts, a.tris)
        ctx.build(sa, node_format=fmt)
        sb = ctx.upload_scene(b.verts, b.tris)
        ctx.build(sb, node_format=fmt)
        scenes[fmt] = (sa, sb)
    pats = [(ctx.upload_pattern(a.dirs, a.n_az), len(a.dirs)),
            (ctx.upload_pattern(b.dirs, b.n_az), len(b.dirs)),
            (ctx.upload_pattern(synth.lidar_pattern(5, -10, 10, 37), 37), 185)]
    pool = {0: cuda(a.poses), 1: cuda(np.repeat(b.poses, 16, 0))}
    yield ctx, scenes, pats, pool
    ctx.close()


def make_jobs(scenes, pats, pool, n_jobs, seed):
    rng = np.random.default_rng(seed)
    jobs, off = [], 0
    for i in range(n_jobs):
        k = int(rng.integers(2))
        p, nb = pats[int(rng.integers(len(pats)))]
        envs = int(rng.integers(1, 7))
        e0 = int(rng.integers(0, 16 - envs + 1))
        jobs.append(Job(scenes[k], p, pool[k][e0:e0 + envs].contiguous(),
                        float(rng.choice([0.0, 0.1])), float(rng.choice([20.0, 120.0])), off))
        off += envs * nb + int(rng.integers(0, 5))   # gaps between slices
    return jobs, off


def cast_pair(ctx, jobs, n, stream):
    import torch
    r0 = torch.full((n,), -3.0, dtype=torch.float32, device="cuda")
    h0 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    r1, h1 = r0.clone(), h0.clone()
    ctx.raycast(jobs, r0, h0, stream=stream)
    return (r0, h0), (r1, h1)


@pytest.mark.parametrize("fmt,persistent", [(1, 0), (0, 0), (1, 1)])
def test_noalloc_matches_batch_on_two_calls(world, fmt, persistent):
    import torch
    ctx, scenes, pats, pool = world
    stream = torch.cuda.current_stream()
    try:
        if persistent:
            ctx.set_tuning(persistent=1, stack_lds=8, refill_min=48, blocks_per_cu=2,
                           chunk_max=1024, waves_cap=0)
        big, n_big = make_jobs(scenes[fmt], pats, pool, 40, 10 + fmt + 2 * persistent)
        small, n_small = make_jobs(scenes[fmt], pats, pool, 5, 20 + fmt + 2 * persistent)
        ref_big, out_big = cast_pair(ctx, big, n_big, stream)
        ref_small, out_small = cast_pair(ctx, small, n_small, stream)
        torch.cuda.synchronize()
        before = ctx.device_bytes()
        log(f"noalloc fmt={fmt} persistent={persistent}: {len(big)} jobs / {n_big} rays, "
            f"then {len(small)} jobs / {n_small} rays")
        # two calls in a row on one stream, the second smaller
        ctx.raycast(big, *out_big, stream=stream, mode="noalloc")
        ctx.raycast(small, *out_small, stream=stream, mode="noalloc")
        torch.cuda.synchronize()
        for (rr, hh), (r, h) in ((ref_big, out_big), (ref_small, out_small)):
            assert torch.equal(h, hh)
            assert torch.equal(r.view(torch.int32), rr.view(torch.int32))
        assert bool((ref_big[1] >= -1).any())
        assert ctx.device_bytes() == before
    finally:
        ctx.reset_tuning()


def test_noalloc_refuses_more_than_256_jobs(world):
    import torch
    ctx, scenes, pats, pool = world
    jobs, n = make_jobs(scenes[1], pats, pool, 257, 3)
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    h = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(RcastError) as e:
        ctx.raycast(jobs, r, h, mode="noalloc")
    assert e.value.status == -1 and "256" in str(e.value)
    ok, n_ok = make_jobs(scenes[1], pats, pool, 256, 4)   # the maximum is accepted
    stream = torch.cuda.current_stream()
    (rr, hh), (r, h) = cast_pair(ctx, ok, n_ok, stream)
    ctx.raycast(ok, r, h, stream=stream, mode="noalloc")
    torch.cuda.synchronize()
    assert torch.equal(h, hh) and torch.equal(r.view(torch.int32), rr.view(torch.int32))
