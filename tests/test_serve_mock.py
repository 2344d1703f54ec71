"""Serving scheduler on the mock device (no GPU): admission by footprint,
continuous batching, ticket life cycle, failure isolation, concurrency.

The mock device runs the library's real scheduler; only the launch is
simulated (host thread, time proportional to rays) and writes
range = ray index within the request, hit = scene id.
"""
import threading
import time

import numpy as np
import pytest

from paper_2509_17390_amd import Context, RcastError
from paper_2509_17390_amd.rcast import RC_DEVICE_MOCK, RC_OK, RC_PENDING

pytestmark = pytest.mark.timeout(120)


def mock_ctx():
    c = Context(RC_DEVICE_MOCK)
    v = np.zeros((3, 3), np.float32)
    v[1, 0] = 1
    v[2, 1] = 1
    t = np.array([[0, 1, 2]], np.int32)
    scenes = [c.upload_scene(v, t) for _ in range(3)]
    for s in scenes:
        c.build(s)
    pats = [c.upload_pattern(np.tile([[1, 0, 0]], (n, 1)).astype(np.float32), 0)
            for n in (100, 1000, 5000)]
    return c, scenes, pats


def poses(n, seed=0):
    rng = np.random.default_rng(seed)
    p = np.zeros((n, 12), np.float32)
    p[:, [0, 5, 10]] = 1.0
    p[:, [3, 7, 11]] = rng.uniform(-1, 1, (n, 3))
    return p


def wait(c, tk, timeout_s=20.0):
    st, lat = c.poll(tk, int(timeout_s * 1e6))
    return st, lat


def test_basic_lifecycle_and_results():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=64 << 20, max_inflight=2)
    reqs = []
    for i in range(12):
        s, p = scenes[i % 2], pats[i % 3]
        n_envs = 1 + i
        tk = c.submit(s, p, poses(n_envs, i), 0.0, 10.0)
        reqs.append((tk, s, n_envs * (100, 1000, 5000)[i % 3]))
    for tk, s, n in reqs:
        st, lat = wait(c, tk)
        assert st == RC_OK and lat >= 0.0
        rng, hit = c.fetch(tk, n)
        assert np.array_equal(rng, np.arange(n, dtype=np.float32))   # its own slice
        assert np.all(hit == s)
        c.release(tk)
    stats = c.serve_stats()
    assert stats["submitted"] == stats["completed"] == 12
    assert stats["bytes_in_use"] == 0 and stats["pending"] == 0
    with pytest.raises(RcastError):
        c.release(reqs[0][0])          # already released
    c.serve_stop()
    c.close()


def test_admission_respects_arena_and_batches():
    c, scenes, pats = mock_ctx()
    arena = 2 << 20                       # outputs: (2 MiB - 256 KiB) / 8 = 229,376 rays
    c.serve_start(arena_bytes=arena, max_inflight=2, mock_ns_per_ray=200)
    tks = [c.submit(scenes[0], pats[1], poses(40), 0.0, 1.0) for _ in range(20)]  # 40k rays each
    done = 0
    peak_seen = 0
    while done < len(tks):
        for tk in list(tks):
            st, _ = c.poll(tk, 0)
            if st == RC_OK:
                c.release(tk)
                tks.remove(tk)
                done += 1
        s = c.serve_stats()
        peak_seen = max(peak_seen, s["bytes_in_use"])
        time.sleep(0.001)
    s = c.serve_stats()
    assert s["peak_bytes"] <= arena and peak_seen <= arena
    assert s["max_batch_requests"] >= 2     # several requests shared a launch
    assert s["launches"] < 20
    c.serve_stop()
    c.close()


def test_oversize_request_rejected_at_submit():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=1 << 20)
    with pytest.raises(RcastError) as e:
        c.submit(scenes[0], pats[2], poses(100), 0.0, 1.0)   # 500k rays > capacity
    assert e.value.status == -2
    assert c.serve_stats()["rejected"] == 1
    c.serve_stop()
    c.close()


def test_poll_pending_release_busy_and_cancel():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=8 << 20, max_inflight=1, mock_ns_per_ray=2000)
    long_tk = c.submit(scenes[0], pats[1], poses(100), 0.0, 1.0)      # 100k rays: 0.2 s
    time.sleep(0.03)                        # launched alone: the only slot is taken
    queued = c.submit(scenes[1], pats[0], poses(1), 0.0, 1.0)
    time.sleep(0.02)
    st, _ = c.poll(long_tk, 0)
    assert st == RC_PENDING
    with pytest.raises(RcastError) as e:
        c.release(long_tk)                  # on the device
    assert e.value.status == -4
    c.release(queued)                       # still queued: cancelled
    assert c.serve_stats()["cancelled"] == 1
    assert c.poll(queued, 0)[0] == -3       # unknown ticket now
    st, _ = wait(c, long_tk)
    assert st == RC_OK
    c.release(long_tk)
    c.serve_stop()
    c.close()


def test_failure_isolated_to_its_requests():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=64 << 20, max_inflight=1, mock_ns_per_ray=1000,
                  mock_fail_scene=scenes[1] + 1)
    block = c.submit(scenes[0], pats[1], poses(40), 0.0, 1.0)   # 40k rays: 40 ms
    time.sleep(0.005)                       # block runs alone; the rest queue behind it
    mixed = [c.submit(scenes[i % 2], pats[0], poses(3), 0.0, 1.0) for i in range(6)]
    assert wait(c, block)[0] == RC_OK
    for i, tk in enumerate(mixed):
        st, _ = wait(c, tk)
        if i % 2 == 1:
            assert st == -5                 # the simulated device error
        else:
            assert st == RC_OK
            rng, hit = c.fetch(tk, 300)
            assert np.all(hit == scenes[0])
    s = c.serve_stats()
    assert s["failed"] == 3 and s["completed"] == 4
    assert s["max_batch_requests"] >= 2     # failures shared launches with successes
    c.serve_stop()
    c.close()


def test_continuous_batching_overlaps_small_with_large():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=64 << 20, max_inflight=2, mock_ns_per_ray=1000)
    big = c.submit(scenes[0], pats[2], poses(60), 0.0, 1.0)     # 300k rays: 0.3 s
    time.sleep(0.02)
    small = [c.submit(scenes[1], pats[0], poses(1), 0.0, 1.0) for _ in range(5)]
    for tk in small:
        assert wait(c, tk)[0] == RC_OK
    st, _ = c.poll(big, 0)
    assert st == RC_PENDING                 # the small ones did not wait for it
    assert c.serve_stats()["peak_inflight"] == 2
    assert wait(c, big)[0] == RC_OK
    c.serve_stop()
    c.close()


def test_batch_cap_splits_launches_and_runs_large_requests_alone():
    c, scenes, pats = mock_ctx()
    # 1M rays per launch at most; requests of 400k rays (two fit) and one of
    # 3M rays (above the cap: runs alone)
    c.serve_start(arena_bytes=256 << 20, max_inflight=1, max_batch_rays_m=1,
                  mock_ns_per_ray=20)
    block = c.submit(scenes[0], pats[1], poses(100), 0.0, 1.0)   # 100k rays, holds the slot
    time.sleep(0.005)
    small = [c.submit(scenes[1], pats[1], poses(400), 0.0, 1.0) for _ in range(6)]
    big = c.submit(scenes[2], pats[2], poses(600), 0.0, 1.0)     # 3M rays
    for tk in [block] + small + [big]:
        assert wait(c, tk)[0] == RC_OK
    s = c.serve_stats()
    assert s["max_batch_requests"] == 2      # never more than the cap allows
    assert s["launches"] >= 1 + 3 + 1
    rng, hit = c.fetch(big, 3_000_000)
    assert np.array_equal(rng[:10], np.arange(10, dtype=np.float32)) and np.all(hit == scenes[2])
    c.serve_stop()
    c.close()


def _completion_order(c, tickets, timeout_s=20.0):
    done = {}
    t0 = time.perf_counter()
    while len(done) < len(tickets) and time.perf_counter() - t0 < timeout_s:
        for tk in tickets:
            if tk not in done and c.poll(tk, 0)[0] == RC_OK:
                done[tk] = time.perf_counter()
                c.release(tk)            # results hold arena memory until released
        time.sleep(0.0005)
    assert len(done) == len(tickets)
    return done


@pytest.mark.parametrize("policy,max_wait_ms,small_first", [(0, 0, False), (1, 10_000, True),
                                                           (1, 20, False)])
def test_admission_policy(policy, max_wait_ms, small_first):
    """A 200k-ray request queued ahead of five 10k-ray ones while a 100k-ray
    launch holds the only slot; the arena takes 229k rays.  Arrival order
    runs the large one first; small-first runs the small ones first unless
    the large one has already waited max_wait_ms."""
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=2 << 20, max_inflight=1, mock_ns_per_ray=1000,
                  policy=policy, max_wait_ms=max_wait_ms)
    block = c.submit(scenes[0], pats[1], poses(100), 0.0, 1.0)   # 100k rays: 0.1 s
    time.sleep(0.01)
    big = c.submit(scenes[1], pats[2], poses(40), 0.0, 1.0)      # 200k rays
    time.sleep(0.05)                                             # big ages 50 ms
    small = [c.submit(scenes[2], pats[1], poses(10), 0.0, 1.0) for _ in range(5)]
    done = _completion_order(c, [block, big] + small)
    last_small = max(done[tk] for tk in small)
    if small_first:
        assert last_small < done[big]
    else:
        assert done[big] <= last_small
    c.serve_stop()
    c.close()


def test_bad_policy_rejected():
    c, scenes, pats = mock_ctx()
    with pytest.raises(RcastError):
        c.serve_start(policy=2)
    with pytest.raises(RcastError):
        c.serve_start(policy=1, max_wait_ms=-1)
    c.close()


def test_concurrent_submitters():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=64 << 20, max_inflight=3, mock_ns_per_ray=5)
    got = []
    lock = threading.Lock()

    def worker(k):
        mine = []
        for i in range(25):
            n_envs = 1 + (i + k) % 4
            tk = c.submit(scenes[k % 3], pats[i % 2], poses(n_envs, k * 100 + i), 0.0, 1.0)
            mine.append((tk, scenes[k % 3], n_envs * (100, 1000)[i % 2]))
        for tk, s, n in mine:
            assert wait(c, tk)[0] == RC_OK
            rng, hit = c.fetch(tk, n)
            assert np.array_equal(rng, np.arange(n, dtype=np.float32)) and np.all(hit == s)
            c.release(tk)
        with lock:
            got.extend(t for t, _, _ in mine)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(set(got)) == 100
    s = c.serve_stats()
    assert s["completed"] == 100 and s["bytes_in_use"] == 0
    c.serve_stop()
    c.close()


def test_released_scene_fails_its_queued_requests():
    c, scenes, pats = mock_ctx()
    c.serve_start(arena_bytes=64 << 20, max_inflight=1, mock_ns_per_ray=1000)
    block = c.submit(scenes[0], pats[1], poses(50), 0.0, 1.0)    # holds the only slot
    time.sleep(0.01)
    doomed = c.submit(scenes[2], pats[0], poses(2), 0.0, 1.0)
    ok = c.submit(scenes[0], pats[0], poses(2), 0.0, 1.0)
    c.release_scene(scenes[2])
    assert wait(c, block)[0] == RC_OK
    assert wait(c, doomed)[0] == -3
    assert wait(c, ok)[0] == RC_OK
    c.serve_stop()
    c.close()


def test_mock_context_rules():
    c, scenes, pats = mock_ctx()
    with pytest.raises(RcastError) as e:
        c.serve_stop()                       # not running
    assert e.value.status == -6
    with pytest.raises(RcastError):
        c.serve_start(max_inflight=9)
    c.serve_start()
    with pytest.raises(RcastError):
        c.serve_start()                      # already running
    with pytest.raises(RcastError):
        c.submit(99, pats[0], poses(1), 0.0, 1.0)
    with pytest.raises(RcastError):
        c.submit(scenes[0], pats[0], poses(1), 2.0, 1.0)
    bad = poses(1)
    bad[0, 3] = np.nan
    with pytest.raises(RcastError):
        c.submit(scenes[0], pats[0], bad, 0.0, 1.0)
    # stop with work queued: returns, and tickets are gone afterwards
    tks = [c.submit(scenes[0], pats[1], poses(5), 0.0, 1.0) for _ in range(4)]
    c.serve_stop()
    assert c.poll(tks[0], 0)[0] == -6        # server gone
    c.close()


# ---------------------------------------------------------------------------
# Scene release while in use: the handle dies at once, the memory (a host
# copy of the vertices that the simulated device reads during the launch)
# is freed only after the last batch using it has finished.

def _mock_scene(c, n_verts=4000, seed=3):
    rng = np.random.default_rng(seed)
    v = rng.uniform(-5, 5, (n_verts, 3)).astype(np.float32)
    t = np.arange(3 * (n_verts // 3), dtype=np.int32).reshape(-1, 3)
    s = c.upload_scene(v, t)
    c.build(s)
    return s, 12 * n_verts


def _wait_inflight(c, n=1, timeout_s=5.0):
    t0 = time.perf_counter()
    while c.serve_stats()["inflight"] < n:
        assert time.perf_counter() - t0 < timeout_s
        time.sleep(0.0005)


def test_release_while_running_defers_the_free():
    c, scenes, pats = mock_ctx()
    base = c.device_bytes()
    s, nbytes = _mock_scene(c)
    assert c.device_bytes() == base + nbytes
    c.serve_start(arena_bytes=64 << 20, max_inflight=1, mock_ns_per_ray=2000)
    tk = c.submit(s, pats[1], poses(100), 0.0, 1.0)              # 100k rays: 0.2 s
    _wait_inflight(c)
    time.sleep(0.01)
    c.release_scene(s)                                           # returns at once
    with pytest.raises(RcastError) as e:
        c.scene_info(s)
    assert e.value.status == -3
    with pytest.raises(RcastError) as e:
        c.submit(s, pats[0], poses(1), 0.0, 1.0)
    assert e.value.status == -3
    with pytest.raises(RcastError) as e:
        c.release_scene(s)                                       # already released
    assert e.value.status == -3
    assert c.device_bytes() == base + nbytes                     # still in use
    s2, nbytes2 = _mock_scene(c, 30, seed=4)
    assert s2 != s                                               # the slot is not reused yet
    st, _ = wait(c, tk)
    assert st == RC_OK                                           # the scene stayed intact
    rng, hit = c.fetch(tk, 100_000)
    assert np.array_equal(rng, np.arange(100_000, dtype=np.float32)) and np.all(hit == s)
    assert c.device_bytes() == base + nbytes2                    # freed after the batch
    c.release(tk)
    c.serve_stop()
    c.release_scene(s2)
    assert c.device_bytes() == base
    c.close()


def test_release_between_resolution_and_launch():
    """The release lands in the window after the batch has resolved (and
    referenced) its scene but before the launch is issued."""
    c, scenes, pats = mock_ctx()
    base = c.device_bytes()
    s, nbytes = _mock_scene(c)
    c.serve_start(arena_bytes=64 << 20, max_inflight=1, mock_ns_per_ray=0,
                  mock_launch_delay_us=300_000)
    tk = c.submit(s, pats[0], poses(3), 0.0, 1.0)
    _wait_inflight(c)
    time.sleep(0.05)                                             # inside the 0.3 s window
    c.release_scene(s)
    assert c.device_bytes() == base + nbytes
    st, _ = wait(c, tk)
    assert st == RC_OK
    rng, hit = c.fetch(tk, 300)
    assert np.array_equal(rng, np.arange(300, dtype=np.float32)) and np.all(hit == s)
    assert c.device_bytes() == base
    c.release(tk)
    c.serve_stop()
    c.close()


def test_release_of_an_idle_scene_frees_at_once_and_reuses_the_slot():
    c, scenes, pats = mock_ctx()
    base = c.device_bytes()
    s, nbytes = _mock_scene(c)
    assert c.device_bytes() == base + nbytes
    c.release_scene(s)
    assert c.device_bytes() == base
    s2, _ = _mock_scene(c, 60)
    assert s2 == s                                               # the freed slot comes back
    c.close()


def test_released_scene_shared_by_running_and_queued_requests():
    """One batch of a scene runs while another request on it is queued: the
    release fails the queued one, the running one completes, and the memory
    goes once the running batch has finished."""
    c, scenes, pats = mock_ctx()
    base = c.device_bytes()
    s, nbytes = _mock_scene(c)
    c.serve_start(arena_bytes=64 << 20, max_inflight=1, mock_ns_per_ray=2000)
    running = c.submit(s, pats[1], poses(60), 0.0, 1.0)         # 60k rays: 0.12 s
    _wait_inflight(c)
    queued = c.submit(s, pats[0], poses(2), 0.0, 1.0)
    c.release_scene(s)
    assert wait(c, running)[0] == RC_OK
    assert wait(c, queued)[0] == -3
    assert c.device_bytes() == base
    c.serve_stop()
    c.close()


def test_budget_counts_mock_scenes():
    c = Context(RC_DEVICE_MOCK, budget_bytes=100_000)
    v = np.zeros((6000, 3), np.float32)
    t = np.arange(18000, dtype=np.int32).reshape(-1, 3) % 6000
    a = c.upload_scene(v, t)                                     # 72 kB
    with pytest.raises(RcastError) as e:
        c.upload_scene(v, t)                                     # would exceed 100 kB
    assert e.value.status == -2
    c.release_scene(a)
    b = c.upload_scene(v, t)                                     # fits again
    assert b == a
    c.close()
