"""The GPU parity checker (tests/gpu_util.py) on the CPU: it accepts the
oracle's own answers and rejects planted wrong answers on rays with several
correct answers -- a hit behind the nearest surface (a ray that slipped
through a shared edge), a miss where the oracle hits, and a triangle the ray
does not hit."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_flagged, compare_with_oracle


@pytest.fixture(scope="module")
def doubled_room():
    # every face twice: each hit has an exact duplicate, so every ray is
    # flagged ambiguous; the box's diagonals and corners give edge-near rays
    v, t = synth.box_room()
    t2 = np.concatenate([t, t]).astype(np.int32)
    poses = np.stack([synth.yaw_pose((5, 4, 1.5), 0.0), synth.yaw_pose((2, 6, 1.0), 2.0)])
    # beams from the first pose at the room's corners and at a face's
    # diagonal (edge-near), then a regular pattern
    aim = np.array([[10, 8, 3], [0, 0, 0], [10, 0, 3], [10, 6, 2.25]], np.float64) - (5, 4, 1.5)
    dirs = np.concatenate([aim.astype(np.float32), synth.lidar_pattern(8, -60, 60, 90)])
    out = oracle.raycast(v, t2, poses, dirs, 0.0, 100.0, checked=True)
    return v, t2, poses, dirs, out


def _gpu_like(out):
    t, ids = out[0], out[1]
    return t.astype(np.float32), ids.copy()


def test_accepts_the_oracles_answer(doubled_room):
    v, t, poses, dirs, out = doubled_room
    assert np.all(out[2] != 0)                      # all flagged
    g_r, g_h = _gpu_like(out)
    st = compare_with_oracle(v, t, poses, dirs, 0.0, 100.0, g_r, g_h, oracle_out=out,
                             min_checked_frac=0.0)
    assert st["flagged_checked"] == len(g_h)


def test_accepts_the_duplicate_triangle(doubled_room):
    v, t, poses, dirs, out = doubled_room
    g_r, g_h = _gpu_like(out)
    g_h = np.where(g_h >= 0, (g_h + 12) % 24, g_h)    # the other copy: equally correct
    check_flagged(v, t, poses, dirs, 0.0, 100.0, None, out[0], out[1], out[2], g_r, g_h)


def test_rejects_a_hit_behind_the_nearest_surface(doubled_room):
    v, t, poses, dirs, out = doubled_room
    g_r, g_h = _gpu_like(out)
    i = int(np.flatnonzero(out[1] >= 0)[5])
    g_r[i] = np.float32(out[0][i] + 0.25)
    with pytest.raises(AssertionError, match="beyond the nearest hit"):
        check_flagged(v, t, poses, dirs, 0.0, 100.0, None, out[0], out[1], out[2], g_r, g_h)


def test_rejects_a_miss_on_a_ray_that_is_not_edge_near(doubled_room):
    v, t, poses, dirs, out = doubled_room
    g_r, g_h = _gpu_like(out)
    i = int(np.flatnonzero((out[1] >= 0) & ((out[2] & oracle.FLAG_EDGE_NEAR) == 0))[3])
    g_r[i], g_h[i] = np.inf, -1
    with pytest.raises(AssertionError, match="missed where the oracle hits"):
        check_flagged(v, t, poses, dirs, 0.0, 100.0, None, out[0], out[1], out[2], g_r, g_h)


def test_allows_a_miss_on_an_edge_near_ray(doubled_room):
    v, t, poses, dirs, out = doubled_room
    g_r, g_h = _gpu_like(out)
    en = np.flatnonzero((out[1] >= 0) & ((out[2] & oracle.FLAG_EDGE_NEAR) != 0))
    assert len(en) > 0
    g_r[en[0]], g_h[en[0]] = np.inf, -1
    check_flagged(v, t, poses, dirs, 0.0, 100.0, None, out[0], out[1], out[2], g_r, g_h)


def test_rejects_a_triangle_the_ray_does_not_hit(doubled_room):
    v, t, poses, dirs, out = doubled_room
    g_r, g_h = _gpu_like(out)
    i = int(np.flatnonzero((out[1] >= 0) & ((out[2] & oracle.FLAG_EDGE_NEAR) == 0))[7])
    o, d = oracle.make_rays(poses, dirs)
    wrong = next(k for k in range(len(t)) if oracle.tri_test(o[i], d[i], *v[t[k]]) is None)
    g_h[i] = wrong
    with pytest.raises(AssertionError):
        check_flagged(v, t, poses, dirs, 0.0, 100.0, None, out[0], out[1], out[2], g_r, g_h)
