"""Checks on the seeded synthetic inputs (meshes, poses, beam patterns)."""
import numpy as np

import synth


def _edge_use_counts(tris, nv):
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), axis=1)
    key = e[:, 0].astype(np.int64) * nv + e[:, 1]
    _, c = np.unique(key, return_counts=True)
    return c


def test_box_room_and_sphere_closed():
    for v, t in (synth.box_room(), synth.uv_sphere((0, 0, 0), 1.0, 64, 32)):
        assert np.all(_edge_use_counts(t, len(v)) == 2)
        assert t.min() >= 0 and t.max() < len(v)


def test_room_sphere_scene_shape():
    s = synth.room_sphere_scene(0)
    assert s.tris.shape == (12 + 3968, 3)
    assert s.n_rays == 5760 and s.dirs.shape == (5760, 3)
    c = s.meta["sphere_center"]
    assert np.all(c >= 1.1) and np.all(c <= np.array([8.9, 6.9, 1.9]))
    p = s.poses[0, [3, 7, 11]]
    assert np.all(p > 0.3) and np.linalg.norm(p - c) >= 1.3


def test_pattern_layout_and_units():
    d = synth.lidar_pattern(16, -15.0, 15.0, 360)
    assert d.shape == (5760, 3) and d.dtype == np.float32
    assert np.allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=1e-7)
    el = np.degrees(np.arcsin(d[:, 2].astype(np.float64)))
    assert np.allclose(el[::360], np.linspace(-15, 15, 16), atol=1e-4)
    # j = el * n_az + az; azimuth 1 is +1 deg
    assert np.allclose(np.degrees(np.arctan2(d[1, 1], d[1, 0])), 1.0, atol=1e-4)


def test_marching_cubes_mesh_closed_and_deterministic():
    sdf = synth.indoor_sdf(3, n_prims=40)
    v1, t1 = synth.polygonise(sdf, 0.1)
    v2, t2 = synth.polygonise(sdf, 0.1)
    assert np.array_equal(v1, v2) and np.array_equal(t1, t2)
    assert len(t1) > 10000
    assert np.all(_edge_use_counts(t1, len(v1)) == 2)
    assert t1.min() >= 0 and t1.max() < len(v1)
    # vertices sit on the zero set up to the linear-interpolation error
    f = sdf.sdf(v1[:: max(1, len(v1) // 2000)])
    assert np.abs(f).max() < 0.1


def test_free_space_poses_clearance():
    sdf = synth.indoor_sdf(3, n_prims=40)
    poses = synth.free_space_poses(sdf, 32, 7)
    assert poses.shape == (32, 12)
    assert np.all(sdf.sdf(poses[:, [3, 7, 11]]) >= 0.3 - 1e-6)
    R = poses[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]].reshape(-1, 3, 3).astype(np.float64)
    assert np.allclose(R @ R.transpose(0, 2, 1), np.eye(3), atol=1e-6)


def test_terrain_scene():
    v, t, height, boxes = synth.terrain_scene(4, 50_000, n_boxes=20)
    assert 45_000 < len(t) < 56_000
    assert t.min() >= 0 and t.max() < len(v)
    poses = synth.terrain_poses(height, boxes, 5, 1)
    z = poses[:, 11] - height(poses[:, 3], poses[:, 7])
    assert np.all((z >= 1.5 - 1e-4) & (z <= 3.0 + 1e-4))


def test_workload_configs_are_complete():
    """Every benchmark workload's seeds and sizes are stored, and the stored
    room-sphere pattern is the one the generator draws."""
    for name in ("room_sphere", "indoor_1m", "batched_4096", "uneven_64", "serve_16"):
        c = synth.workload_config(name)
        assert c["name"] == name and c["description"]
        assert len(c["t_range"]) == 2 and c["t_range"][0] < c["t_range"][1]
    rs = synth.workload_config("room_sphere")
    s = synth.room_sphere_scene(rs["scene_seed"])
    p = rs["pattern"]
    assert len(s.dirs) == p["rings"] * p["azimuths"] and s.n_az == p["azimuths"]
    assert (s.t_min, s.t_max) == tuple(rs["t_range"])
    b = synth.workload_config("batched_4096")
    bp = b["pattern"]
    assert b["envs"] * bp["rings"] * bp["azimuths"] == 134_217_728
