"""CPU oracle for the point-cloud fidelity metrics -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product library never does, and the two share no
code.

FGGS-LiDAR Sec. V ("Metrics") reports the symmetric Chamfer distance and the
F-score at 0.05 m between a simulated LiDAR point cloud P and the ground-truth
one G (the same sensor pose and scan pattern on the ground-truth mesh).
Written out directly, in FP64, with scipy's k-d tree as the nearest-neighbour
primitive:

  d(p, G)    = min over g in G of |p - g|
  CD         = ( mean over P of d(p, G) + mean over G of d(g, P) ) / 2
  precision  = |{ p in P : d(p, G) <= tau }| / |P|
  recall     = |{ g in G : d(g, P) <= tau }| / |G|
  F          = 2 precision recall / (precision + recall)   (0 if both are 0)

Readings taken where the paper is silent (also listed in the design notes):

  M1  Distances are Euclidean, not squared, in metres; CD averages the two
      directed means (so identical clouds give 0 and a rigid offset s gives
      |s| when it is below the point spacing).
  M2  "Within tau" is inclusive (d <= tau).
  M3  A LiDAR point is origin + range * direction for every beam that hit;
      misses are not points.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def nearest(ref, query):
    """d(q, ref) and the index of a nearest reference point, FP64."""
    ref = np.asarray(ref, dtype=np.float32).astype(np.float64)
    query = np.asarray(query, dtype=np.float32).astype(np.float64)
    if len(ref) == 0:
        return np.full(len(query), np.inf), np.full(len(query), -1, dtype=np.int64)
    d, i = cKDTree(ref).query(query, k=1)
    return d, i


def chamfer_fscore(P, G, tau: float = 0.05):
    """(CD, mean d(P, G), mean d(G, P), precision, recall, F) (readings M1, M2)."""
    dpg, _ = nearest(G, P)
    dgp, _ = nearest(P, G)
    mpg = float(np.mean(dpg)) if len(dpg) else float("nan")
    mgp = float(np.mean(dgp)) if len(dgp) else float("nan")
    t = float(np.float32(tau))
    prec = float(np.mean(dpg <= t)) if len(dpg) else 0.0
    rec = float(np.mean(dgp <= t)) if len(dgp) else 0.0
    f = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
    return 0.5 * (mpg + mgp), mpg, mgp, prec, rec, f


def lidar_points(poses, dirs, rng, hit):
    """Points origin + range * normalize(R d) of the beams that hit (reading
    M3), FP64 from the float32 inputs; layout of rng/hit: [env][beam]."""
    poses = np.asarray(poses, dtype=np.float32).astype(np.float64).reshape(-1, 3, 4)
    dirs = np.asarray(dirs, dtype=np.float32).astype(np.float64)
    rng = np.asarray(rng, dtype=np.float64).reshape(len(poses), len(dirs))
    hit = np.asarray(hit).reshape(len(poses), len(dirs))
    out = []
    for e in range(len(poses)):
        R, t = poses[e][:, :3], poses[e][:, 3]
        d = dirs @ R.T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        ok = hit[e] >= 0
        out.append(t + rng[e][ok, None] * d[ok])
    return np.concatenate(out) if out else np.zeros((0, 3))
