"""CPU oracle for mesh optimisation -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product library never does, and the two share no
code.

FGGS-LiDAR Sec. IV-B ("Mesh optimization") smooths the simplified mesh with
Taubin's non-shrinking two-step Laplacian smoothing, (lambda, mu) =
(0.5, -0.53) by default (Sec. V, "Implementation"), keeping boundary
vertices in place.  Written out directly with numpy:

  N(i)   = the distinct vertices sharing an edge with vertex i (never i)
  L(x)_i = (sum over j in N(i) of x_j) / |N(i)| - x_i      (umbrella operator)
  one iteration:  x <- x + lambda L(x);  x <- x + mu L(x)

Readings taken where the paper is silent (also in the design notes):

  S1  Uniform weights over the distinct 1-ring neighbours.
  S2  A boundary vertex is one with an incident edge that belongs to exactly
      one triangle; boundary vertices and vertices without neighbours do not
      move.
  S3  Arithmetic is float32, one rounded operation at a time: the neighbour
      sum runs over N(i) in ascending index order starting from 0, then the
      division by |N(i)|, then x + f * (mean - x) (subtraction, product,
      sum).  Both sides follow this order, so results are bit-identical.
"""
from __future__ import annotations

import numpy as np


def neighbours(nv: int, tris):
    """(sorted distinct neighbour lists as a padded [nv, maxdeg] array with
    -1, degree [nv], boundary flag [nv]) (readings S1, S2)."""
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    a = np.concatenate([t[:, 0], t[:, 0], t[:, 1], t[:, 1], t[:, 2], t[:, 2]])
    b = np.concatenate([t[:, 1], t[:, 2], t[:, 0], t[:, 2], t[:, 0], t[:, 1]])
    keep = a != b
    a, b = a[keep], b[keep]
    pairs, mult = np.unique(np.stack([a, b], axis=1), axis=0, return_counts=True)
    deg = np.bincount(pairs[:, 0], minlength=nv).astype(np.int64)
    boundary = np.zeros(nv, dtype=bool)
    boundary[pairs[mult == 1, 0]] = True
    maxdeg = int(deg.max()) if nv and len(pairs) else 0
    nb = np.full((nv, max(maxdeg, 1)), -1, dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(deg)])[:-1]
    rank = np.arange(len(pairs)) - start[pairs[:, 0]]
    nb[pairs[:, 0], rank] = pairs[:, 1]
    return nb, deg, boundary


def taubin(verts, tris, lam: float = 0.5, mu: float = -0.53, iterations: int = 10):
    """Taubin smoothing (readings S1-S3), float32 [nv, 3]."""
    x = np.asarray(verts, dtype=np.float32).copy()
    nv = len(x)
    nb, deg, boundary = neighbours(nv, tris)
    move = (deg > 0) & ~boundary
    degf = deg.astype(np.float32)
    for _ in range(iterations):
        for f in (np.float32(lam), np.float32(mu)):
            acc = np.zeros_like(x)
            for k in range(nb.shape[1]):
                m = k < deg
                acc[m] = acc[m] + x[nb[m, k]]
            mean = np.zeros_like(x)
            mean[move] = acc[move] / degf[move, None]
            step = (f * (mean - x)).astype(np.float32)
            x = np.where(move[:, None], (x + step).astype(np.float32), x)
    return x
