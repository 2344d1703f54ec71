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
  S3  The definition is evaluated in FP64 (``taubin_fp64``), with the
      parameters as the float32 values the library takes; it also returns a
      per-vertex bound on any float32 evaluation that sums the neighbours in
      some order, divides by |N(i)| and forms x + f (mean - x) (derivation in
      its docstring), the tolerance of the GPU comparison.  ``taubin`` is one
      such float32 evaluation, one rounded operation at a time: the neighbour
      sum over N(i) in ascending index order starting from 0, the division,
      then the subtraction, product and sum.  The GPU follows the same
      order, so it is also compared bit for bit as a second check.
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


U32 = 2.0 ** -24   # unit roundoff of float32


def taubin_fp64(verts, tris, lam: float = 0.5, mu: float = -0.53, iterations: int = 10):
    """Taubin smoothing by its definition in FP64 (readings S1, S2), and a
    per-vertex, per-coordinate bound on |x_fp32 - x| for a float32
    evaluation of the same steps.  Returns (x [nv, 3], bound [nv, 3]).

    One step with factor f in float32 from a state y (the float32 iterate):
    the sum of d = |N(i)| neighbours, d - 1 roundings, errs by at most
    gamma_(d-1) sum |y_j| (gamma_k = k u / (1 - k u), u = 2^-24); the
    division, subtraction, product and sum each add u times their result's
    magnitude, so the local error is at most
      r_i = 1.01 (|f| (gamma_(d-1) M_i + u (|m_i| + |m_i - y_i|))
                  + u (|s_i| + |y'_i|)),
    M_i = mean |y_j|, m_i = the mean, s_i = f (m_i - y_i), y'_i = y_i + s_i
    (1.01 covers the second-order terms).  The step is linear,
    T(y)_i = (1 - f) y_i + f mean_j y_j, so an error e carried into it comes
    out at most |1 - f| e_i + |f| mean_j e_j.  The bound is that recurrence
    from e = 0, with the local terms evaluated on the FP64 iterate; fixed
    vertices carry no error."""
    x = np.asarray(verts, dtype=np.float32).astype(np.float64).copy()
    nv = len(x)
    nb, deg, boundary = neighbours(nv, tris)
    move = (deg > 0) & ~boundary
    e = np.zeros_like(x)
    d = deg.astype(np.float64)
    safe = np.maximum(d, 1.0)
    gamma = (d - 1) * U32 / (1 - (d - 1) * U32)
    for _ in range(iterations):
        for f in (float(np.float32(lam)), float(np.float32(mu))):
            acc = np.zeros_like(x)
            acc_abs = np.zeros_like(x)
            acc_e = np.zeros_like(x)
            for k in range(nb.shape[1]):
                m = k < deg
                acc[m] += x[nb[m, k]]
                acc_abs[m] += np.abs(x[nb[m, k]])
                acc_e[m] += e[nb[m, k]]
            mean = acc / safe[:, None]
            step = f * (mean - x)
            new = x + step
            r = 1.01 * (abs(f) * (gamma[:, None] * acc_abs / safe[:, None]
                                  + U32 * (np.abs(mean) + np.abs(mean - x)))
                        + U32 * (np.abs(step) + np.abs(new)))
            e_new = abs(1 - f) * e + abs(f) * acc_e / safe[:, None] + r
            x = np.where(move[:, None], new, x)
            e = np.where(move[:, None], e_new, 0.0)
    return x, e


# ---------------------------------------------------------------------------
# Quadric-error decimation by vertex clustering
#
# Readings (also in the design notes):
#   D1  The decimation is quadric-error vertex clustering (the parallel form
#       of quadric decimation): vertices are grouped by a uniform grid of
#       cell size c anchored at the mesh's box minimum; every group becomes
#       one vertex placed at the minimiser of the sum of its vertices'
#       quadrics (area-weighted plane quadrics of the incident triangles),
#       or at the mean of its vertices when that minimiser is ill-posed or
#       leaves the group's cell widened by one cell; triangles whose three
#       corners fall into three different groups are kept, in input order.
#   D2  "Boundary protected": vertices on an edge of one triangle form
#       groups of their own and keep their position.
#   D3  The target face ratio sets c: geometric bisection (12 steps) of c
#       between extent / 1023 and the extent for the smallest tried c whose
#       face count is at most floor(ratio * triangles).
#   D4  Arithmetic: FP64 in the orders written below; positions rounded to
#       float32 at the end.

UPPER = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def face_quadrics(verts, tris):
    """Area-weighted plane quadric of every triangle, FP64 [nt, 10] (UPPER
    order of the 4x4 matrix), zero for zero-area triangles."""
    v = np.asarray(verts, dtype=np.float32).astype(np.float64)
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    e1, e2 = b - a, c - a
    nx = e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1]
    ny = e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2]
    nz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    ln = np.sqrt((nx * nx + ny * ny) + nz * nz)
    ok = ln > 0
    safe = np.where(ok, ln, 1.0)
    ux, uy, uz = nx / safe, ny / safe, nz / safe
    d = -((ux * a[:, 0] + uy * a[:, 1]) + uz * a[:, 2])
    w = 0.5 * ln
    p = [ux, uy, uz, d]
    K = np.stack([w * (p[i] * p[j]) for i, j in UPPER], axis=1)
    K[~ok] = 0.0
    return K


def vertex_quadrics(nv, tris, K):
    """Sum over each vertex's incident triangles in ascending index order."""
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    nt = len(t)
    pairs = []
    for k in range(3):
        pairs.append(np.stack([t[:, k], np.arange(nt)], axis=1))
    pv = np.unique(np.concatenate(pairs), axis=0)          # (vertex, triangle), distinct, sorted
    Q = np.zeros((nv, 10))
    if len(pv) == 0:
        return Q
    cnt = np.bincount(pv[:, 0], minlength=nv)
    start = np.concatenate([[0], np.cumsum(cnt)])[:-1]
    rank = np.arange(len(pv)) - start[pv[:, 0]]
    for r in range(int(rank.max()) + 1):
        sel = rank == r
        Q[pv[sel, 0]] = Q[pv[sel, 0]] + K[pv[sel, 1]]
    return Q


def _cells(v64, lo, c):
    ext = np.asarray(v64.max(axis=0) if len(v64) else lo, dtype=np.float64) - lo
    n = np.floor(ext / c).astype(np.int64) + 1
    idx = np.floor((v64 - lo) / c).astype(np.int64)
    return idx, n


def cluster_once(verts, tris, c, boundary):
    """Group id of every vertex (groups ordered by cell index, then boundary
    singletons by vertex index) and the kept-triangle mask (reading D1, D2)."""
    v32 = np.asarray(verts, dtype=np.float32)
    v64 = v32.astype(np.float64)
    lo = v32.min(axis=0).astype(np.float64)
    idx, n = _cells(v64, lo, c)
    key = idx[:, 0] + n[0] * (idx[:, 1] + n[1] * idx[:, 2])
    big = int(n[0] * n[1] * n[2])
    nv = len(v32)
    full = np.where(boundary, big + np.arange(nv), key)
    uniq, gid = np.unique(full, return_inverse=True)
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    g = gid[t]
    keep = (g[:, 0] != g[:, 1]) & (g[:, 1] != g[:, 2]) & (g[:, 0] != g[:, 2])
    return gid, len(uniq), keep, idx, lo


def representative(Qc, members, v64, cell_idx, lo, c):
    """Position of one group (reading D1)."""
    q = Qc
    a00, a01, a02, b0 = q[0], q[1], q[2], -q[3]
    a11, a12, b1 = q[4], q[5], -q[6]
    a22, b2 = q[7], -q[8]
    det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02)
    tr = (a00 + a11) + a22
    t3 = tr / 3.0
    if tr > 0 and abs(det) > 1e-6 * ((t3 * t3) * t3):
        x0 = (b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2) + a02 * (b1 * a12 - a11 * b2)) / det
        x1 = (a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02) + a02 * (a01 * b2 - b1 * a02)) / det
        x2 = (a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02) + b0 * (a01 * a12 - a11 * a02)) / det
        x = np.array([x0, x1, x2])
        cmin = lo + (cell_idx - 1) * c
        cmax = lo + (cell_idx + 2) * c
        if np.all(x >= cmin) and np.all(x <= cmax):
            return x
    s = np.zeros(3)
    for m in members:
        s = s + v64[m]
    return s / len(members)


def decimate(verts, tris, ratio: float):
    """Decimated mesh (verts float32 [n, 3], tris int32 [m, 3]) and the cell
    size used (readings D1-D4)."""
    v32 = np.asarray(verts, dtype=np.float32)
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    nv, nt = len(v32), len(t)
    _, _, boundary = neighbours(nv, t)
    v64 = v32.astype(np.float64)
    ext = float((v32.max(axis=0).astype(np.float64) - v32.min(axis=0).astype(np.float64)).max())
    target = int(np.floor(float(np.float32(ratio)) * nt))

    def faces(c):
        return int(cluster_once(v32, t, c, boundary)[2].sum())

    c_lo, c_hi = ext / 1023.0, ext
    if faces(c_lo) <= target:
        c = c_lo
    else:
        for _ in range(12):
            mid = float(np.sqrt(c_lo * c_hi))
            if faces(mid) <= target:
                c_hi = mid
            else:
                c_lo = mid
        c = c_hi
    gid, ng, keep, idx, lo = cluster_once(v32, t, c, boundary)
    K = face_quadrics(v32, t)
    Q = vertex_quadrics(nv, t, K)
    order = np.argsort(gid, kind="stable")
    starts = np.searchsorted(gid[order], np.arange(ng))
    ends = np.searchsorted(gid[order], np.arange(ng), side="right")
    used = np.zeros(ng, dtype=bool)
    kt = t[keep]
    used[gid[kt].ravel()] = True
    newid = np.cumsum(used) - 1
    out_v = []
    for gi in np.nonzero(used)[0]:
        members = order[starts[gi]:ends[gi]]
        if boundary[members[0]]:
            out_v.append(v64[members[0]])
            continue
        Qc = np.zeros(10)
        for m in members:
            Qc = Qc + Q[m]
        out_v.append(representative(Qc, members, v64, idx[members[0]], lo, c))
    out_v = np.array(out_v, dtype=np.float64).reshape(-1, 3).astype(np.float32)
    out_t = newid[gid[kt]].astype(np.int32)
    return out_v, out_t, c


# ---------------------------------------------------------------------------
# Removal of tiny components
#
# Sec. IV-B removes tiny components while decimating.  Readings (also in the
# design notes):
#   D5  Two triangles are connected when they share a vertex; a component is
#       a class of the transitive closure, labelled by its lowest vertex
#       index.  Components with fewer than min_faces triangles are removed
#       (a component of exactly min_faces is kept).  The remaining triangles
#       keep their input order; the vertices they reference keep their input
#       order and are numbered densely, and vertices no triangle references
#       are dropped.


def component_labels(nv: int, tris):
    """Lowest vertex index of each vertex's component in the graph whose
    edges are the triangle sides (scipy's connected components as the
    primitive); a vertex in no triangle is its own component."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    if nv == 0:
        return np.zeros(0, dtype=np.int64)
    rows = np.concatenate([t[:, 0], t[:, 1], t[:, 2]])
    cols = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(nv, nv))
    ncomp, lab = connected_components(g, directed=False)
    lowest = np.full(ncomp, nv, dtype=np.int64)
    np.minimum.at(lowest, lab, np.arange(nv))
    return lowest[lab]


def remove_small_components(verts, tris, min_faces: int):
    """(verts float32 [n, 3], tris int32 [m, 3], vertex labels [nv]) after
    dropping the components of fewer than min_faces triangles (reading D5)."""
    v = np.asarray(verts, dtype=np.float32).reshape(-1, 3)
    t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    nv = len(v)
    labels = component_labels(nv, t)
    if len(t) == 0:
        return np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), labels
    faces = np.bincount(labels[t[:, 0]], minlength=nv)
    keep = faces[labels[t[:, 0]]] >= min_faces
    kt = t[keep]
    used = np.zeros(nv, dtype=bool)
    used[kt.ravel()] = True
    newid = np.cumsum(used) - 1
    return v[used].copy(), newid[kt].astype(np.int32).reshape(-1, 3), labels
