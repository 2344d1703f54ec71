"""CPU oracle for quadric-error decimation -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product library never does, and the two share no
code.

FGGS-LiDAR Sec. IV-B ("Mesh optimization") simplifies the raw isosurface with
quadric-error decimation to a target face count or ratio, and Sec. V
("Implementation") sets its defaults: face ratio 0.1, three rounds, boundary
protected.  The paper names no further detail.  The method is the quadric
error metric of Garland and Heckbert (1997): every vertex carries the sum of
the squared-distance quadrics of the planes of its faces, an edge (u, v) is
contracted to the point x minimising x^T (Q_u + Q_v) x, the contraction
costing that minimum, cheapest contractions first.  Contracting one edge at
a time is sequential by nature; this definition contracts many edges at once
(an independent set of locally cheapest ones, as parallel decimations do)
so that it can run data-parallel, and it is written here plainly, one edge
and one face at a time.

Readings (also listed in the design notes):

  Q0  Faces with a repeated corner index are not triangles and are dropped
      first.  F0 = the number of remaining faces.
  Q1  "3 rounds": round k = 1..R (R = 3) runs until at most
      T_k = ceil(F0 * ratio^(k / R)) faces remain (FP64, C-library pow), or
      no edge can be contracted.  Each round starts afresh from the current
      mesh: plane quadrics and protected vertices are recomputed.
  Q2  Plane quadric of a face (a, b, c): n = (b - a) x (c - a),
      q = (n_x, n_y, n_z, -n.a), K = q q^T / (n.n) (zero when n.n = 0), so
      [x 1] K [x 1]^T is the squared distance of x to the face's plane;
      faces are weighted equally (Garland and Heckbert's plain form).  A
      vertex's quadric is the sum over its faces in ascending face order;
      a contraction adds the two quadrics, Q_u + Q_v, in that order.
  Q3  "Boundary protected": an edge shared by other than exactly two faces
      (a boundary or non-manifold edge) protects both its vertices, which
      never move and whose edges are never contracted.
  Q4  An edge (u, v), u < v, of a face is a candidate when neither vertex is
      protected, it lies on exactly two faces, and u and v have exactly two
      common neighbours (the link condition of Dey et al. 1999, which keeps
      a closed manifold closed and manifold).
  Q5  Placement: with A = the upper-left 3x3 block of Q = Q_u + Q_v and
      b = -(q03, q13, q23), when trace(A) > 0 and |det A| >
      1e-6 (trace(A) / 3)^3 the minimiser x* = A^-1 b (Cramer's rule,
      cofactors along the first row); it is used when
      |x* - m|^2 <= 4 |p_v - p_u|^2 (m the edge midpoint).  Otherwise
      x* is the cheapest of p_u, p_v, m (the first of them on a tie), which
      keeps contractions along a crease on the crease.  The cost is
      [x* 1] Q [x* 1]^T, clamped at 0 and rounded to float32.
  Q6  A candidate is dropped when moving u and v to x* flips a face: for
      every face that has u or v but not both, with old normal n and new
      normal n', n.n > 0 requires n.n' > 0.
  Q7  One step: candidates are ordered by (float32 cost, pi(e)), where e is
      the edge's rank in the lexicographic order of all (u, v), u < v, edges
      of the live faces and pi is a fixed bijection of 32-bit integers (the
      "lowbias32" integer hash of C. Wellons' hash prospector: xorshift 16,
      multiply 0x7feb352d, xorshift 15, multiply 0x846ca68b, xorshift 16, all
      mod 2^32).  The hash, not the plain index order, breaks ties: flat
      regions give many exactly equal costs, and index order (spatially
      coherent on generated meshes) would leave one local minimum per flat
      region and step, so a step would contract about one edge; hashed
      priorities make the locally cheapest edges an independent set of a
      constant fraction of the candidates, as parallel decimation needs.
      Keys are unique (pi is a bijection).  With F faces left and target T,
      only the ceil((F - T) / 2) first ones are eligible (an interior
      contraction removes two faces).  An eligible edge
      is contracted when no eligible edge at any vertex of its two closed
      1-rings comes before it; such edges have no two endpoints in common or
      adjacent, so their contractions touch disjoint faces and commute.  Contraction: u takes x* and Q_u + Q_v; v is removed; faces
      with v now use u; the two faces with both are removed.  The cheapest
      eligible edge always qualifies, so every step makes progress.
  Q8  Arithmetic FP64 in the orders written below; positions are rounded to
      float32 once, at the end.  Output: the remaining vertices that a face
      uses, in ascending input index, numbered densely, and the remaining
      faces in ascending input order.
"""
from __future__ import annotations

import math

import numpy as np

UPPER = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def cross(a, b):
    """(a x b) componentwise, FP64."""
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def dot3(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def face_normal(pa, pb, pc):
    """n = (b - a) x (c - a) (reading Q2)."""
    e1 = (pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2])
    e2 = (pc[0] - pa[0], pc[1] - pa[1], pc[2] - pa[2])
    return cross(e1, e2)


def plane_quadric(pa, pb, pc):
    """K = q q^T / (n.n), upper triangle in UPPER order (reading Q2)."""
    n = face_normal(pa, pb, pc)
    nn = dot3(n, n)
    if nn == 0.0:
        return [0.0] * 10
    d = -dot3(n, pa)
    q = (n[0], n[1], n[2], d)
    return [(q[i] * q[j]) / nn for i, j in UPPER]


def quadric_cost(Q, x):
    """[x 1] Q [x 1]^T for Q in UPPER order."""
    x0, x1, x2 = x
    r0 = ((Q[0] * x0 + Q[1] * x1) + Q[2] * x2) + Q[3]
    r1 = ((Q[1] * x0 + Q[4] * x1) + Q[5] * x2) + Q[6]
    r2 = ((Q[2] * x0 + Q[5] * x1) + Q[7] * x2) + Q[8]
    r3 = ((Q[3] * x0 + Q[6] * x1) + Q[8] * x2) + Q[9]
    return ((x0 * r0 + x1 * r1) + x2 * r2) + r3


def minimiser(Q):
    """x* = A^-1 b by Cramer's rule when A is well conditioned (reading Q5),
    else None."""
    a00, a01, a02, b0 = Q[0], Q[1], Q[2], -Q[3]
    a11, a12, b1 = Q[4], Q[5], -Q[6]
    a22, b2 = Q[7], -Q[8]
    det = (a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02)) + \
        a02 * (a01 * a12 - a11 * a02)
    tr = (a00 + a11) + a22
    t3 = tr / 3.0
    if not (tr > 0.0 and abs(det) > 1e-6 * ((t3 * t3) * t3)):
        return None
    x0 = ((b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2)) +
          a02 * (b1 * a12 - a11 * b2)) / det
    x1 = ((a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02)) +
          a02 * (a01 * b2 - b1 * a02)) / det
    x2 = ((a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02)) +
          b0 * (a01 * a12 - a11 * a02)) / det
    return (x0, x1, x2)


def placement(Q, pu, pv):
    """(x*, cost) of contracting an edge with endpoints pu, pv (reading Q5)."""
    m = (0.5 * (pu[0] + pv[0]), 0.5 * (pu[1] + pv[1]), 0.5 * (pu[2] + pv[2]))
    x = minimiser(Q)
    if x is not None:
        dx = (x[0] - m[0], x[1] - m[1], x[2] - m[2])
        e = (pv[0] - pu[0], pv[1] - pu[1], pv[2] - pu[2])
        if not (dot3(dx, dx) <= 4.0 * dot3(e, e)):
            x = None
    if x is None:
        best = None
        for cand in (pu, pv, m):
            c = quadric_cost(Q, cand)
            if best is None or c < best[1]:
                best = (cand, c)
        x = best[0]
    c = quadric_cost(Q, x)
    return tuple(x), float(np.float32(max(c, 0.0)))


MASK32 = 0xFFFFFFFF


def perm32(e: int) -> int:
    """pi(e) of reading Q7: lowbias32 (xorshift-multiply), a bijection of
    32-bit integers."""
    x = e & MASK32
    x ^= x >> 16
    x = (x * 0x7FEB352D) & MASK32
    x ^= x >> 15
    x = (x * 0x846CA68B) & MASK32
    x ^= x >> 16
    return x


def round_targets(f0: int, ratio: float, rounds: int):
    """T_k = ceil(F0 * ratio^(k / R)), k = 1..R (reading Q1)."""
    r = float(np.float32(ratio))
    return [int(math.ceil(f0 * math.pow(r, k / rounds))) for k in range(1, rounds + 1)]


class _Mesh:
    """Mutable FP64 mesh: positions, faces (None once removed)."""

    def __init__(self, verts, tris):
        v = np.asarray(verts, dtype=np.float32).astype(np.float64).reshape(-1, 3)
        self.p = [tuple(r) for r in v]
        t = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.f = [tuple(int(i) for i in r) if len(set(r)) == 3 else None for r in t]   # Q0

    def live(self):
        return [k for k, f in enumerate(self.f) if f is not None]

    def incidence(self):
        """vertex -> ascending live faces; vertex -> neighbour set; edge -> face count."""
        vf, nb, ec = {}, {}, {}
        for k in self.live():
            f = self.f[k]
            for i in range(3):
                a, b = f[i], f[(i + 1) % 3]
                vf.setdefault(a, []).append(k)
                nb.setdefault(a, set()).update((b, f[(i + 2) % 3]))
                e = (min(a, b), max(a, b))
                ec[e] = ec.get(e, 0) + 1
        return vf, nb, ec


def _quadrics(m: _Mesh, vf):
    Kf = {}
    for k in m.live():
        a, b, c = m.f[k]
        Kf[k] = plane_quadric(m.p[a], m.p[b], m.p[c])
    Q = {}
    for v, faces in vf.items():
        acc = [0.0] * 10
        for k in faces:                       # ascending face order
            acc = [acc[i] + Kf[k][i] for i in range(10)]
        Q[v] = acc
    return Q


def _flips(m: _Mesh, vf, u, v, x):
    """True when moving u and v to x flips a face (reading Q6)."""
    for k in sorted(set(vf[u]) | set(vf[v])):
        f = m.f[k]
        if u in f and v in f:
            continue
        old = [m.p[i] for i in f]
        new = [x if i in (u, v) else m.p[i] for i in f]
        n0 = face_normal(*old)
        if dot3(n0, n0) > 0.0 and not (dot3(n0, face_normal(*new)) > 0.0):
            return True
    return False


def candidates(m: _Mesh, Q, protected):
    """{(u, v): (key, x*)} with key = (float32 cost, pi(edge rank)) (readings
    Q4-Q7)."""
    vf, nb, ec = m.incidence()
    out = {}
    for e, ((u, v), cnt) in enumerate(sorted(ec.items())):
        if cnt != 2 or u in protected or v in protected:
            continue
        if len(nb[u] & nb[v]) != 2:
            continue
        Qe = [Q[u][i] + Q[v][i] for i in range(10)]
        x, cost = placement(Qe, m.p[u], m.p[v])
        if _flips(m, vf, u, v, x):
            continue
        out[(u, v)] = ((cost, perm32(e)), x, Qe)
    return out, vf, nb


def select(cands, nb, need: int):
    """The edges contracted in one step (reading Q7)."""
    order = sorted(cands.items(), key=lambda kv: kv[1][0])[:need]
    best = {}
    for (u, v), (key, _, _) in order:
        for w in (u, v):
            if w not in best or key < best[w]:
                best[w] = key
    none = (math.inf, math.inf)
    chosen = []
    for (u, v), (key, x, Qe) in order:
        ring = {u, v} | nb[u] | nb[v]
        if all(best.get(w, none) >= key for w in ring):
            chosen.append((u, v, x, Qe))
    return chosen


def decimate_qem(verts, tris, ratio: float = 0.1, rounds: int = 3, trace=None):
    """Decimated mesh (verts float32 [n, 3], tris int32 [m, 3]) by readings
    Q0-Q8.  `trace`, when a list, receives (round, faces before, contracted)
    per step."""
    m = _Mesh(verts, tris)
    f0 = len(m.live())
    for k, target in enumerate(round_targets(f0, ratio, rounds)):
        vf, nb, ec = m.incidence()
        protected = set()
        for (a, b), cnt in ec.items():
            if cnt != 2:
                protected.update((a, b))
        Q = _quadrics(m, vf)
        while True:
            nf = len(m.live())
            if nf <= target:
                break
            cands, vf, nb = candidates(m, Q, protected)
            if not cands:
                break
            need = (nf - target + 1) // 2
            chosen = select(cands, nb, need)
            for u, v, x, Qe in chosen:
                m.p[u] = x
                Q[u] = Qe
                for fk in set(vf[v]):
                    f = m.f[fk]
                    if u in f:
                        m.f[fk] = None
                    else:
                        m.f[fk] = tuple(u if i == v else i for i in f)
            if trace is not None:
                trace.append((k, nf, len(chosen)))
    live = m.live()
    used = sorted({i for fk in live for i in m.f[fk]})
    newid = {old: new for new, old in enumerate(used)}
    out_v = np.array([m.p[i] for i in used], dtype=np.float64).reshape(-1, 3).astype(np.float32)
    out_t = np.array([[newid[i] for i in m.f[fk]] for fk in live], dtype=np.int32).reshape(-1, 3)
    return out_v, out_t
