"""CPU oracle for the narrow-band TSDF and marching cubes -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product library never does, and the two share no
code (the marching-cubes table is generated here by its own implementation
of the construction described below).

What it computes is FGGS-LiDAR Sec. IV-B ("Binary denoising and
re-thresholding", "Narrow-band TSDF", "Isosurface extraction") on the
surface mask V of Sec. IV-A, written out directly with numpy and scipy:

  V'      = G * V                       (smoothing eq.)
  V~      = [V' >= tau]  or  [V' >= Quantile_q(V')]   (re-threshold eqs.)
  O       = the 6-connected component of free voxels (V~ = 0) joined to a
            padded frame around the grid;  s = +1 on O, -1 elsewhere
  S_0     = { x : some 6-neighbour y has V~(y) != V~(x) }   (boundary set)
  p(x)    = the first shell S_m of a 6-neighbour expansion from S_0 that
            reaches x;  delta = p h                            (distance eq.)
  phi     = clip(s delta, -r, r)                                (TSDF eq.)
  mesh    = marching cubes of phi at iso on the lattice of voxel centres

Readings taken where the paper is silent (each is also listed in the design
notes):

  T1  The Gaussian kernel of scale sigma (metres; sigma_v = sigma / h voxels)
      is the binomial kernel with n = max(1, floor(2 sigma_v^2 + 1/2)) steps,
      weights C(2n, n + k) for k = -n..n (variance n / 2, the discrete
      Gaussian of integer weights), separable on the three axes, zero outside
      the grid; V' = sum / 2^(6n).  All sums are exact integers, and V~ is
      decided exactly: sum >= ceil(tau 2^(6n)).  n <= 10.
  T2  Quantile re-threshold: Quantile_q(V') over all N voxels of the grid,
      interpolated linearly between consecutive order statistics (numpy's
      default): with V' sorted ascending, x_0 <= ... <= x_(N-1), position
      p = q (N - 1) (FP64, q the float32 input), k = floor(p), Quantile =
      x_k + (p - k)(x_(k+1) - x_k).  No value of V' lies strictly between
      x_k and x_(k+1), so V' >= Quantile exactly when V' >= x_k (p = k) or
      V' >= x_(k+1) (p > k); decided on the integer sums like the fixed form.
  T2b mc_step (Isosurface extraction): marching cubes of phi sampled at
      every mc_step-th lattice point of each axis, (i, j, k) mc_step for
      i <= (nx - 1) / mc_step and so on, as a grid of spacing fl32(s h) and
      origin fl32(o - (s - 1) h / 2) per axis (FP64 from the float32 o and
      h, rounded once; s = mc_step), whose voxel centres o' + (i + 1/2) s h
      fall on the fine centres o + (i s + 1/2) h (mc_step = 1: the plain
      form).
  T3  The padded frame is free, so a free voxel on the grid boundary is
      outside; in S_0 a neighbour outside the grid counts as free (0).
  T4  Shells are counted up to P = ceil(r / h); a voxel not reached by then
      gets |phi| = r.  delta = p h is a float32 product, then clipped.
  T5  Marching cubes: lattice points are voxel centres, cells are 2 x 2 x 2
      groups of them; a corner is inside when phi < iso.  A crossed edge
      (one corner inside) carries one vertex, at t = (iso - phi_a) /
      (phi_b - phi_a) from its lower corner a (float32, in this operation
      order: x = c_a + t h with c_a the float32 centre).  Vertices are
      numbered by (lattice point, axis +x/+y/+z); triangles by (cell,
      position in the case).  The case table: on each cube face, walk its
      corners counter-clockwise about the outward normal; each crossing from
      outside to inside starts a segment that ends at the next crossing from
      inside to outside (so diagonal inside corners on a face are kept apart);
      chaining the segments of the six faces gives closed loops; each loop
      starts at its lowest-numbered edge (edges numbered by (axis, lower
      corner)) and loops are taken in that order.  Each loop is cut into a
      fan (a, v_i, v_i+1) from its first vertex a (in loop order) whose
      diagonals all cross the cube's interior, i.e. join edges that share no
      face (a diagonal lying on a face could overlap the neighbouring cell's
      triangles; every loop of the 256 cases has such a vertex).  Triangles
      face the outside region (phi >= iso).
  T6  Vertex normals (Sec. IV-B: normals from the gradient of phi, pointing
      outward): at every lattice point the gradient of phi in units of phi
      per voxel, per axis the central difference (phi(+1) - phi(-1)) * 1/2,
      one-sided (phi(1) - phi(0), phi(n-1) - phi(n-2)) on the grid's first
      and last point, 0 on an axis of size 1.  A vertex at t on the edge from
      a to b takes n = (1 - t) g_a + t g_b and returns n / |n| ((0, 0, 0) if
      |n| = 0).  phi grows outward (s = +1 outside), so the normals point
      out of the solid.

The definitions of T5 (vertex positions) and T6 (normals) are evaluated two
ways.  ``marching_cubes_fp64`` is the definition itself: every quantity in
FP64 from the float32 phi, origin and spacing, and it returns per-vertex
bounds for any float32 evaluation (derivation in its docstring), the
tolerance of the GPU comparison.  ``marching_cubes`` is one float32
evaluation, one rounded operation at a time in a fixed order (t, then
x = c_a + t h with c_a the float32 centre; w = 1 - t, n_k = w g_a,k +
t g_b,k as two products and a sum, l = sqrt((n_x n_x + n_y n_y) + n_z n_z),
n_k / l); the GPU follows the same order, so it is also compared bit for
bit as a second check.  The inside/outside decisions, the case table and
the numbering are exact comparisons of the same float32 phi in both.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage

# cube corners: bit k of the case index is corner k; corner k = (k & 1, k >> 1 & 1, k >> 2 & 1)
CORNERS = [(k & 1, (k >> 1) & 1, (k >> 2) & 1) for k in range(8)]
# cube edges: (corner a, corner b) with b = a + unit vector along `axis`; ordered by (axis, a)
EDGES = []
for axis in range(3):
    for a in range(8):
        if not (a >> axis) & 1:
            EDGES.append((a, a | (1 << axis), axis))
EDGE_ID = {(a, b): i for i, (a, b, _) in enumerate(EDGES)}
EDGE_ID.update({(b, a): i for i, (a, b, _) in enumerate(EDGES)})


def _faces():
    """Six faces, each as its 4 corners counter-clockwise about the outward
    normal (right-handed)."""
    faces = []
    for axis in range(3):
        u, v = (axis + 1) % 3, (axis + 2) % 3          # (u, v, axis) right-handed
        for side in (0, 1):
            def corner(cu, cv):
                c = [0, 0, 0]
                c[axis], c[u], c[v] = side, cu, cv
                return c[0] | (c[1] << 1) | (c[2] << 2)
            ring = [corner(0, 0), corner(1, 0), corner(1, 1), corner(0, 1)]   # CCW about +axis
            if side == 0:
                ring = ring[::-1]                                            # outward is -axis
            faces.append(ring)
    return faces


FACES = _faces()


def case_loops(case: int):
    """Closed loops of cube edges for one case (reading T5)."""
    inside = [(case >> k) & 1 for k in range(8)]
    succ = {}
    for ring in FACES:
        cross = []   # (position along the walk, edge, kind) kind 'in' = outside->inside
        for i in range(4):
            a, b = ring[i], ring[(i + 1) % 4]
            if inside[a] != inside[b]:
                cross.append((i, EDGE_ID[(a, b)], "in" if inside[b] else "out"))
        for j, (i, e, kind) in enumerate(cross):
            if kind != "in":
                continue
            for step in range(1, len(cross)):
                _, e2, k2 = cross[(j + step) % len(cross)]
                if k2 == "out":
                    succ[e] = e2
                    break
    loops = []
    seen = set()
    for e0 in sorted(succ):
        if e0 in seen:
            continue
        loop = [e0]
        seen.add(e0)
        e = succ[e0]
        while e != e0:
            loop.append(e)
            seen.add(e)
            e = succ[e]
        loops.append(loop)
    return loops


def _edge_faces():
    out = {}
    for fi, ring in enumerate(FACES):
        for i in range(4):
            out.setdefault(EDGE_ID[(ring[i], ring[(i + 1) % 4])], set()).add(fi)
    return out


EDGE_FACES = _edge_faces()


def fan_apex(loop):
    """Position in the loop of the first vertex whose diagonals join edges
    with no common face (reading T5)."""
    k = len(loop)
    for j in range(k):
        if all(not (EDGE_FACES[loop[j]] & EDGE_FACES[loop[i]])
               for i in range(k) if i not in (j, (j + 1) % k, (j - 1) % k)):
            return j
    raise AssertionError("no interior fan apex")


def case_table():
    """Triangles (edge triples) of every case, [256] lists."""
    table = []
    for case in range(256):
        tris = []
        for loop in case_loops(case):
            j = fan_apex(loop)
            ring = loop[j:] + loop[:j]
            for i in range(1, len(ring) - 1):
                tris.append((ring[0], ring[i], ring[i + 1]))
        table.append(tris)
    return table


_TABLE = None


def table():
    global _TABLE
    if _TABLE is None:
        _TABLE = case_table()
    return _TABLE


# ---------------------------------------------------------------------------
def binomial_steps(sigma_m: float, h: float) -> int:
    sv = float(np.float32(sigma_m)) / float(np.float32(h))
    n = max(1, int(math.floor(2.0 * sv * sv + 0.5)))
    if n > 10:
        raise ValueError("smoothing scale too large (n > 10)")
    return n


def denoise(surf, sigma_m: float, h: float, tau: float):
    """V~ = [G * V >= tau] with the binomial kernel of reading T1 (exact
    integers).  surf: uint8 [nz][ny][nx].  Returns (V~ uint8, sum int64)."""
    n = binomial_steps(sigma_m, h)
    w = np.array([math.comb(2 * n, n + k) for k in range(-n, n + 1)], dtype=np.int64)
    acc = np.asarray(surf).astype(np.int64)
    for axis in (2, 1, 0):
        acc = ndimage.correlate1d(acc, w, axis=axis, mode="constant", cval=0)
    thr = math.ceil(float(np.float32(tau)) * 2.0 ** (6 * n))
    return (acc >= thr).astype(np.uint8), acc


def quantile_threshold(acc, q: float) -> int:
    """The integer sum thr with [V' >= Quantile_q(V')] = [sum >= thr]
    (reading T2)."""
    flat = np.sort(np.asarray(acc, dtype=np.int64).ravel())
    n = flat.size
    pos = float(np.float32(q)) * float(n - 1)
    k = int(math.floor(pos))
    return int(flat[k]) if pos == k else int(flat[k + 1])


def denoise_quantile(surf, sigma_m: float, h: float, q: float):
    """V~ = [G * V >= Quantile_q(G * V)] (readings T1, T2).  Returns (V~, sum)."""
    _, acc = denoise(surf, sigma_m, h, 0.0)
    return (acc >= quantile_threshold(acc, q)).astype(np.uint8), acc


def outside(vt):
    """O: free voxels 6-connected to the padded frame (reading T3)."""
    free = np.pad(np.asarray(vt) == 0, 1, mode="constant", constant_values=True)
    lab, _ = ndimage.label(free)          # 6-connectivity (the default structure)
    return (lab == lab[0, 0, 0])[1:-1, 1:-1, 1:-1]


def boundary_set(vt):
    """S_0 (reading T3: outside the grid counts as 0)."""
    v = np.pad(np.asarray(vt).astype(np.int8), 1, mode="constant", constant_values=0)
    c = v[1:-1, 1:-1, 1:-1]
    s = np.zeros(c.shape, dtype=bool)
    for sl in [(slice(0, -2), slice(1, -1), slice(1, -1)), (slice(2, None), slice(1, -1), slice(1, -1)),
               (slice(1, -1), slice(0, -2), slice(1, -1)), (slice(1, -1), slice(2, None), slice(1, -1)),
               (slice(1, -1), slice(1, -1), slice(0, -2)), (slice(1, -1), slice(1, -1), slice(2, None))]:
        s |= v[sl] != c
    return s


def shells(s0, P: int):
    """p(x): first-arrival shell of a 6-neighbour expansion from S_0; -1 if
    not reached within P shells.  Breadth-first by explicit layers."""
    p = np.full(s0.shape, -1, dtype=np.int32)
    p[s0] = 0
    front = s0.copy()
    for m in range(1, P + 1):
        f = np.pad(front, 1, mode="constant", constant_values=False)
        nb = (f[:-2, 1:-1, 1:-1] | f[2:, 1:-1, 1:-1] | f[1:-1, :-2, 1:-1] | f[1:-1, 2:, 1:-1]
              | f[1:-1, 1:-1, :-2] | f[1:-1, 1:-1, 2:])
        new = nb & (p < 0)
        p[new] = m
        front = new
    return p


def tsdf(surf, h: float, sigma_m: float, tau: float, r: float, quantile=None):
    """(phi float32, V~, sign, p) for the surface mask `surf` (readings T1-T4);
    with quantile = q the re-threshold is the quantile form (tau unused)."""
    if quantile is None:
        vt, _ = denoise(surf, sigma_m, h, tau)
    else:
        vt, _ = denoise_quantile(surf, sigma_m, h, quantile)
    sgn = np.where(outside(vt), 1, -1).astype(np.int8)
    hf, rf = np.float32(h), np.float32(r)
    P = int(math.ceil(float(rf) / float(hf)))
    p = shells(boundary_set(vt), P)
    delta = np.where(p >= 0, p.astype(np.float32) * hf, rf).astype(np.float32)
    phi = np.clip(sgn.astype(np.float32) * delta, -rf, rf).astype(np.float32)
    return phi, vt, sgn, p


def marching_cubes_step(phi, origin, h: float, step: int, iso: float = 0.0,
                        normals: bool = False):
    """Marching cubes with mc_step (reading T2b): the plain extraction on
    phi[::step, ::step, ::step] with spacing fl32(step h)."""
    h32 = float(np.float32(h))
    hs = float(np.float32(h32 * step))
    o2 = tuple(float(np.float32(float(np.float32(o)) - (step - 1) * h32 / 2.0)) for o in origin)
    sub = np.ascontiguousarray(np.asarray(phi)[::step, ::step, ::step])
    return marching_cubes(sub, o2, hs, iso, normals=normals)


def lattice_gradient(phi):
    """Gradient of phi at every lattice point, float32 [nz, ny, nx, 3] in
    (x, y, z) order, phi per voxel (reading T6)."""
    phi = np.asarray(phi, dtype=np.float32)
    g = np.zeros(phi.shape + (3,), dtype=np.float32)
    half = np.float32(0.5)
    for a in range(3):
        k = 2 - a                                   # array axis of x, y, z
        n = phi.shape[k]
        if n < 2:
            continue
        f = np.moveaxis(phi, k, 0)
        d = np.zeros_like(f)
        d[1:n - 1] = (f[2:] - f[:n - 2]) * half
        d[0] = f[1] - f[0]
        d[n - 1] = f[n - 1] - f[n - 2]
        g[..., a] = np.moveaxis(d, 0, k)
    return g


def marching_cubes(phi, origin, h: float, iso: float = 0.0, normals: bool = False):
    """Mesh of phi at iso (reading T5): (verts float32 [nv, 3], tris int32
    [nt, 3]) in the canonical numbering; with normals=True also the vertex
    normals float32 [nv, 3] (reading T6)."""
    phi = np.asarray(phi, dtype=np.float32)
    nz, ny, nx = phi.shape
    isof = np.float32(iso)
    hf = np.float32(h)
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    cx = (o[0] + (np.arange(nx) + 0.5) * float(hf)).astype(np.float32)
    cy = (o[1] + (np.arange(ny) + 0.5) * float(hf)).astype(np.float32)
    cz = (o[2] + (np.arange(nz) + 0.5) * float(hf)).astype(np.float32)
    inside = phi < isof
    # vertices: crossed lattice edges numbered by (point, axis)
    n_pts = nx * ny * nz
    crossed = np.zeros((n_pts, 3), dtype=bool)
    ins = inside.ravel()
    flat = phi.ravel()
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    steps = (1, nx, nx * ny)
    limits = (ix < nx - 1, iy < ny - 1, iz < nz - 1)
    for axis in range(3):
        ok = limits[axis]
        idx = np.nonzero(ok)[0]
        crossed[idx, axis] = ins[idx] != ins[idx + steps[axis]]
    vid = np.full((n_pts, 3), -1, dtype=np.int64)
    order = np.nonzero(crossed.ravel())[0]
    vid.ravel()[order] = np.arange(order.size)
    pt, ax = order // 3, order % 3
    fa = flat[pt]
    fb = flat[pt + np.array(steps)[ax]]
    t = ((isof - fa) / (fb - fa)).astype(np.float32)
    verts = np.stack([cx[ix[pt]], cy[iy[pt]], cz[iz[pt]]], axis=1).astype(np.float32)
    moved = (verts[np.arange(pt.size), ax] + (t * hf).astype(np.float32)).astype(np.float32)
    verts[np.arange(pt.size), ax] = moved
    # triangles: cells numbered by their lowest lattice point
    tab = table()
    cell = np.nonzero(limits[0] & limits[1] & limits[2])[0]
    case = np.zeros(cell.size, dtype=np.int64)
    for k, (dx, dy, dz) in enumerate(CORNERS):
        case |= ins[cell + dx + dy * nx + dz * nx * ny].astype(np.int64) << k
    busy = (case != 0) & (case != 255)          # the other cases have no triangle
    cell, case = cell[busy], case[busy]
    tris = []
    for c, cs in zip(cell, case):
        for tri in tab[cs]:
            ids = []
            for e in tri:
                a, _, axis = EDGES[e]
                dx, dy, dz = CORNERS[a]
                ids.append(vid[c + dx + dy * nx + dz * nx * ny, axis])
            tris.append(ids)
    tris = np.array(tris, dtype=np.int32).reshape(-1, 3)
    if not normals:
        return verts, tris
    G = lattice_gradient(phi).reshape(-1, 3)
    w = (np.float32(1.0) - t).astype(np.float32)
    nrm = ((w[:, None] * G[pt]).astype(np.float32)
           + (t[:, None] * G[pt + np.array(steps)[ax]]).astype(np.float32)).astype(np.float32)
    l2 = ((nrm[:, 0] * nrm[:, 0] + nrm[:, 1] * nrm[:, 1]) + nrm[:, 2] * nrm[:, 2]).astype(np.float32)
    ln = np.sqrt(l2).astype(np.float32)
    ok = ln > 0
    nrm[ok] = (nrm[ok] / ln[ok, None]).astype(np.float32)
    nrm[~ok] = 0.0
    return verts, tris, nrm


U32 = 2.0 ** -24   # unit roundoff of float32


def marching_cubes_fp64(phi, origin, h: float, iso: float = 0.0):
    """Vertex positions and normals of the marching-cubes mesh of phi at iso
    by the definitions T5 and T6 in FP64 (same vertices and numbering as
    ``marching_cubes``), with per-vertex bounds on any float32 evaluation:

      verts [nv, 3], normals [nv, 3] (FP64), pos_tol [nv, 3], nrm_tol [nv]

    Position (T5): x = c_a + t h on the edge's axis, c_a elsewhere, with
    c_a = o + (i + 1/2) h and t = (iso - phi_a) / (phi_b - phi_a).  In float32
    c_a is one rounding from its exact value at most 1.01 u (|o| + 2 |c_a|)
    away (u = 2^-24; a product and a sum, or a correct rounding); t comes
    from two exact-input subtractions and a division, so
    |t32 - t| <= 3.01 u t; then x32 = c_a32 + t32 h adds the rounding of the
    product and the sum:
      |x32 - x| <= 1.01 u (|o| + 2 |c_a|) + 4.1 u h + 1.01 u |x|.
    Normal (T6): the float32 gradient differs from the exact difference of
    the float32 phi by at most u |g| per component; w = 1 - t by at most
    4.01 u, and the two products and the sum add three roundings, so
      |n32_k - n_k| <= 7.1 u (|g_a,k| + |g_b,k|),
    and the unit vector moves by at most 2 |dn| / |n| plus the rounding of
    the length and the division (6 u):
      |n32/|n32| - n/|n||_k <= 14.2 u |(|g_a| + |g_b|)| / |n| + 6 u.
    Where |n| = 0 the direction is undefined and the bound is +inf."""
    phi = np.asarray(phi, dtype=np.float32)
    nz, ny, nx = phi.shape
    isod = float(np.float32(iso))
    hd = float(np.float32(h))
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    inside = phi < np.float32(iso)
    n_pts = nx * ny * nz
    ins = inside.ravel()
    flat = phi.ravel().astype(np.float64)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    steps = (1, nx, nx * ny)
    limits = (ix < nx - 1, iy < ny - 1, iz < nz - 1)
    crossed = np.zeros((n_pts, 3), dtype=bool)
    for axis in range(3):
        idx = np.nonzero(limits[axis])[0]
        crossed[idx, axis] = ins[idx] != ins[idx + steps[axis]]
    order = np.nonzero(crossed.ravel())[0]
    pt, ax = order // 3, order % 3
    nb = pt + np.array(steps)[ax]
    fa, fb = flat[pt], flat[nb]
    t = (isod - fa) / (fb - fa)
    c = np.stack([o[0] + (ix[pt] + 0.5) * hd, o[1] + (iy[pt] + 0.5) * hd,
                  o[2] + (iz[pt] + 0.5) * hd], axis=1)
    x = c.copy()
    rows = np.arange(pt.size)
    x[rows, ax] = c[rows, ax] + t * hd
    moving = np.zeros_like(x, dtype=bool)
    moving[rows, ax] = True
    pos_tol = 1.01 * U32 * (np.abs(o)[None, :] + 2.0 * np.abs(c)) \
        + np.where(moving, 4.1 * U32 * hd + 1.01 * U32 * np.abs(x), 0.0)
    # normals: exact differences of the float32 phi
    G = np.zeros((nz, ny, nx, 3))
    p64 = phi.astype(np.float64)
    for a in range(3):
        k = 2 - a
        n = phi.shape[k]
        if n < 2:
            continue
        f = np.moveaxis(p64, k, 0)
        d = np.zeros_like(f)
        d[1:n - 1] = (f[2:] - f[:n - 2]) * 0.5
        d[0] = f[1] - f[0]
        d[n - 1] = f[n - 1] - f[n - 2]
        G[..., a] = np.moveaxis(d, 0, k)
    G = G.reshape(-1, 3)
    ga, gb = G[pt], G[nb]
    nvec = (1.0 - t)[:, None] * ga + t[:, None] * gb
    ln = np.linalg.norm(nvec, axis=1)
    ok = ln > 0
    nrm = np.zeros_like(nvec)
    nrm[ok] = nvec[ok] / ln[ok, None]
    spread = np.linalg.norm(np.abs(ga) + np.abs(gb), axis=1)
    nrm_tol = np.full(pt.size, np.inf)
    nrm_tol[ok] = 14.2 * U32 * spread[ok] / ln[ok] + 6.0 * U32
    return x, nrm, pos_tol, nrm_tol
