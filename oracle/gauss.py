"""FP64 CPU oracle for Gaussian-to-occupancy conversion -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product library never does, and the two share no
code.

What it computes is the definition of FGGS-LiDAR Sec. IV-A ("Grid query and
occupancy evaluation") on the Gaussian model of Sec. III-A, written out
directly, tile by tile, with numpy in FP64:

  w_i(x)   = exp(-1/2 (x - mu_i)^T Sigma_i^-1 (x - mu_i)),
             Sigma_i = R_i S_i S_i^T R_i^T                       (Sec. III-A)
  C_tile   = { G_i : b_i intersects B_tile }                     (tile culling)
  D(v)     = sum over G_i in C_tile(v) of w_i(v) * alpha_i^2     (density)
  V_occ    = [ D(v) > theta ]                                    (threshold)
  Int      = AND of V_occ over the 6-neighbourhood and the voxel itself
  Surf     = V_occ AND NOT Int                                   (surface mask)

The culling set is found by testing every Gaussian box against every tile box
(no hierarchy): the LBVH of Sec. IV-A only accelerates this query, it does not
change its answer.

Readings taken where the paper is silent (each is also listed in the design
notes):

  G1  Parameters: mean mu (xyz), rotation as a quaternion (w, x, y, z) that
      need not be normalised (R is the rotation of q/|q|), linear scales
      s > 0 (S = diag(s)) and opacity alpha in [0, 1].
  G2  Gaussian box b_i: the exact axis-aligned box of the k-sigma ellipsoid
      (x - mu)^T Sigma^-1 (x - mu) <= k^2, i.e. mu +- k sqrt(diag Sigma);
      k = 3 by default.  Membership in C_tile is a floating-point decision,
      so both this oracle and the GPU evaluate the box in FP64 in one fixed
      operation order (``gauss_boxes``) and round each end to the nearest
      float32; the tile test then compares float32 values exactly.
  G3  Voxel (i, j, k) is the cell o + [i, i+1] x [j, j+1] x [k, k+1] * h; its
      centre is v = o + (i + 1/2, j + 1/2, k + 1/2) h.
  G4  Tile (tx, ty, tz) holds voxels tB <= i < min((t+1)B, n) on each axis;
      B_tile is the closed box spanned by those cells, each end evaluated in
      FP64 and rounded to the nearest float32.
  G5  Boxes are closed: touching counts as intersecting.
  G6  In Int, neighbours outside the grid count as unoccupied, so occupied
      voxels on the grid boundary are surface voxels.
  G7  The threshold is strict, as printed: D = theta is unoccupied.

Layouts: voxel arrays are [nz][ny][nx] (x fastest); tile arrays
[tz][ty][tx].
"""
from __future__ import annotations

import math

import numpy as np

LOG2E = 1.0 / math.log(2.0)


def _rotation_terms(quats):
    """R of q/|q| for quaternions (w, x, y, z), FP64, in the fixed operation
    order that also defines the Gaussian boxes (reading G2)."""
    q = np.asarray(quats, dtype=np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    n = ((w * w + x * x) + y * y) + z * z
    s = 2.0 / n
    R = np.empty((q.shape[0], 3, 3), dtype=np.float64)
    R[:, 0, 0] = 1.0 - s * (y * y + z * z)
    R[:, 0, 1] = s * (x * y - w * z)
    R[:, 0, 2] = s * (x * z + w * y)
    R[:, 1, 0] = s * (x * y + w * z)
    R[:, 1, 1] = 1.0 - s * (x * x + z * z)
    R[:, 1, 2] = s * (y * z - w * x)
    R[:, 2, 0] = s * (x * z - w * y)
    R[:, 2, 1] = s * (y * z + w * x)
    R[:, 2, 2] = 1.0 - s * (x * x + y * y)
    return R


def rotation_matrices(quats):
    """R_i (Sec. III-A) for each quaternion, FP64 [N, 3, 3]."""
    return _rotation_terms(quats)


def gauss_boxes(means, quats, scales, k: float = 3.0):
    """Gaussian boxes b_i (reading G2), float32 [N, 6] = lo xyz, hi xyz.

    Half-extent on axis a: e_a = k * sqrt(Sigma_aa) with
    Sigma_aa = sum_j (R_aj s_j)^2, accumulated as ((c0^2 + c1^2) + c2^2);
    every step is one IEEE FP64 operation, then mu -+ e is rounded to the
    nearest float32."""
    mu = np.asarray(means, dtype=np.float32).astype(np.float64)
    sc = np.asarray(scales, dtype=np.float32).astype(np.float64)
    kk = float(np.float32(k))
    R = _rotation_terms(np.asarray(quats, dtype=np.float32))
    out = np.empty((mu.shape[0], 6), dtype=np.float32)
    for a in range(3):
        c0 = R[:, a, 0] * sc[:, 0]
        c1 = R[:, a, 1] * sc[:, 1]
        c2 = R[:, a, 2] * sc[:, 2]
        saa = (c0 * c0 + c1 * c1) + c2 * c2
        e = kk * np.sqrt(saa)
        out[:, a] = (mu[:, a] - e).astype(np.float32)
        out[:, 3 + a] = (mu[:, a] + e).astype(np.float32)
    return out


class Grid:
    """Voxel grid of Sec. IV-A: origin o, spacing h, dims (nx, ny, nz), tile
    edge B (voxels), density threshold theta."""

    def __init__(self, origin, h, dims, tile=8, theta=0.5):
        self.origin = np.asarray(origin, dtype=np.float32)
        self.h = np.float32(h)
        self.dims = tuple(int(d) for d in dims)
        self.tile = int(tile)
        self.theta = np.float32(theta)

    @property
    def tiles(self):
        B = self.tile
        return tuple((n + B - 1) // B for n in self.dims)

    def tile_box(self, t):
        """B_tile of tile t = (tx, ty, tz) (readings G3, G4), float32 [6]."""
        B = self.tile
        lo = np.empty(3, dtype=np.float32)
        hi = np.empty(3, dtype=np.float32)
        for a in range(3):
            i0 = t[a] * B
            i1 = min(i0 + B, self.dims[a])
            o = float(self.origin[a])
            h = float(self.h)
            lo[a] = np.float32(o + i0 * h)
            hi[a] = np.float32(o + i1 * h)
        return np.concatenate([lo, hi])

    def tile_voxels(self, t):
        """Index ranges (per axis) of the voxels of tile t."""
        B = self.tile
        return [(t[a] * B, min(t[a] * B + B, self.dims[a])) for a in range(3)]

    def centres(self, ix, iy, iz):
        """Voxel centres (reading G3), FP64, for index vectors."""
        o = self.origin.astype(np.float64)
        h = float(self.h)
        return (o[0] + (np.asarray(ix) + 0.5) * h,
                o[1] + (np.asarray(iy) + 0.5) * h,
                o[2] + (np.asarray(iz) + 0.5) * h)


def tile_members(boxes, tbox):
    """Indices of the Gaussians whose box meets the closed tile box (the
    culling set C_tile; reading G5).  float32 comparisons, exact."""
    b = np.asarray(boxes, dtype=np.float32)
    m = np.ones(b.shape[0], dtype=bool)
    for a in range(3):
        m &= (b[:, a] <= tbox[3 + a]) & (b[:, 3 + a] >= tbox[a])
    return np.nonzero(m)[0]


def tile_counts(boxes, grid: Grid):
    """|C_tile| for every tile, int64 [tz][ty][tx]."""
    tx, ty, tz = grid.tiles
    out = np.zeros((tz, ty, tx), dtype=np.int64)
    for k in range(tz):
        for j in range(ty):
            for i in range(tx):
                out[k, j, i] = tile_members(boxes, grid.tile_box((i, j, k))).size
    return out


def _terms(pts, mu, R, sc, al):
    """w_i(v) alpha_i^2 for points pts [V, 3] and Gaussians (FP64), plus the
    whitened coordinates u = S^-1 R^T (v - mu) [V, K, 3] and q = |u|^2."""
    d = pts[:, None, :] - mu[None, :, :]                       # [V, K, 3]
    u = np.einsum("vka,kab->vkb", d, R) / sc[None, :, :]       # (R^T d)_b / s_b
    q = np.sum(u * u, axis=2)                                  # d^T Sigma^-1 d
    t = np.exp(-0.5 * q) * (al * al)[None, :]
    return t, u, q


def density(params, grid: Grid, k: float = 3.0, with_error: bool = False):
    """D(v) for every voxel (FP64 [nz][ny][nx]) and |C_tile| per tile.

    params = (means [N,3], quats [N,4], scales [N,3], opacity [N]), float32.
    With ``with_error`` also returns E(v), the error scale of an FP32
    evaluation in tile-local coordinates:
        E(v) = sum_i t_i (1 + q_i + sum_b |u_ib| L_i / s_ib),
    t_i = w_i(v) alpha_i^2, L_i = the tile diagonal + |v - mu_i|.  An FP32
    evaluation of one term has relative error of order 2^-24 times
    (1 + q + sum_b |u_b| L / s_b): the whitened coordinates u_b carry the
    rounding of positions of size L divided by the scale s_b, and the
    exponent multiplies relative errors of q by q."""
    means, quats, scales, opac = params
    mu = np.asarray(means, dtype=np.float32).astype(np.float64)
    sc = np.asarray(scales, dtype=np.float32).astype(np.float64)
    al = np.asarray(opac, dtype=np.float32).astype(np.float64)
    R = rotation_matrices(np.asarray(quats, dtype=np.float32))
    boxes = gauss_boxes(means, quats, scales, k)
    nx, ny, nz = grid.dims
    D = np.zeros((nz, ny, nx), dtype=np.float64)
    E = np.zeros((nz, ny, nx), dtype=np.float64) if with_error else None
    tx, ty, tz = grid.tiles
    counts = np.zeros((tz, ty, tx), dtype=np.int64)
    diag = math.sqrt(3.0) * grid.tile * float(grid.h)
    for kt in range(tz):
        for jt in range(ty):
            for it in range(tx):
                t = (it, jt, kt)
                mem = tile_members(boxes, grid.tile_box(t))
                counts[kt, jt, it] = mem.size
                if mem.size == 0:
                    continue
                (x0, x1), (y0, y1), (z0, z1) = grid.tile_voxels(t)
                iz, iy, ix = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1),
                                         np.arange(x0, x1), indexing="ij")
                cx, cy, cz = grid.centres(ix.ravel(), iy.ravel(), iz.ravel())
                pts = np.stack([cx, cy, cz], axis=1)
                terms, u, q = _terms(pts, mu[mem], R[mem], sc[mem], al[mem])
                D[z0:z1, y0:y1, x0:x1] = terms.sum(axis=1).reshape(iz.shape)
                if with_error:
                    dist = np.linalg.norm(pts[:, None, :] - mu[mem][None], axis=2)
                    L = diag + dist
                    g = np.sum(np.abs(u) / sc[mem][None], axis=2) * L
                    E[z0:z1, y0:y1, x0:x1] = np.sum(
                        terms * (1.0 + q + g), axis=1).reshape(iz.shape)
    if with_error:
        return D, counts, E
    return D, counts


def density_at(params, grid: Grid, voxels, k: float = 3.0):
    """D(v) and E(v) (see ``density``) at the voxels [M, 3] = (i, j, k) only,
    with each voxel's own tile culling set; FP64.  Also returns |C_tile| of
    each voxel's tile.  For spot checks of large grids."""
    means, quats, scales, opac = params
    mu = np.asarray(means, dtype=np.float32).astype(np.float64)
    sc = np.asarray(scales, dtype=np.float32).astype(np.float64)
    al = np.asarray(opac, dtype=np.float32).astype(np.float64)
    R = rotation_matrices(np.asarray(quats, dtype=np.float32))
    boxes = gauss_boxes(means, quats, scales, k)
    vox = np.asarray(voxels, dtype=np.int64)
    B = grid.tile
    D = np.zeros(vox.shape[0])
    E = np.zeros(vox.shape[0])
    K = np.zeros(vox.shape[0], dtype=np.int64)
    diag = math.sqrt(3.0) * B * float(grid.h)
    tiles = vox // B
    order = np.lexsort((tiles[:, 0], tiles[:, 1], tiles[:, 2]))
    start = 0
    while start < order.size:
        t = tuple(tiles[order[start]])
        end = start
        while end < order.size and tuple(tiles[order[end]]) == t:
            end += 1
        sel = order[start:end]
        mem = tile_members(boxes, grid.tile_box(t))
        K[sel] = mem.size
        if mem.size:
            cx, cy, cz = grid.centres(vox[sel, 0], vox[sel, 1], vox[sel, 2])
            pts = np.stack([cx, cy, cz], axis=1)
            terms, u, q = _terms(pts, mu[mem], R[mem], sc[mem], al[mem])
            D[sel] = terms.sum(axis=1)
            dist = np.linalg.norm(pts[:, None, :] - mu[mem][None], axis=2)
            g = np.sum(np.abs(u) / sc[mem][None], axis=2) * (diag + dist)
            E[sel] = np.sum(terms * (1.0 + q + g), axis=1)
        start = end
    return D, E, K


def occupancy(D, theta):
    """V_occ = [D > theta] (threshold equation, reading G7), uint8."""
    return (np.asarray(D) > theta).astype(np.uint8)


def surface(occ):
    """Surf = V_occ AND NOT Int, Int = V_occ on the voxel and all six face
    neighbours (readings G6: outside the grid is unoccupied), uint8."""
    o = np.asarray(occ).astype(bool)
    p = np.pad(o, 1, mode="constant", constant_values=False)
    c = p[1:-1, 1:-1, 1:-1]
    interior = (c & p[:-2, 1:-1, 1:-1] & p[2:, 1:-1, 1:-1]
                & p[1:-1, :-2, 1:-1] & p[1:-1, 2:, 1:-1]
                & p[1:-1, 1:-1, :-2] & p[1:-1, 1:-1, 2:])
    return (o & ~interior).astype(np.uint8)


def voxelize(params, grid: Grid, k: float = 3.0):
    """The whole conversion: (D, V_occ, Surf, |C_tile|)."""
    D, counts = density(params, grid, k)
    occ = occupancy(D, grid.theta)
    return D, occ, surface(occ), counts
