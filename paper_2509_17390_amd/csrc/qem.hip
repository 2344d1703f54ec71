// qem.hip -- quadric-error decimation by rounds of parallel edge
// contraction on gfx950 (FGGS-LiDAR Sec. IV-B "Mesh optimization":
// quadric-error decimation to a face ratio; Sec. V: ratio 0.1, three
// rounds, boundary protected).
//
// The quadric error metric is Garland and Heckbert's (1997): a vertex
// carries the sum of the squared-distance quadrics of its faces' planes, an
// edge (u, v) contracts to the point x* minimising x^T (Q_u + Q_v) x at that
// minimum's cost, cheapest first.  One contraction at a time is sequential;
// here a step contracts an independent set of locally cheapest edges at
// once, so the work of a step is data-parallel over vertices, edges and
// faces:
//
//   round k = 1..R runs until at most ceil(F0 ratio^(k/R)) faces remain (or
//   nothing can contract); at its start the plane quadrics are summed anew
//   and the vertices on a boundary or non-manifold edge (an edge not on
//   exactly two faces) are protected for the round.  One step:
//   1. incidence from the live faces: each vertex's faces (ascending) and
//      its distinct neighbours (ascending); edges (u < v) numbered in
//      lexicographic order by a scan of the neighbour counts above u;
//   2. candidates: edges on exactly two faces, both ends unprotected,
//      exactly two common neighbours (the link condition, so a closed
//      manifold stays closed and manifold); x* is A^-1 b by Cramer's rule
//      when A (the 3x3 block of Q_u + Q_v) is well conditioned and x* lies
//      near the edge, else the cheapest of the ends and the midpoint; an
//      edge whose contraction would flip a face is dropped; key = (float32
//      cost, pi(edge number)) with pi a fixed bijection of 32-bit integers,
//      so exactly equal costs (flat regions) are ordered pseudo-randomly
//      and the locally cheapest edges are many, not one per flat region;
//   3. the ceil((F - T) / 2) smallest keys are eligible (a radix select of
//      the threshold key; an interior contraction removes two faces);
//   4. an eligible edge contracts when no eligible edge at any vertex of
//      its two closed one-rings has a smaller key (per-vertex 64-bit atomic
//      minima); no end of such an edge is an end or a neighbour of an end
//      of another, so their contractions touch disjoint faces and run in
//      place;
//   5. faces are renamed through the contraction map; the two faces of
//      each contracted edge degenerate and are dropped.
// A step changes the mesh only inside the closed one-rings of the edges it
// contracts: the next step rebuilds the incidence and evaluates the edges
// of those ("dirty") vertices alone, and every other edge keeps its cost
// and point under its new number.
// Positions, quadrics and costs are FP64 throughout, each operation in a
// fixed order (compiled with -ffp-contract=off), so a run is deterministic
// and matches a plain CPU evaluation of the same steps; positions are
// rounded to float32 once, at the end.
#include "mesh_internal.h"

#include <float.h>
#include <math.h>
#include <stddef.h>

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kNone = ~0ull;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Adds v of every thread of the block to *dst with one atomic: a
// shuffle-reduction per wave, then the waves' sums through LDS (a counter
// that every thread of a large launch hit directly serialised the launch).
// Every thread of the block must call it.
__device__ __forceinline__ void block_add(uint32_t v, uint32_t *dst)
{
    __shared__ uint32_t part[kBlock / 64];
    __syncthreads();   // an earlier call's sum is read before part is reused
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        if (t) atomicAdd(dst, t);
    }
}

// pi: "lowbias32" of C. Wellons' hash prospector (xorshift-multiply rounds,
// each invertible mod 2^32, so pi is a bijection and keys stay unique)
__device__ __forceinline__ uint32_t perm32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// n = (b - a) x (c - a)
__device__ __forceinline__ void face_normal(const double a[3], const double b[3],
                                            const double c[3], double n[3])
{
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    cross3(e1, e2, n);
}

__device__ __forceinline__ void load3(const double *__restrict__ P, int i, double r[3])
{
    r[0] = P[3 * (int64_t)i];
    r[1] = P[3 * (int64_t)i + 1];
    r[2] = P[3 * (int64_t)i + 2];
}

// Plane quadric K = q q^T / (n.n) of a face, q = (n, -n.a), upper triangle
// row by row: (00 01 02 03 11 12 13 22 23 33); zero for a degenerate face.
__device__ void plane_quadric(const double a[3], const double b[3], const double c[3],
                              double K[10])
{
    double n[3];
    face_normal(a, b, c, n);
    const double nn = dot3(n, n);
    if (nn == 0.0) {
        for (int i = 0; i < 10; ++i) K[i] = 0.0;
        return;
    }
    const double q[4] = {n[0], n[1], n[2], -dot3(n, a)};
    int k = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) K[k++] = (q[i] * q[j]) / nn;
}

// [x 1] Q [x 1]^T
__device__ __forceinline__ double quadric_cost(const double Q[10], const double x[3])
{
    const double r0 = ((Q[0] * x[0] + Q[1] * x[1]) + Q[2] * x[2]) + Q[3];
    const double r1 = ((Q[1] * x[0] + Q[4] * x[1]) + Q[5] * x[2]) + Q[6];
    const double r2 = ((Q[2] * x[0] + Q[5] * x[1]) + Q[7] * x[2]) + Q[8];
    const double r3 = ((Q[3] * x[0] + Q[6] * x[1]) + Q[8] * x[2]) + Q[9];
    return ((x[0] * r0 + x[1] * r1) + x[2] * r2) + r3;
}

// x* = A^-1 b by Cramer's rule (cofactors along the first row) when
// trace(A) > 0 and |det A| > 1e-6 (trace / 3)^3; false otherwise.
__device__ bool minimiser(const double Q[10], double x[3])
{
    const double a00 = Q[0], a01 = Q[1], a02 = Q[2], b0 = -Q[3];
    const double a11 = Q[4], a12 = Q[5], b1 = -Q[6];
    const double a22 = Q[7], b2 = -Q[8];
    const double det = (a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02)) +
                       a02 * (a01 * a12 - a11 * a02);
    const double tr = (a00 + a11) + a22;
    const double t3 = tr / 3.0;
    if (!(tr > 0.0 && fabs(det) > 1e-6 * ((t3 * t3) * t3))) return false;
    x[0] = ((b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2)) +
            a02 * (b1 * a12 - a11 * b2)) / det;
    x[1] = ((a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02)) +
            a02 * (a01 * b2 - b1 * a02)) / det;
    x[2] = ((a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02)) +
            b0 * (a01 * a12 - a11 * a02)) / det;
    return true;
}

// Placement of an edge's contraction and its cost: x* when it lies within
// twice the edge length of the midpoint m, else the cheapest of pu, pv, m
// (the first on a tie).
__device__ double placement(const double Q[10], const double pu[3], const double pv[3],
                            double x[3])
{
    const double m[3] = {0.5 * (pu[0] + pv[0]), 0.5 * (pu[1] + pv[1]), 0.5 * (pu[2] + pv[2])};
    bool ok = minimiser(Q, x);
    if (ok) {
        const double dx[3] = {x[0] - m[0], x[1] - m[1], x[2] - m[2]};
        const double e[3] = {pv[0] - pu[0], pv[1] - pu[1], pv[2] - pu[2]};
        ok = dot3(dx, dx) <= 4.0 * dot3(e, e);
    }
    if (!ok) {
        // the cheapest of pu, pv, m; the first on a tie
        const double cu = quadric_cost(Q, pu), cv = quadric_cost(Q, pv), cm = quadric_cost(Q, m);
        const bool tv = cv < cu;
        const double cb = tv ? cv : cu;
        const bool tm = cm < cb;
        for (int i = 0; i < 3; ++i) x[i] = tm ? m[i] : (tv ? pv[i] : pu[i]);
    }
    return quadric_cost(Q, x);
}

__global__ __launch_bounds__(kBlock) void k_qem_init(const float *__restrict__ verts, int64_t nv,
                                                     const int32_t *__restrict__ tris, int64_t nt,
                                                     double *__restrict__ P,
                                                     int32_t *__restrict__ F)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nv)
        for (int k = 0; k < 3; ++k) P[3 * i + k] = (double)verts[3 * i + k];
    if (i < nt) {
        const int32_t a = tris[3 * i], b = tris[3 * i + 1], c = tris[3 * i + 2];
        // a face with a repeated corner is no triangle: dropped at once
        const bool dead = a == b || b == c || a == c;
        F[3 * i] = dead ? -1 : a;
        F[3 * i + 1] = b;
        F[3 * i + 2] = c;
    }
}

__global__ __launch_bounds__(kBlock) void k_qem_fill_faces(const int32_t *__restrict__ F,
                                                           int64_t nt, uint32_t *__restrict__ fcnt,
                                                           int32_t *__restrict__ fl,
                                                           uint32_t *__restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt || F[3 * t] < 0) return;
    for (int k = 0; k < 3; ++k) {
        const int32_t v = F[3 * t + k];
        const uint32_t s = atomicAdd(&fcnt[v], 1u);
        if (s < (uint32_t)kQemFaces) fl[(int64_t)v * kQemFaces + s] = (int32_t)t;
        else atomicOr(&flags[0], 1u);
    }
}

__device__ __forceinline__ bool face_has(const int32_t *__restrict__ F, int32_t t, int32_t w)
{
    return F[3 * (int64_t)t] == w || F[3 * (int64_t)t + 1] == w || F[3 * (int64_t)t + 2] == w;
}

// The distinct neighbours of v (ascending) from its n faces f into b;
// returns their number (at most kQemNbrs, else flags[0] |= 2).
__device__ int build_ring(const int32_t *__restrict__ F, const int32_t *f, int n, int64_t v,
                          int32_t *b, uint32_t *__restrict__ flags)
{
    int m = 0;
    for (int k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) {
            const int32_t w = F[3 * (int64_t)f[k] + c];
            if (w == (int32_t)v) continue;
            int j = m;
            while (j > 0 && b[j - 1] > w) --j;
            if (j > 0 && b[j - 1] == w) continue;
            if (m == kQemNbrs) {
                atomicOr(&flags[0], 2u);
                continue;
            }
            for (int i = m; i > j; --i) b[i] = b[i - 1];
            b[j] = w;
            ++m;
        }
    return m;
}

// Per vertex: sort its faces, collect its distinct neighbours (ascending),
// count those above it; at a round's start also sum its faces' plane
// quadrics (ascending face order) and protect it when an edge at it is not
// on exactly two faces.
__global__ __launch_bounds__(kBlock) void k_qem_vertex(const double *__restrict__ P,
                                                       const int32_t *__restrict__ F, int64_t nv,
                                                       const uint32_t *__restrict__ fcnt,
                                                       int32_t *__restrict__ fl,
                                                       int32_t *__restrict__ fdeg,
                                                       int32_t *__restrict__ nb,
                                                       int32_t *__restrict__ ndeg,
                                                       uint32_t *__restrict__ nlarge,
                                                       double *__restrict__ Q,
                                                       uint8_t *__restrict__ prot,
                                                       int round_start,
                                                       int32_t *__restrict__ absorbed,
                                                       uint32_t *__restrict__ flags)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    absorbed[v] = -1;
    const int n = fcnt[v] < (uint32_t)kQemFaces ? (int)fcnt[v] : kQemFaces;
    int32_t *f = fl + v * kQemFaces;
    for (int k = 1; k < n; ++k) {
        const int32_t x = f[k];
        int j = k;
        while (j > 0 && f[j - 1] > x) {
            f[j] = f[j - 1];
            --j;
        }
        f[j] = x;
    }
    fdeg[v] = n;
    int32_t *b = nb + v * kQemNbrs;
    const int m = build_ring(F, f, n, v, b, flags);
    ndeg[v] = m;
    uint32_t above = 0;
    for (int k = 0; k < m; ++k) above += b[k] > (int32_t)v ? 1u : 0u;
    nlarge[v] = above;
    if (!round_start) return;
    double acc[10];
    for (int i = 0; i < 10; ++i) acc[i] = 0.0;
    for (int k = 0; k < n; ++k) {
        const int64_t t = f[k];
        double pa[3], pb[3], pc[3], K[10];
        load3(P, F[3 * t], pa);
        load3(P, F[3 * t + 1], pb);
        load3(P, F[3 * t + 2], pc);
        plane_quadric(pa, pb, pc, K);
        for (int i = 0; i < 10; ++i) acc[i] = acc[i] + K[i];
    }
    for (int i = 0; i < 10; ++i) Q[10 * v + i] = acc[i];
    uint8_t p = 0;
    for (int k = 0; k < m && !p; ++k) {
        int cnt = 0;
        for (int i = 0; i < n; ++i) cnt += face_has(F, f[i], b[k]) ? 1 : 0;
        p = cnt != 2 ? 1 : 0;
    }
    prot[v] = p;
}

// Between a round's steps, per dirty vertex: its live faces are those of
// its previous list still alive (a contraction renames faces, it never
// adds a face to a vertex it did not touch), plus, for the u of a
// contracted edge (u, v), the live faces of v's list, merged in ascending
// order; then its neighbours anew.  v itself is left to u's thread, which
// empties v's lists after reading them.
__global__ __launch_bounds__(kBlock) void k_qem_vertex_update(
    const int32_t *__restrict__ F, int64_t nv, const uint8_t *__restrict__ dirty,
    const int32_t *__restrict__ remap, int32_t *__restrict__ absorbed, int32_t *__restrict__ fl,
    int32_t *__restrict__ fdeg, int32_t *__restrict__ nb, int32_t *__restrict__ ndeg,
    uint32_t *__restrict__ nlarge, uint32_t *__restrict__ flags)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv || !dirty[v] || remap[v] >= 0) return;
    int32_t *f = fl + v * kQemFaces;
    const int n0 = fdeg[v];
    int a = 0;
    for (int k = 0; k < n0; ++k) {
        const int32_t t = f[k];
        if (F[3 * (int64_t)t] >= 0) f[a++] = t;
    }
    int n = a;
    const int32_t w = absorbed[v];
    if (w >= 0) {
        absorbed[v] = -1;
        const int32_t *g = fl + (int64_t)w * kQemFaces;
        const int m0 = fdeg[w];
        int nb_live = 0;
        for (int k = 0; k < m0; ++k) nb_live += F[3 * (int64_t)g[k]] >= 0 ? 1 : 0;
        if (a + nb_live > kQemFaces) {
            atomicOr(&flags[0], 1u);
        } else {
            // merge from the top: v's own list sits at the front of the
            // destination, so no entry is overwritten before it is read
            int i = a - 1, j = m0 - 1;
            for (int o = a + nb_live - 1; o > i; --o) {
                while (F[3 * (int64_t)g[j]] < 0) --j;
                if (i < 0 || g[j] > f[i]) f[o] = g[j--];
                else f[o] = f[i--];
            }
            n = a + nb_live;
        }
        fdeg[w] = 0;
        ndeg[w] = 0;
        nlarge[w] = 0;
    }
    fdeg[v] = n;
    int32_t *b = nb + v * kQemNbrs;
    const int m = build_ring(F, f, n, v, b, flags);
    ndeg[v] = m;
    uint32_t above = 0;
    for (int k = 0; k < m; ++k) above += b[k] > (int32_t)v ? 1u : 0u;
    nlarge[v] = above;
}

// Candidate test of the edge (u, v): true with the contraction point x and
// the float32 cost bits when the edge may contract (readings of the header
// comment).
__device__ bool edge_candidate(const double *__restrict__ P, const int32_t *__restrict__ F,
                               const int32_t *__restrict__ fl, const int32_t *__restrict__ fdeg,
                               const int32_t *__restrict__ nb, const int32_t *__restrict__ ndeg,
                               const double *__restrict__ Q, const uint8_t *__restrict__ prot,
                               int64_t u, int32_t v, int nu, int fu, double x[3],
                               uint32_t *cbits)
{
    const int32_t *bu = nb + u * kQemNbrs;
    const int32_t *lu = fl + u * kQemFaces;
    int fc = 0;
    for (int i = 0; i < fu; ++i) fc += face_has(F, lu[i], v) ? 1 : 0;
    if (fc != 2 || prot[u] || prot[v]) return false;
    // link condition: exactly two common neighbours
    const int32_t *bv = nb + (int64_t)v * kQemNbrs;
    const int nvv = ndeg[v];
    int i = 0, j = 0, common = 0;
    while (i < nu && j < nvv) {
        if (bu[i] < bv[j]) ++i;
        else if (bu[i] > bv[j]) ++j;
        else { ++common; ++i; ++j; }
    }
    if (common != 2) return false;
    double Qe[10], pu[3], pv[3];
    for (int q = 0; q < 10; ++q) Qe[q] = Q[10 * u + q] + Q[10 * (int64_t)v + q];
    load3(P, (int32_t)u, pu);
    load3(P, v, pv);
    const double c = placement(Qe, pu, pv, x);
    // no face of u or v (other than the two on the edge) may flip
    for (int side = 0; side < 2; ++side) {
        const int64_t w = side == 0 ? u : (int64_t)v;
        const int32_t *lw = fl + w * kQemFaces;
        const int fw = fdeg[w];
        for (int i2 = 0; i2 < fw; ++i2) {
            const int64_t t = lw[i2];
            const int32_t c0 = F[3 * t], c1 = F[3 * t + 1], c2 = F[3 * t + 2];
            const bool hu = c0 == (int32_t)u || c1 == (int32_t)u || c2 == (int32_t)u;
            const bool hv = c0 == v || c1 == v || c2 == v;
            if (hu && hv) continue;
            double a[3], b[3], cc[3], n0[3], n1[3];
            load3(P, c0, a);
            load3(P, c1, b);
            load3(P, c2, cc);
            face_normal(a, b, cc, n0);
            if (!(dot3(n0, n0) > 0.0)) continue;
            // the corner at u or v moves to x (selects, not a pointer, so
            // the corners stay in registers)
            const bool m0 = c0 == (int32_t)u || c0 == v;
            const bool m1 = !m0 && (c1 == (int32_t)u || c1 == v);
            const bool m2 = !m0 && !m1;
            for (int q = 0; q < 3; ++q) {
                a[q] = m0 ? x[q] : a[q];
                b[q] = m1 ? x[q] : b[q];
                cc[q] = m2 ? x[q] : cc[q];
            }
            face_normal(a, b, cc, n1);
            if (!(dot3(n0, n1) > 0.0)) return false;
        }
    }
    // cost clamped at 0 (a NaN stays) and rounded to float32; -0 and +0
    // share one key
    const double cl = 0.0 > c ? 0.0 : c;
    float c32 = (float)cl;
    if (c32 == 0.0f) c32 = 0.0f;
    *cbits = __float_as_uint(c32);
    return true;
}

// Per vertex u with a dirty end role (every vertex at a round's start, else
// the dirty ones): every edge (u, v > u) in ascending v, numbered from
// eoff[u], is marked for k_qem_eval (cand = 2).
__global__ __launch_bounds__(kBlock) void k_qem_edges(int64_t nv, const int32_t *__restrict__ nb,
                                                      const int32_t *__restrict__ ndeg,
                                                      const uint32_t *__restrict__ eoff,
                                                      const uint8_t *__restrict__ dirty, int full,
                                                      uint8_t *__restrict__ cand,
                                                      int32_t *__restrict__ eu,
                                                      int32_t *__restrict__ ev)
{
    const int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (u >= nv || !(full || dirty[u])) return;
    const int nu = ndeg[u];
    const int32_t *bu = nb + u * kQemNbrs;
    uint32_t e = eoff[u];
    for (int k = 0; k < nu; ++k) {
        const int32_t v = bu[k];
        if (v <= (int32_t)u) continue;
        eu[e] = (int32_t)u;
        ev[e] = v;
        cand[e] = 2;
        ++e;
    }
}

// One thread per edge of the previous step whose lower end u is clean:
// u's edges are the same, in the same order, so the edge moves from its
// previous number to e - eoff_old[u] + eoff[u].  With v clean too its
// result is unchanged (its ends, their faces, neighbours, positions and
// quadrics are all as before) and only the key's low word becomes pi of
// the new number; with v dirty it is marked for k_qem_eval.
__global__ __launch_bounds__(kBlock) void k_qem_carry(
    int64_t n_old, const int32_t *__restrict__ eu_old, const int32_t *__restrict__ ev_old,
    const uint8_t *__restrict__ dirty, const uint32_t *__restrict__ eoff,
    const uint32_t *__restrict__ eoff_old, const uint64_t *__restrict__ key_old,
    const uint8_t *__restrict__ cand_old, const double *__restrict__ X_old,
    uint64_t *__restrict__ key, uint8_t *__restrict__ cand, double *__restrict__ X,
    int32_t *__restrict__ eu, int32_t *__restrict__ ev, uint32_t *__restrict__ counters)
{
    const int64_t eo = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t found = 0;
    if (eo < n_old) {
        const int32_t u = eu_old[eo];
        if (!dirty[u]) {
            const int32_t v = ev_old[eo];
            const uint32_t e = (uint32_t)eo - eoff_old[u] + eoff[u];
            eu[e] = u;
            ev[e] = v;
            if (dirty[v]) {
                cand[e] = 2;
            } else if (cand_old[eo]) {
                for (int q = 0; q < 3; ++q) X[3 * (int64_t)e + q] = X_old[3 * eo + q];
                key[e] = (key_old[eo] & 0xffffffff00000000ull) | perm32(e);
                cand[e] = 1;
                found = 1;
            } else {
                key[e] = kNone;
                cand[e] = 0;
            }
        }
    }
    block_add(found, &counters[0]);
}

// One thread per edge marked by k_qem_edges: the candidate test, its key
// (float32 cost bits, pi(e)) or "none", and its point.
__global__ __launch_bounds__(kBlock) void k_qem_eval(
    const double *__restrict__ P, const int32_t *__restrict__ F, int64_t n,
    const int32_t *__restrict__ fl, const int32_t *__restrict__ fdeg,
    const int32_t *__restrict__ nb, const int32_t *__restrict__ ndeg,
    const double *__restrict__ Q, const uint8_t *__restrict__ prot,
    const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
    uint64_t *__restrict__ key, uint8_t *__restrict__ cand, double *__restrict__ X,
    uint32_t *__restrict__ counters)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t found = 0;
    if (e < n && cand[e] == 2) {
        const int64_t u = eu[e];
        const int32_t v = ev[e];
        double x[3];
        uint32_t cbits = 0;
        const bool c = edge_candidate(P, F, fl, fdeg, nb, ndeg, Q, prot, u, v, ndeg[u], fdeg[u],
                                      x, &cbits);
        if (c) {
            for (int q = 0; q < 3; ++q) X[3 * e + q] = x[q];
            found = 1;
        }
        key[e] = c ? ((uint64_t)cbits << 32) | perm32((uint32_t)e) : kNone;
        cand[e] = c ? 1 : 0;
    }
    block_add(found, &counters[0]);
}

// Radix select of the rank-th smallest key (1-based), one byte per pass
// from the top: sel = {prefix, mask, rank}; after the eight passes prefix
// holds the selected key.
struct SelState {
    unsigned long long prefix, mask;
    unsigned long long rank;
    unsigned long long all;   // every key is eligible: the passes do nothing
};
static_assert(offsetof(SelState, prefix) == 0, "the selected key is read at offset 0");

__global__ __launch_bounds__(kBlock) void k_qem_hist(const uint64_t *__restrict__ key, int64_t n,
                                                     const SelState *__restrict__ st, int shift,
                                                     uint32_t *__restrict__ hist)
{
    if (st->all) return;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint64_t k = key[i];
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// The digit holding the rank-th key: the first d whose inclusive count
// reaches rank (digit 255 takes any rest), by a scan of the 256 counts in
// LDS, one thread per digit; the counts are cleared for the next pass.
__global__ __launch_bounds__(256) void k_qem_pick(SelState *st, uint32_t *hist, int shift)
{
    if (st->all) return;
    __shared__ unsigned long long c[256];
    const int i = threadIdx.x;
    const unsigned long long h = hist[i];
    c[i] = h;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned long long add = i >= o ? c[i - o] : 0ull;
        __syncthreads();
        c[i] += add;
        __syncthreads();
    }
    const unsigned long long r = st->rank, before = c[i] - h;
    const bool mine = before < r && (i == 255 || c[i] >= r);
    __syncthreads();   // every thread has read the rank before it changes
    if (mine) {
        st->rank = r - before;
        st->prefix |= (unsigned long long)i << shift;
        st->mask |= 0xffull << shift;
    }
    hist[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_qem_best(const uint64_t *__restrict__ key, int64_t n,
                                                     const int32_t *__restrict__ eu,
                                                     const int32_t *__restrict__ ev,
                                                     const SelState *__restrict__ st,
                                                     unsigned long long *__restrict__ best)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    const uint64_t k = key[e];
    if (k == kNone || (!st->all && k > st->prefix)) return;
    atomicMin(&best[eu[e]], k);
    atomicMin(&best[ev[e]], k);
}

__global__ __launch_bounds__(kBlock) void k_qem_choose(
    const uint64_t *__restrict__ key, int64_t n, const int32_t *__restrict__ eu,
    const int32_t *__restrict__ ev, const SelState *__restrict__ st,
    const unsigned long long *__restrict__ best, const int32_t *__restrict__ nb,
    const int32_t *__restrict__ ndeg, const double *__restrict__ X, double *__restrict__ P,
    const int32_t *__restrict__ fl, const int32_t *__restrict__ fdeg, int32_t *__restrict__ F,
    double *__restrict__ Q, int32_t *__restrict__ remap, uint8_t *__restrict__ dirty,
    int32_t *__restrict__ absorbed, uint32_t *__restrict__ counters)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t k = e < n ? key[e] : kNone;
    bool ok = k != kNone && (st->all || k <= st->prefix);
    const int32_t u = ok ? eu[e] : 0, v = ok ? ev[e] : 0;
    ok = ok && best[u] >= k && best[v] >= k;
    uint32_t killed = 0;
    for (int side = 0; side < 2 && ok; ++side) {
        const int64_t w = side == 0 ? u : v;
        const int32_t *b = nb + w * kQemNbrs;
        const int m = ndeg[w];
        for (int i = 0; i < m && ok; ++i) ok = best[b[i]] >= k;
    }
    if (ok) {
        // no end of an edge chosen in this step is an end or a neighbour of
        // an end of another: each updates its own u in place
        for (int i = 0; i < 10; ++i)
            Q[10 * (int64_t)u + i] = Q[10 * (int64_t)u + i] + Q[10 * (int64_t)v + i];
        for (int i = 0; i < 3; ++i) P[3 * (int64_t)u + i] = X[3 * e + i];
        remap[v] = u;
        absorbed[u] = v;
        // v's faces: the two on the edge degenerate and are dropped, the
        // others take u for v (no face has ends of two chosen edges)
        const int32_t *lv = fl + (int64_t)v * kQemFaces;
        const int fv = fdeg[v];
        for (int i = 0; i < fv; ++i) {
            const int64_t t = lv[i];
            const int32_t c0 = F[3 * t], c1 = F[3 * t + 1], c2 = F[3 * t + 2];
            if (c0 == u || c1 == u || c2 == u) {
                F[3 * t] = -1;
                ++killed;
            } else {
                F[3 * t + (c0 == v ? 0 : (c1 == v ? 1 : 2))] = u;
            }
        }
        // the closed one-rings change: their vertices are evaluated anew
        // in the next step (two rings may share a vertex: equal stores)
        dirty[u] = 1;
        dirty[v] = 1;
        for (int side = 0; side < 2; ++side) {
            const int64_t w = side == 0 ? u : v;
            const int32_t *b = nb + w * kQemNbrs;
            const int m = ndeg[w];
            for (int i = 0; i < m; ++i) dirty[b[i]] = 1;
        }
    }
    block_add(ok ? 1u : 0u, &counters[1]);
    block_add(killed, &counters[2]);
}

__global__ __launch_bounds__(kBlock) void k_qem_live(const int32_t *__restrict__ F, int64_t nt,
                                                     uint32_t *__restrict__ counters)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    block_add(t < nt && F[3 * t] >= 0 ? 1u : 0u, &counters[2]);
}

__global__ __launch_bounds__(kBlock) void k_qem_used(const int32_t *__restrict__ F, int64_t nt,
                                                     uint32_t *__restrict__ used,
                                                     uint32_t *__restrict__ keep)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const bool live = F[3 * t] >= 0;
    keep[t] = live ? 1u : 0u;
    if (live)
        for (int k = 0; k < 3; ++k) used[F[3 * t + k]] = 1u;
}

__global__ __launch_bounds__(kBlock) void k_qem_emit(const double *__restrict__ P, int64_t nv,
                                                     const uint32_t *__restrict__ used,
                                                     const uint32_t *__restrict__ newid,
                                                     const int32_t *__restrict__ F, int64_t nt,
                                                     const uint32_t *__restrict__ keep,
                                                     const uint32_t *__restrict__ tpos,
                                                     float *__restrict__ out_verts,
                                                     int32_t *__restrict__ out_tris)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nv && used[i])
        for (int k = 0; k < 3; ++k) out_verts[3 * (int64_t)newid[i] + k] = (float)P[3 * i + k];
    if (i < nt && keep[i])
        for (int k = 0; k < 3; ++k)
            out_tris[3 * (int64_t)tpos[i] + k] = (int32_t)newid[F[3 * i + k]];
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u8(uint8_t *p, int64_t n, uint8_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long *p, int64_t n,
                                                     unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_sel_init(SelState *st, unsigned long long rank, uint32_t *hist)
{
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->rank = rank;
        st->all = 0;
    }
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
}

// The need smallest candidate keys are eligible: all of them when need is
// at least the candidate count (counters[0]), else a select of the need-th.
__global__ void k_sel_init_need(SelState *st, unsigned long long need,
                                const uint32_t *__restrict__ counters, uint32_t *hist)
{
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->rank = need;
        st->all = need >= (unsigned long long)counters[0] ? 1ull : 0ull;
    }
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
}

}  // namespace

size_t qem_sel_bytes() { return sizeof(SelState) + 256 * sizeof(uint32_t); }
size_t radix_select_state_bytes() { return qem_sel_bytes(); }

hipError_t qem_init_launch(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                           double *P, int32_t *F, hipStream_t s)
{
    const int64_t n = nv > nt ? nv : nt;
    hipLaunchKernelGGL(k_qem_init, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, verts, nv, tris,
                       nt, P, F);
    return hipGetLastError();
}

hipError_t qem_incidence_launch(const QemBuffers &b, int64_t nv, int64_t nt, int round_start,
                                hipStream_t s)
{
    if (!round_start) {
        hipLaunchKernelGGL(k_qem_vertex_update, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s,
                           b.F, nv, b.dirty, b.remap, b.absorbed, b.fl, b.fdeg, b.nb, b.ndeg,
                           b.nlarge, b.counters + 3);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, b.fcnt, nv, 0u);
    hipLaunchKernelGGL(k_qem_fill_faces, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, b.F, nt,
                       b.fcnt, b.fl, b.counters + 3);
    hipLaunchKernelGGL(k_qem_vertex, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, b.P, b.F, nv,
                       b.fcnt, b.fl, b.fdeg, b.nb, b.ndeg, b.nlarge, b.Q, b.prot, round_start,
                       b.absorbed, b.counters + 3);
    return hipGetLastError();
}

hipError_t qem_edges_launch(const QemBuffers &b, int64_t nv, int64_t n_edges, int64_t n_old,
                            int round_start, hipStream_t s)
{
    if (!round_start && n_old > 0)
        hipLaunchKernelGGL(k_qem_carry, dim3(grid_for(n_old, kBlock)), dim3(kBlock), 0, s, n_old,
                           b.eu_old, b.ev_old, b.dirty, b.eoff, b.eoff_old, b.key_old, b.cand_old,
                           b.X_old, b.key, b.cand, b.X, b.eu, b.ev, b.counters);
    hipLaunchKernelGGL(k_qem_edges, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, nv, b.nb,
                       b.ndeg, b.eoff, b.dirty, round_start, b.cand, b.eu, b.ev);
    if (n_edges > 0)
        hipLaunchKernelGGL(k_qem_eval, dim3(grid_for(n_edges, kBlock)), dim3(kBlock), 0, s, b.P,
                           b.F, n_edges, b.fl, b.fdeg, b.nb, b.ndeg, b.Q, b.prot, b.eu, b.ev,
                           b.key, b.cand, b.X, b.counters);
    return hipGetLastError();
}

static hipError_t radix_passes(const uint64_t *keys, int64_t n, SelState *st, uint32_t *hist,
                               hipStream_t s)
{
    unsigned g = grid_for(n, kBlock);
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_qem_hist, dim3(g), dim3(kBlock), 0, s, keys, n, st, shift, hist);
        hipLaunchKernelGGL(k_qem_pick, dim3(1), dim3(256), 0, s, st, hist, shift);
    }
    return hipGetLastError();
}

hipError_t radix_select_u64_launch(const uint64_t *keys, int64_t n, uint64_t rank, char *state,
                                   hipStream_t s)
{
    SelState *st = reinterpret_cast<SelState *>(state);
    uint32_t *hist = reinterpret_cast<uint32_t *>(state + sizeof(SelState));
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, st, (unsigned long long)rank, hist);
    return radix_passes(keys, n, st, hist, s);
}

const uint64_t *radix_select_value(const char *state)
{
    return reinterpret_cast<const uint64_t *>(state);   // SelState::prefix
}

hipError_t qem_select_launch(const QemBuffers &b, int64_t n_edges, uint64_t need, hipStream_t s)
{
    SelState *st = reinterpret_cast<SelState *>(b.sel);
    uint32_t *hist = reinterpret_cast<uint32_t *>(b.sel + sizeof(SelState));
    hipLaunchKernelGGL(k_sel_init_need, dim3(1), dim3(256), 0, s, st, (unsigned long long)need,
                       b.counters, hist);
    return radix_passes(b.key, n_edges, st, hist, s);
}

hipError_t qem_live_launch(const QemBuffers &b, int64_t nt, hipStream_t s)
{
    hipLaunchKernelGGL(k_qem_live, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, b.F, nt,
                       b.counters);
    return hipGetLastError();
}

hipError_t qem_contract_launch(const QemBuffers &b, int64_t nv, int64_t n_edges, hipStream_t s)
{
    const SelState *st = reinterpret_cast<const SelState *>(b.sel);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, b.best, nv,
                       ~0ull);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s,
                       reinterpret_cast<uint32_t *>(b.remap), nv, 0xffffffffu);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, b.dirty, nv,
                       (uint8_t)0);
    if (n_edges > 0) {
        hipLaunchKernelGGL(k_qem_best, dim3(grid_for(n_edges, kBlock)), dim3(kBlock), 0, s, b.key,
                           n_edges, b.eu, b.ev, st, b.best);
        hipLaunchKernelGGL(k_qem_choose, dim3(grid_for(n_edges, kBlock)), dim3(kBlock), 0, s,
                           b.key, n_edges, b.eu, b.ev, st, b.best, b.nb, b.ndeg, b.X, b.P,
                           b.fl, b.fdeg, b.F, b.Q, b.remap, b.dirty, b.absorbed, b.counters);
    }
    return hipGetLastError();
}

hipError_t qem_used_launch(const int32_t *F, int64_t nt, uint32_t *used, uint32_t *keep,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_qem_used, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, F, nt, used,
                       keep);
    return hipGetLastError();
}

hipError_t qem_emit_launch(const double *P, int64_t nv, const uint32_t *used,
                           const uint32_t *newid, const int32_t *F, int64_t nt,
                           const uint32_t *keep, const uint32_t *tpos, float *out_verts,
                           int32_t *out_tris, hipStream_t s)
{
    const int64_t n = nv > nt ? nv : nt;
    hipLaunchKernelGGL(k_qem_emit, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, P, nv, used,
                       newid, F, nt, keep, tpos, out_verts, out_tris);
    return hipGetLastError();
}
