// trace.hip -- batched LiDAR ray casting kernels (gfx950).
//
// FGGS-LiDAR Sec. IV-C: one lane per beam; each ray r_j(t) = t_s + t R_s d_j
// walks the triangle LBVH near-child first and discards every node whose
// entry distance exceeds the best hit so far (and every triangle beyond it);
// the result is the nearest intersection t*_j over [t_min, t_max].
//
// Execution (gfx950, wave64).  The launch shape is a runtime choice
// (rc_tuning, picked per workload by the autotuner):
//  * One ray per lane over a flat grid (the default).  Rays are numbered
//    job by job and environment by environment; inside an environment,
//    consecutive lanes take a tile_az x tile_el block of beams (packet
//    tiling), so a wave's 64 rays have nearly equal directions and walk
//    nearly the same nodes.  A register cap (launch bounds) keeps 8 waves per
//    SIMD resident; the traversal stack lives in scratch.  By default each
//    workgroup is one wave: a wave whose rays are done frees its slot at once
//    instead of waiting for the slowest wave of a larger workgroup (10%
//    faster than four-wave workgroups on the headline batch); four-wave
//    workgroups spread a small launch over more CUs.
//  * Persistent waves.  The launch's rays are split into one contiguous
//    range per XCD (workgroups are dispatched round-robin over the 8 XCDs,
//    so block b runs on XCD b % 8 and takes rays from range b % 8 first,
//    keeping neighbouring environments in one L2); when its range is empty
//    a wave steals from the others.  Wavefront-ballot refill: a wave keeps
//    traversing while fewer than `refill_min` of its 64 lanes are idle; the
//    idle lanes then take consecutive rays from the wave's pool in lane order
//    (prefix count of the idle ballot).
//  * Stack: optionally the first `SS` entries of every lane's traversal
//    stack live in LDS (slot-major, so the 64 lanes of a wave touch 64
//    consecutive words); deeper entries are in scratch.  A Karras tree over
//    3b-bit codes plus index tie-breaks is at most 62 levels deep, so 64
//    entries always suffice (96 for 4-wide nodes: at most three pushes per
//    level).
//  * Node formats: the binary tree with FP32 child boxes, or 4-wide nodes
//    with 8-bit child boxes in the node's frame (see node_step_q8).
//
// Numerics (compiled with -ffp-contract=off so every variant rounds alike):
//  * Ray: direction R_s d_j is formed and normalised in FP64, then rounded to
//    FP32 for the traversal.
//  * Triangle test: the watertight test of Woop, Benthin and Wald (2013) in
//    FP32 -- translate, permute so the dominant direction axis is z, shear
//    -- then the 2-D edge functions U, V, W.  A sign is trusted only when
//    |U| exceeds a forward error bound of its two products; a miss needs one
//    trusted positive and one trusted negative sign.  Otherwise the edge
//    functions are recomputed in FP64 from the same FP32 sheared
//    coordinates, where the products are exact and so every sign is exact.
//    Shared edges produce exactly negated products in both triangles, so the
//    decision is consistent across them and no ray slips between triangles.
//  * Box test: slabs (lo - o) * (1/d) with the far distance scaled by
//    1 + 2*gamma_3 (Ize 2013), widened further by a relative margin so a box
//    is only culled when it cannot hold a triangle whose FP32 distance would
//    beat the current best.
//  * Candidates compare as (t, triangle id) pairs, so exact ties go to the
//    lowest id whatever the visit order: every kernel variant, the BVH and
//    the brute-force kernel agree bit for bit.
//  * The winner's range is recomputed in FP64 from the FP64 ray and the
//    triangle's plane, then rounded to FP32.
#include "rc_internal.h"

#include <float.h>
#include <math.h>

namespace {

constexpr int kBlock = 256;      // persistent kernel: 4 waves per workgroup
constexpr int64_t kMaxRaysPerDispatch = (int64_t)1 << 30;
constexpr int kStack = 64;           // >= depth of any Karras tree (62 key bits)
constexpr float kErrU = 2.384185791015625e-07f;  // 2^-22: sign certificate factor
constexpr float kBoxGrow = 7.152557373046875e-07f;  // 12u > 2 gamma_3: far-distance growth
constexpr float kCullRel = 6.103515625e-05f;     // 2^-14 relative culling margin

struct RayW {
    float o[3];        // origin, permuted (kx, ky, kz)
    float Sx, Sy, Sz;  // shear constants
    int kx, ky, kz;
    float org[3];      // origin, world axes
    float inv[3];      // 1 / direction, world axes (clamped away from 0)
};

// Node and triangle records are read through global-address-space pointers:
// the record arrays are reached through the job table, so the compiler would
// otherwise emit flat loads, which must be waited for as a group (they count
// on both the vector-memory and the LDS counters) and cannot use the global
// addressing forms.
typedef float gvec4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const gvec4 gvec4_g;

__device__ __forceinline__ float4 ldg4(const void *p, int64_t i)
{
    const gvec4 v = ((const gvec4_g *)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ NodeRec load_node_vec(const NodeRec *nodes, int i)
{
    NodeRec n;
    n.q0 = ldg4(nodes, 4 * (int64_t)i);
    n.q1 = ldg4(nodes, 4 * (int64_t)i + 1);
    n.q2 = ldg4(nodes, 4 * (int64_t)i + 2);
    const float4 w = ldg4(nodes, 4 * (int64_t)i + 3);
    n.q3 = make_int4(__float_as_int(w.x), __float_as_int(w.y), __float_as_int(w.z),
                     __float_as_int(w.w));
    return n;
}

// Node records never change while a traversal runs, so a record that every
// active lane of the wave needs can be read once through the scalar data
// cache (the constant address space with a wave-uniform address) instead of
// by 64 lanes through the vector memory path, whose address and data units
// are the traversal's busiest resource.
typedef __attribute__((address_space(4))) const gvec4 gvec4_c;

__device__ __forceinline__ NodeRec load_node(const NodeRec *nodes, int i)
{
    const int i0 = __builtin_amdgcn_readfirstlane(i);
    const uint64_t p = (uint64_t)(uintptr_t)nodes;
    const uint32_t plo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t phi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    const uint64_t p0 = ((uint64_t)phi << 32) | plo;
    if (__ballot(i != i0 || p != p0) == 0ull) {
        const gvec4_c *q = (const gvec4_c *)(uintptr_t)p0 + 4 * (int64_t)i0;
        const gvec4 a = q[0], b = q[1], c = q[2], d = q[3];
        NodeRec n;
        n.q0 = make_float4(a.x, a.y, a.z, a.w);
        n.q1 = make_float4(b.x, b.y, b.z, b.w);
        n.q2 = make_float4(c.x, c.y, c.z, c.w);
        n.q3 = make_int4(__float_as_int(d.x), __float_as_int(d.y), __float_as_int(d.z),
                         __float_as_int(d.w));
        return n;
    }
    return load_node_vec(nodes, i);
}

__device__ __forceinline__ TriRec load_tri(const TriRec *tris, int i)
{
    TriRec t;
    t.a = ldg4(tris, 3 * (int64_t)i);
    t.b = ldg4(tris, 3 * (int64_t)i + 1);
    t.c = ldg4(tris, 3 * (int64_t)i + 2);
    return t;
}

__device__ __forceinline__ float sel3(float a, float b, float c, int k)
{
    return k == 0 ? a : (k == 1 ? b : c);
}

// FP64 unit direction R * b / |R * b|
__device__ __forceinline__ void ray_dir64(const float *p, const float *b, double d[3])
{
    for (int i = 0; i < 3; ++i)
        d[i] = (double)p[4 * i + 0] * (double)b[0] + (double)p[4 * i + 1] * (double)b[1] +
               (double)p[4 * i + 2] * (double)b[2];
    const double rn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) d[i] *= rn;
}

__device__ __forceinline__ void make_ray(const float *p, const float *b, RayW &r)
{
    double d[3];
    ray_dir64(p, b, d);
    float d32[3] = {(float)d[0], (float)d[1], (float)d[2]};
    r.org[0] = p[3];
    r.org[1] = p[7];
    r.org[2] = p[11];
    int kz = 0;
    if (fabsf(d32[1]) > fabsf(d32[kz])) kz = 1;
    if (fabsf(d32[2]) > fabsf(d32[kz])) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (d32[kz] < 0.0f) { int s = kx; kx = ky; ky = s; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    const float dkx = sel3(d32[0], d32[1], d32[2], kx);
    const float dky = sel3(d32[0], d32[1], d32[2], ky);
    const float dkz = sel3(d32[0], d32[1], d32[2], kz);
    r.Sx = dkx / dkz;
    r.Sy = dky / dkz;
    r.Sz = 1.0f / dkz;
    r.o[0] = sel3(r.org[0], r.org[1], r.org[2], kx);
    r.o[1] = sel3(r.org[0], r.org[1], r.org[2], ky);
    r.o[2] = sel3(r.org[0], r.org[1], r.org[2], kz);
    for (int i = 0; i < 3; ++i) {
        float di = d32[i];
        float safe = fabsf(di) > 1e-20f ? di : copysignf(1e-20f, di);
        r.inv[i] = 1.0f / safe;
    }
}

// FP64 re-evaluation from the FP32 sheared coordinates (products exact).
// Returns the FP32 ray parameter of a hit, NaN on a miss (by value: an
// out-parameter lives in private memory, and the caller's loop would wait
// for its reload before the next triangle's loads).
__device__ __noinline__ float woop64(float Ax, float Ay, float Bx, float By, float Cx, float Cy,
                                    float Az, float Bz, float Cz, float Sz)
{
    const float miss = __int_as_float(0x7fc00000);
    double U = (double)Cx * (double)By - (double)Cy * (double)Bx;
    double V = (double)Ax * (double)Cy - (double)Ay * (double)Cx;
    double W = (double)Bx * (double)Ay - (double)By * (double)Ax;
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return miss;
    double det = U + V + W;
    if (det == 0.0) return miss;
    double T = U * ((double)Sz * (double)Az) + V * ((double)Sz * (double)Bz) +
               W * ((double)Sz * (double)Cz);
    return (float)(T / det);
}

// Watertight test of one triangle record; returns true and the FP32 ray
// parameter on a hit.
__device__ __forceinline__ bool woop32(const RayW &r, const float4 &q0, const float4 &q1,
                                       const float4 &q2, float *t_out)
{
    const float A_x = sel3(q0.x, q0.y, q0.z, r.kx) - r.o[0];
    const float A_y = sel3(q0.x, q0.y, q0.z, r.ky) - r.o[1];
    const float A_z = sel3(q0.x, q0.y, q0.z, r.kz) - r.o[2];
    const float B_x = sel3(q0.w, q1.x, q1.y, r.kx) - r.o[0];
    const float B_y = sel3(q0.w, q1.x, q1.y, r.ky) - r.o[1];
    const float B_z = sel3(q0.w, q1.x, q1.y, r.kz) - r.o[2];
    const float C_x = sel3(q1.z, q1.w, q2.x, r.kx) - r.o[0];
    const float C_y = sel3(q1.z, q1.w, q2.x, r.ky) - r.o[1];
    const float C_z = sel3(q1.z, q1.w, q2.x, r.kz) - r.o[2];
    // shear with one rounding per coordinate; a vertex shared by several
    // triangles gets the same sheared coordinates in each
    const float Ax = fmaf(-r.Sx, A_z, A_x), Ay = fmaf(-r.Sy, A_z, A_y);
    const float Bx = fmaf(-r.Sx, B_z, B_x), By = fmaf(-r.Sy, B_z, B_y);
    const float Cx = fmaf(-r.Sx, C_z, C_x), Cy = fmaf(-r.Sy, C_z, C_y);
    const float u1 = Cx * By, u2 = Cy * Bx;
    const float v1 = Ax * Cy, v2 = Ay * Cx;
    const float w1 = Bx * Ay, w2 = By * Ax;
    const float U = u1 - u2, V = v1 - v2, W = w1 - w2;
    const float eU = kErrU * (fabsf(u1) + fabsf(u2));
    const float eV = kErrU * (fabsf(v1) + fabsf(v2));
    const float eW = kErrU * (fabsf(w1) + fabsf(w2));
    const bool pU = U > eU, nU = U < -eU;
    const bool pV = V > eV, nV = V < -eV;
    const bool pW = W > eW, nW = W < -eW;
    if ((pU || pV || pW) && (nU || nV || nW)) return false;  // certain miss
    if (!((pU || nU) && (pV || nV) && (pW || nW))) {
        const float t64 = woop64(Ax, Ay, Bx, By, Cx, Cy, A_z, B_z, C_z, r.Sz);
        *t_out = t64;
        return t64 == t64;
    }
    // all three signs certain and equal
    const float det = U + V + W;
    const float T = r.Sz * fmaf(U, A_z, fmaf(V, B_z, W * C_z));
    *t_out = T / det;
    return true;
}

// (t, id) before (bt, bid) in lexicographic order; evaluated without
// branches
__device__ __forceinline__ bool better(float t, int id, float bt, int bid)
{
    return (t < bt) | ((t == bt) & (id < bid));
}

// FP64 range of the winning triangle along the FP64 ray (plane equation).
__device__ float refine_range(const float *p, const float *b, const TriRec &tr, float t32)
{
    double d[3];
    ray_dir64(p, b, d);
    const double o[3] = {p[3], p[7], p[11]};
    const double v0[3] = {tr.a.x, tr.a.y, tr.a.z};
    const double v1[3] = {tr.a.w, tr.b.x, tr.b.y};
    const double v2[3] = {tr.b.z, tr.b.w, tr.c.x};
    const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    const double num = nn[0] * (v0[0] - o[0]) + nn[1] * (v0[1] - o[1]) + nn[2] * (v0[2] - o[2]);
    const double den = nn[0] * d[0] + nn[1] * d[1] + nn[2] * d[2];
    const double t = num / den;
    if (!isfinite(t)) return t32;
    return (float)t;
}

__device__ __forceinline__ int find_job(const DevJob *jobs, int n_jobs, int64_t g)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].ray_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// slab test of one child box; returns the entry distance or +inf on a miss
__device__ __forceinline__ float slab(const RayW &r, float lox, float hix, float loy, float hiy,
                                      float loz, float hiz, float t_lo, float t_hi)
{
    const float tx0 = (lox - r.org[0]) * r.inv[0], tx1 = (hix - r.org[0]) * r.inv[0];
    const float ty0 = (loy - r.org[1]) * r.inv[1], ty1 = (hiy - r.org[1]) * r.inv[1];
    const float tz0 = (loz - r.org[2]) * r.inv[2], tz1 = (hiz - r.org[2]) * r.inv[2];
    const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), t_lo));
    float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    tf = tf + fabsf(tf) * kBoxGrow;
    return (tn <= tf && tn <= t_hi) ? tn : INFINITY;
}

// ---------------------------------------------------------------------------
// Per-lane traversal state and stack.

template <int SS, int STK, int BLK>
struct LaneStack {
    static_assert(SS >= 0 && SS < STK, "the LDS ring is smaller than the stack");
    // Node and distance packed in one 8-byte word, so a push or pop is one
    // memory instruction.  With SS > 0 the top min(sp, SS) entries sit in an
    // LDS ring of SS slots (entry k in slot k mod SS, this lane's word at
    // lw[slot * BLK]) and only the entries below it in scratch: a push that
    // finds the ring full moves the ring's oldest entry down, a pop refills
    // the slot it frees from below.  Typical depths never leave LDS, so the
    // scratch lines (which the other resident waves evict from L2 before
    // they come back) are rarely touched.
    uint64_t *lw;
    uint64_t sw[STK - SS];
    static __device__ __forceinline__ uint64_t pack(int n, float t)
    {
        return (uint64_t)(uint32_t)n | ((uint64_t)__float_as_uint(t) << 32);
    }
    __device__ __forceinline__ void put(int k, int n, float t)
    {
        const uint64_t w = pack(n, t);
        if constexpr (SS == 0) {
            sw[k] = w;
        } else {
            uint64_t *slot = lw + (k % SS) * BLK;
            if (k >= SS) sw[k - SS] = *slot;
            *slot = w;
        }
    }
    __device__ __forceinline__ void get(int k, int &n, float &t)
    {
        uint64_t w;
        if constexpr (SS == 0) {
            w = sw[k];
        } else {
            uint64_t *slot = lw + (k % SS) * BLK;
            w = *slot;
            if (k >= SS) *slot = sw[k - SS];
        }
        n = (int)(uint32_t)w;
        t = __uint_as_float((uint32_t)(w >> 32));
    }
};

struct LaneRay {
    RayW r;
    const NodeRec *nodes;
    const TriRec *tris;
    const float *pose;
    const float *beam;
    int64_t out;
    float t_min, t_max, t_lo, t_hi, best_t;
    int best_id, best_leaf, node, sp, n_tris_scene, fetched;
    int n_nodes, n_tris;
    bool corrupt;
};

__device__ __forceinline__ uint32_t udiv(uint32_t n, UDiv u)
{
    const uint32_t t = __umulhi(u.m, n);
    return (t + ((n - t) >> (u.sh & 0xffu))) >> (u.sh >> 8);
}

// which beam the q-th ray of an environment is (packet tiling)
__device__ __forceinline__ uint32_t tile_beam(const DevJob &jb, uint32_t q)
{
    const uint32_t tw = (uint32_t)jb.tile_az, th = (uint32_t)jb.tile_el;
    const uint32_t naz = (uint32_t)jb.n_az;
    const uint32_t per = tw * th;
    const uint32_t tile = udiv(q, jb.div_tile), rr = q - tile * per;
    const uint32_t tiles_az = (uint32_t)jb.tiles_az;
    const uint32_t te = udiv(tile, jb.div_tiles_az), ta = tile - te * tiles_az;
    const uint32_t row = udiv(rr, jb.div_tile_az), col = rr - row * tw;
    return (te * th + row) * naz + ta * tw + col;
}

__device__ __forceinline__ void test_leaf(LaneRay &L, int leaf)
{
    const TriRec tr = load_tri(L.tris, leaf);
    float t;
    ++L.n_tris;
    if (woop32(L.r, tr.a, tr.b, tr.c, &t)) {
        // the update as selects rather than nested branches: each level of
        // divergent branching costs the wave scalar exec-mask instructions
        const int id = __float_as_int(tr.c.y);
        const bool upd = (t >= L.t_min) & (t <= L.t_max) & better(t, id, L.best_t, L.best_id);
        L.best_t = upd ? t : L.best_t;
        L.best_id = upd ? id : L.best_id;
        L.best_leaf = upd ? leaf : L.best_leaf;
        L.t_hi = upd ? t * (1.0f + kCullRel) : L.t_hi;
    }
}

// Set up the ray with flattened launch index g; returns true if it still
// needs traversal (false: already finished, e.g. empty scene).
__device__ __forceinline__ bool setup_ray(const DevJob *__restrict__ jobs, int n_jobs, int64_t g,
                                          LaneRay &L)
{
    const DevJob &jb = jobs[find_job(jobs, n_jobs, g)];
    const uint32_t local = (uint32_t)(g - jb.ray_begin);   // a job holds < 2^31 rays
    const uint32_t nb = (uint32_t)jb.n_beams;
    const uint32_t e = udiv(local, jb.div_beams);
    const uint32_t q = local - e * nb;
    const uint32_t beam = tile_beam(jb, q);
    L.pose = jb.poses + 12 * (int64_t)e;
    L.beam = jb.dirs + 3 * (int64_t)beam;
    L.out = jb.out_offset + (int64_t)e * nb + beam;
    make_ray(L.pose, L.beam, L.r);
    L.nodes = jb.nodes;
    L.tris = jb.tris;
    L.n_tris_scene = jb.n_tris;
    L.t_min = jb.t_min;
    L.t_max = jb.t_max;
    L.t_lo = jb.t_min * (1.0f - kCullRel);
    L.t_hi = jb.t_max * (1.0f + kCullRel);
    L.best_t = INFINITY;
    L.best_id = 0x7fffffff;
    L.best_leaf = -1;
    L.node = 0;
    L.sp = 0;
    L.fetched = 0;
    L.n_nodes = 0;
    L.n_tris = 0;
    L.corrupt = false;
    if (jb.n_tris == 0) return false;
    if (jb.root_leaf) {
        test_leaf(L, 0);
        return false;
    }
    return true;
}

// One internal-node visit.  Returns true when the ray has finished.
template <int SS, int STK, int BLK>
__device__ __forceinline__ bool node_step(LaneRay &L, LaneStack<SS, STK, BLK> &S)
{
    const NodeRec nd = load_node(L.nodes, L.node);
    ++L.n_nodes;
    const float tl = slab(L.r, nd.q0.x, nd.q0.y, nd.q1.x, nd.q1.y, nd.q2.x, nd.q2.y, L.t_lo, L.t_hi);
    const float tr = slab(L.r, nd.q0.z, nd.q0.w, nd.q1.z, nd.q1.w, nd.q2.z, nd.q2.w, L.t_lo, L.t_hi);
    const int cl = nd.q3.x, cr = nd.q3.y;
    bool hl = tl < INFINITY, hr = tr < INFINITY;
    // leaves are tested on the spot, nearer one first
    {
        int l0 = -1, l1 = -1;
        float t1 = 0.0f;
        if (hl && cl < 0) { l0 = ~cl; hl = false; }
        if (hr && cr < 0) {
            if (l0 < 0) l0 = ~cr;
            else if (tr < tl) { l1 = l0; t1 = tl; l0 = ~cr; }
            else { l1 = ~cr; t1 = tr; }
            hr = false;
        }
        if (l0 >= 0) test_leaf(L, l0);
        if (l1 >= 0 && t1 <= L.t_hi) test_leaf(L, l1);
    }
    hl = hl && tl <= L.t_hi;
    hr = hr && tr <= L.t_hi;
    if (hl && hr) {
        const bool lnear = tl <= tr;
        if (L.sp == STK) { L.corrupt = true; return true; }  // deeper than any Karras tree
        S.put(L.sp, lnear ? cr : cl, lnear ? tr : tl);
        ++L.sp;
        L.node = lnear ? cl : cr;
        return false;
    }
    if (hl) { L.node = cl; return false; }
    if (hr) { L.node = cr; return false; }
    // pop the nearest pending subtree still in range
    while (L.sp > 0) {
        --L.sp;
        int n;
        float t;
        S.get(L.sp, n, t);
        if (t <= L.t_hi) { L.node = n; return false; }
    }
    return true;
}

// Quantised 4-wide node visit.  Each child plane is evaluated in the node's
// frame as t = q * (scale * inv) + (origin - o) * inv with one FMA; the
// entry (exit) distances are lowered (raised) by E_a = 8u (|a| + 255 |b|),
// which bounds the rounding of a, b and the FMA against the exact plane
// distance, so a child box is never culled when its exact box would not be.
constexpr float kQErr = 4.76837158203125e-07f;   // 8u, u = 2^-24
constexpr int kStackQ8 = 96;                     // 3 pushes per level x 31 levels + 1

__device__ __forceinline__ float qbyte(uint32_t w, int k)
{
    return (float)((w >> (8 * k)) & 0xffu);
}

template <int SS, int STK, int BLK>
__device__ __forceinline__ bool node_step_q8(LaneRay &L, LaneStack<SS, STK, BLK> &S)
{
    const NodeRec nd = load_node(L.nodes, L.node);
    ++L.n_nodes;
    const float org[3] = {nd.q0.x, nd.q0.y, nd.q0.z};
    const float scl[3] = {nd.q0.w, nd.q1.x, nd.q1.y};
    const uint32_t qlo[3] = {__float_as_uint(nd.q1.z), __float_as_uint(nd.q2.x),
                             __float_as_uint(nd.q2.z)};
    const uint32_t qhi[3] = {__float_as_uint(nd.q1.w), __float_as_uint(nd.q2.y),
                             __float_as_uint(nd.q2.w)};
    float an[3], af[3], bb[3];
    uint32_t qn[3], qf[3];
    for (int a = 0; a < 3; ++a) {
        const float inv = L.r.inv[a];
        const float aa = (org[a] - L.r.org[a]) * inv;
        const float b = scl[a] * inv;
        // one FMA and one product: E stays above 8u (|a| + 255 |b|) up to
        // two roundings, well inside the bound's factor-two slack
        const float E = kQErr * fmaf(255.0f, fabsf(b), fabsf(aa));
        an[a] = aa - E;
        af[a] = aa + E;
        bb[a] = b;
        const bool neg = inv < 0.0f;
        qn[a] = neg ? qhi[a] : qlo[a];
        qf[a] = neg ? qlo[a] : qhi[a];
    }
    const int32_t cref[4] = {nd.q3.x, nd.q3.y, nd.q3.z, nd.q3.w};
    float t[4];
    int32_t ref[4];
    for (int k = 0; k < 4; ++k) {
        // [t_lo, t_hi] folded into the entry and exit distances
        const float en = fmaxf(fmaxf(fmaf(qbyte(qn[0], k), bb[0], an[0]),
                                     fmaf(qbyte(qn[1], k), bb[1], an[1])),
                               fmaxf(fmaf(qbyte(qn[2], k), bb[2], an[2]), L.t_lo));
        const float ex = fminf(fminf(fmaf(qbyte(qf[0], k), bb[0], af[0]),
                                     fmaf(qbyte(qf[1], k), bb[1], af[1])),
                               fminf(fmaf(qbyte(qf[2], k), bb[2], af[2]), L.t_hi));
        const bool hit = cref[k] != kEmptyChild && en <= ex;
        t[k] = hit ? en : INFINITY;   // a hit's entry distance is finite
        ref[k] = cref[k];
    }
    // ascending by entry distance (5 compare-exchanges)
#define RC_CSWAP(i, j)                                                  \
    if (t[j] < t[i]) {                                                  \
        float tt = t[i]; t[i] = t[j]; t[j] = tt;                        \
        int32_t rr = ref[i]; ref[i] = ref[j]; ref[j] = rr;              \
    }
    RC_CSWAP(0, 1) RC_CSWAP(2, 3) RC_CSWAP(0, 2) RC_CSWAP(1, 3) RC_CSWAP(1, 2)
#undef RC_CSWAP
    // leaves on the spot, nearest first.  One loop iteration per leaf of
    // this lane (not one code copy per child slot), so lanes whose leaves sit
    // in different slots test them together.  Missed children carry +inf,
    // which also t_hi = +inf (an unbounded range) must not admit.
    uint32_t lm = 0;
    for (int k = 0; k < 4; ++k)
        lm |= (ref[k] < 0 && t[k] < INFINITY) ? 1u << k : 0u;
#pragma unroll 1
    while (lm != 0u) {
        const int k = __builtin_ctz(lm);
        lm &= lm - 1u;
        const float tk = k == 0 ? t[0] : (k == 1 ? t[1] : (k == 2 ? t[2] : t[3]));
        const int32_t rk = k == 0 ? ref[0] : (k == 1 ? ref[1] : (k == 2 ? ref[2] : ref[3]));
        if (tk <= L.t_hi) test_leaf(L, ~rk);
    }
    // internal children: continue with the nearest, push the others
    // farthest first
    int next = -1;
    float next_t = 0.0f;
    const float lim = fminf(L.t_hi, FLT_MAX);
    // at most 3 pushes below, so one bound check covers them (a push site
    // of a valid tree has sp <= 3 (31 - 1) = 90).  It and the exits below
    // are selects rather than early returns: every divergent exit costs
    // each visit scalar exec-mask work
    const bool full = L.sp > STK - 3;
    L.corrupt = L.corrupt | full;
    for (int k = 3; k >= 0; --k) {
        if (ref[k] >= 0 && t[k] <= lim) {
            if (next >= 0 && !full) {
                S.put(L.sp, next, next_t);
                ++L.sp;
            }
            next = ref[k];
            next_t = t[k];
        }
    }
    // one exit: continue with the nearest child, else pop the nearest
    // pending subtree still in range
    bool more = next >= 0;
    L.node = more ? next : L.node;
    bool pop = !more;
    while (pop & (L.sp > 0)) {
        --L.sp;
        int n;
        float tt;
        S.get(L.sp, n, tt);
        const bool ok = tt <= L.t_hi;
        L.node = ok ? n : L.node;
        more = ok;
        pop = !ok;
    }
    return !more | full;
}

template <int FMT, int SS, int STK, int BLK>
__device__ __forceinline__ bool visit(LaneRay &L, LaneStack<SS, STK, BLK> &S)
{
    if (FMT == FMT_Q8) return node_step_q8<SS, STK, BLK>(L, S);
    return node_step<SS, STK, BLK>(L, S);
}

// One node visit, then the node-fetch cap: a correct traversal fetches each
// of the n_tris - 1 records at most once, so the cap only stops a corrupted
// tree.  Applied with selects after the visit rather than as a branch out
// of it.  Returns true when the ray has finished.
template <int FMT, int SS, int STK, int BLK>
__device__ __forceinline__ bool visit_capped(LaneRay &L, LaneStack<SS, STK, BLK> &S)
{
    const bool done = visit<FMT>(L, S);
    const bool over = ++L.fetched > L.n_tris_scene + 64;
    L.corrupt = L.corrupt | (!done & over);
    return done | over;
}

template <int MODE>
__device__ __forceinline__ void finish_ray(const LaneRay &L, float *__restrict__ out_range,
                                           int32_t *__restrict__ out_hit,
                                           int32_t *__restrict__ out_nodes,
                                           int32_t *__restrict__ out_tris)
{
    if (L.corrupt) {
        out_range[L.out] = NAN;  // never a valid result: flags a broken hierarchy
        out_hit[L.out] = -2;
    } else if (L.best_leaf >= 0) {
        const TriRec tr = load_tri(L.tris, L.best_leaf);
        out_range[L.out] = refine_range(L.pose, L.beam, tr, L.best_t);
        out_hit[L.out] = L.best_id;
    } else {
        out_range[L.out] = INFINITY;
        out_hit[L.out] = -1;
    }
    if (MODE == TRACE_STATS) {
        out_nodes[L.out] = L.n_nodes;
        out_tris[L.out] = L.n_tris;
    }
}

// ---------------------------------------------------------------------------
// One ray per thread (also the brute-force cross-check).
template <int MODE, int FMT, int SS, int WAVES, int BLK>
__global__ __launch_bounds__(BLK, WAVES) void k_trace(const DevJob *__restrict__ jobs, int n_jobs,
                                                  int64_t g0, int64_t total,
                                                  float *__restrict__ out_range,
                                                  int32_t *__restrict__ out_hit,
                                                  int32_t *__restrict__ out_nodes,
                                                  int32_t *__restrict__ out_tris)
{
    __shared__ uint64_t s_stk[SS > 0 ? SS * BLK : 1];
    const int64_t g = g0 + (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (g >= total) return;
    LaneRay L;
    LaneStack<SS, FMT == FMT_Q8 ? kStackQ8 : kStack, BLK> S;
    S.lw = s_stk + threadIdx.x;
    bool go = setup_ray(jobs, n_jobs, g, L);
    if (MODE == TRACE_BRUTE) {
        for (int k = 0; go && k < L.n_tris_scene; ++k) test_leaf(L, k);
    } else {
        while (go) go = !visit_capped<FMT>(L, S);
    }
    finish_ray<MODE>(L, out_range, out_hit, out_nodes, out_tris);
}

// ---------------------------------------------------------------------------
// Deferred triangle tests (Q8 nodes, one ray per lane).
//
// In the kernels above a lane tests the leaves of a node as soon as it finds
// them, so the whole wave runs the ~110-instruction triangle test whenever
// any one of its lanes has reached a leaf, with the other lanes idle; at the
// headline workload that happens in nearly every loop iteration.  Here the
// node visits only collect (lane, leaf) pairs in a per-wave queue in LDS,
// and the wave alternates between two kinds of step:
//  * node step: every lane that still has nodes to visit visits one; the
//    leaves it finds in range are appended to the queue (a wave prefix sum
//    of the per-lane leaf counts gives each lane its slots);
//  * triangle step, taken once `batch` pairs are queued (or when no lane has
//    nodes left): lane i tests the i-th queued pair against the owner lane's
//    ray (kept in LDS) and folds the hit into the owner's best (t, id) with
//    a 64-bit LDS atomic minimum -- for t >= 0 the bit pattern of t followed
//    by the id orders exactly like the (t, id) pairs -- so one step runs up
//    to 64 tests with every lane busy.
// A lane keeps traversing while its pairs wait: its culling distance is the
// best hit known at the last triangle step, which is never below the true
// best, so culling stays conservative and the result is the same (t, id)
// minimum as on-the-spot testing -- bit-identical, only the set of nodes
// visited changes.  A triangle step runs at most 64 tests and is taken
// before the queue holds 64, so it never holds more than 63 + 4 x 64 pairs.
constexpr int kRing = 320;            // >= 63 + 4 * 64 queued pairs
constexpr int kLeafBits = 26;         // leaf index bits of a queued pair
constexpr uint64_t kNoHit = ~0ull;

struct DeferWave {
    float o[3][64];         // triangle-test frame of each lane's ray: permuted origin
    float s[3][64];         //   shear constants Sx, Sy, Sz
    int k[64];              //   kx | ky << 2 | kz << 4
    float tmin[64], tmax[64];
    const TriRec *tris[64];
    unsigned long long best[64];   // (t bits << 32) | triangle id, kNoHit when none
    int best_leaf[64];
    uint32_t ring[kRing];          // queued pairs: lane << 26 | leaf
};

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Node visit without triangle tests: sets *lm to the in-range leaf children
// (bit k: slot k of ref[], nearest first) and returns true when the lane has
// no node left.
template <int STK, int BLK>
__device__ __forceinline__ bool node_step_q8_collect(LaneRay &L, LaneStack<0, STK, BLK> &S,
                                                     int32_t ref[4], uint32_t *lm)
{
    *lm = 0u;
    if (++L.fetched > L.n_tris_scene + 64) { L.corrupt = true; return true; }
    const NodeRec nd = load_node(L.nodes, L.node);
    ++L.n_nodes;
    const float org[3] = {nd.q0.x, nd.q0.y, nd.q0.z};
    const float scl[3] = {nd.q0.w, nd.q1.x, nd.q1.y};
    const uint32_t qlo[3] = {__float_as_uint(nd.q1.z), __float_as_uint(nd.q2.x),
                             __float_as_uint(nd.q2.z)};
    const uint32_t qhi[3] = {__float_as_uint(nd.q1.w), __float_as_uint(nd.q2.y),
                             __float_as_uint(nd.q2.w)};
    float an[3], af[3], bb[3];
    uint32_t qn[3], qf[3];
    for (int a = 0; a < 3; ++a) {
        const float inv = L.r.inv[a];
        const float aa = (org[a] - L.r.org[a]) * inv;
        const float b = scl[a] * inv;
        const float E = kQErr * fmaf(255.0f, fabsf(b), fabsf(aa));
        an[a] = aa - E;
        af[a] = aa + E;
        bb[a] = b;
        const bool neg = inv < 0.0f;
        qn[a] = neg ? qhi[a] : qlo[a];
        qf[a] = neg ? qlo[a] : qhi[a];
    }
    const int32_t cref[4] = {nd.q3.x, nd.q3.y, nd.q3.z, nd.q3.w};
    float t[4];
    for (int k = 0; k < 4; ++k) {
        const float en = fmaxf(fmaxf(fmaf(qbyte(qn[0], k), bb[0], an[0]),
                                     fmaf(qbyte(qn[1], k), bb[1], an[1])),
                               fmaxf(fmaf(qbyte(qn[2], k), bb[2], an[2]), L.t_lo));
        const float ex = fminf(fminf(fmaf(qbyte(qf[0], k), bb[0], af[0]),
                                     fmaf(qbyte(qf[1], k), bb[1], af[1])),
                               fminf(fmaf(qbyte(qf[2], k), bb[2], af[2]), L.t_hi));
        const bool hit = cref[k] != kEmptyChild && en <= ex;
        t[k] = hit ? en : INFINITY;
        ref[k] = cref[k];
    }
#define RC_CSWAP(i, j)                                                  \
    if (t[j] < t[i]) {                                                  \
        float tt = t[i]; t[i] = t[j]; t[j] = tt;                        \
        int32_t rr = ref[i]; ref[i] = ref[j]; ref[j] = rr;              \
    }
    RC_CSWAP(0, 1) RC_CSWAP(2, 3) RC_CSWAP(0, 2) RC_CSWAP(1, 3) RC_CSWAP(1, 2)
#undef RC_CSWAP
    // missed children carry +inf, which an unbounded range must not admit
    const float lim = fminf(L.t_hi, FLT_MAX);
    uint32_t m = 0;
    for (int k = 0; k < 4; ++k) m |= (ref[k] < 0 && t[k] <= lim) ? 1u << k : 0u;
    *lm = m;
    int next = -1;
    float next_t = 0.0f;
    for (int k = 3; k >= 0; --k) {
        if (ref[k] >= 0 && t[k] <= lim) {
            if (next >= 0) {
                if (L.sp == STK) { L.corrupt = true; return true; }
                S.put(L.sp, next, next_t);
                ++L.sp;
            }
            next = ref[k];
            next_t = t[k];
        }
    }
    if (next >= 0) { L.node = next; return false; }
    while (L.sp > 0) {
        --L.sp;
        int n;
        float tt;
        S.get(L.sp, n, tt);
        if (tt <= L.t_hi) { L.node = n; return false; }
    }
    return true;
}

// Output location of flattened ray g (as setup_ray computes it).
__device__ __forceinline__ void ray_location(const DevJob *__restrict__ jobs, int n_jobs, int64_t g,
                                             const float **pose, const float **beam, int64_t *out)
{
    const DevJob &jb = jobs[find_job(jobs, n_jobs, g)];
    const uint32_t local = (uint32_t)(g - jb.ray_begin);
    const uint32_t nb = (uint32_t)jb.n_beams;
    const uint32_t e = udiv(local, jb.div_beams);
    const uint32_t q = local - e * nb;
    const uint32_t bm = tile_beam(jb, q);
    *pose = jb.poses + 12 * (int64_t)e;
    *beam = jb.dirs + 3 * (int64_t)bm;
    *out = jb.out_offset + (int64_t)e * nb + bm;
}

template <int MODE, int WAVES, int BLK>
__global__ __launch_bounds__(BLK, WAVES) void k_trace_defer(const DevJob *__restrict__ jobs,
                                                        int n_jobs, int64_t g0, int64_t total,
                                                        int batch, float *__restrict__ out_range,
                                                        int32_t *__restrict__ out_hit,
                                                        int32_t *__restrict__ out_nodes,
                                                        int32_t *__restrict__ out_tris)
{
    __shared__ DeferWave s_wave[BLK / 64];
    DeferWave &W = s_wave[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t g = g0 + (int64_t)blockIdx.x * BLK + threadIdx.x;
    const bool valid = g < total;
    LaneRay L;
    LaneStack<0, kStackQ8, BLK> S;
    S.lw = nullptr;
    bool trav = false;
    L.corrupt = false;
    L.n_tris = 0;
    L.n_nodes = 0;
    if (valid) {
        trav = setup_ray(jobs, n_jobs, g, L);
        W.o[0][lane] = L.r.o[0];
        W.o[1][lane] = L.r.o[1];
        W.o[2][lane] = L.r.o[2];
        W.s[0][lane] = L.r.Sx;
        W.s[1][lane] = L.r.Sy;
        W.s[2][lane] = L.r.Sz;
        W.k[lane] = L.r.kx | L.r.ky << 2 | L.r.kz << 4;
        W.tmin[lane] = L.t_min;
        W.tmax[lane] = L.t_max;
        W.tris[lane] = L.tris;
        // a one-triangle scene was tested in setup_ray
        W.best[lane] = L.best_leaf >= 0
                           ? ((unsigned long long)__float_as_uint(L.best_t + 0.0f) << 32) |
                                 (uint32_t)L.best_id
                           : kNoHit;
        W.best_leaf[lane] = L.best_leaf;
    } else {
        W.best[lane] = kNoHit;
        W.best_leaf[lane] = -1;
    }
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t qhead = 0, qtail = 0;   // wave-uniform ring positions in [0, kRing)
    while (true) {
        wave_sync_lds();
        const unsigned long long tb = __ballot(trav);
        uint32_t pend = qtail - qhead;
        if ((int32_t)pend < 0) pend += kRing;
        if (tb == 0 && pend == 0) break;
        if (pend >= 64u || pend >= (uint32_t)batch || tb == 0) {
            // triangle step: lane i tests queued pair i
            const uint32_t n = pend < 64u ? pend : 64u;
            unsigned long long cand = kNoHit;
            int owner = 0, leaf = 0;
            if ((uint32_t)lane < n) {
                uint32_t at = qhead + (uint32_t)lane;
                if (at >= (uint32_t)kRing) at -= kRing;
                const uint32_t pr = W.ring[at];
                owner = (int)(pr >> kLeafBits);
                leaf = (int)(pr & ((1u << kLeafBits) - 1u));
                RayW r;
                r.o[0] = W.o[0][owner];
                r.o[1] = W.o[1][owner];
                r.o[2] = W.o[2][owner];
                r.Sx = W.s[0][owner];
                r.Sy = W.s[1][owner];
                r.Sz = W.s[2][owner];
                const int kk = W.k[owner];
                r.kx = kk & 3;
                r.ky = (kk >> 2) & 3;
                r.kz = kk >> 4;
                const TriRec tr = load_tri(W.tris[owner], leaf);
                float t;
                if (woop32(r, tr.a, tr.b, tr.c, &t) && t >= W.tmin[owner] && t <= W.tmax[owner]) {
                    cand = ((unsigned long long)__float_as_uint(t + 0.0f) << 32) |
                           (uint32_t)__float_as_int(tr.c.y);
                    atomicMin(&W.best[owner], cand);
                }
            }
            wave_sync_lds();
            // the pair that now holds its owner's minimum records the leaf
            // (keys are unique: a leaf is queued at most once per ray)
            if (cand != kNoHit && W.best[owner] == cand) W.best_leaf[owner] = leaf;
            qhead += n;
            if (qhead >= (uint32_t)kRing) qhead -= kRing;
            wave_sync_lds();
            if (trav) {
                const unsigned long long b = W.best[lane];
                if (b != kNoHit) L.t_hi = __uint_as_float((uint32_t)(b >> 32)) * (1.0f + kCullRel);
            }
        } else {
            // node step
            int32_t ref[4];
            uint32_t lm = 0;
            if (trav) trav = !node_step_q8_collect<kStackQ8, BLK>(L, S, ref, &lm);
            const uint32_t cnt = (uint32_t)__popc(lm);
            L.n_tris += (int)cnt;
            const unsigned long long c0 = __ballot(cnt & 1u);
            const unsigned long long c1 = __ballot(cnt & 2u);
            const unsigned long long c2 = __ballot(cnt & 4u);
            uint32_t pos = qtail + lanes_below(c0 & below) + 2u * lanes_below(c1 & below) +
                           4u * lanes_below(c2 & below);
            const uint32_t added = (uint32_t)__popcll(c0) + 2u * (uint32_t)__popcll(c1) +
                                   4u * (uint32_t)__popcll(c2);
#pragma unroll 1
            while (lm != 0u) {
                const int k = __builtin_ctz(lm);
                lm &= lm - 1u;
                const int32_t rk = k == 0 ? ref[0] : (k == 1 ? ref[1] : (k == 2 ? ref[2] : ref[3]));
                const uint32_t at = pos >= (uint32_t)kRing ? pos - kRing : pos;
                W.ring[at] = (uint32_t)lane << kLeafBits | (uint32_t)(~rk);
                ++pos;
            }
            qtail += added;
            if (qtail >= (uint32_t)kRing) qtail -= kRing;
        }
    }
    if (!valid) return;
    const float *pose, *beam;
    ray_location(jobs, n_jobs, g, &pose, &beam, &L.out);
    L.pose = pose;
    L.beam = beam;
    const unsigned long long b = W.best[lane];
    if (b != kNoHit) {
        L.best_leaf = W.best_leaf[lane];
        L.best_t = __uint_as_float((uint32_t)(b >> 32));
        L.best_id = (int)(uint32_t)b;
    } else {
        L.best_leaf = -1;
    }
    finish_ray<MODE>(L, out_range, out_hit, out_nodes, out_tris);
}

// Persistent waves with per-XCD queues, stealing and ballot refill.  Each
// wave keeps a private pool of consecutive ray indices [pool_next, pool_end)
// in scalar registers and refills idle lanes from it; the pool itself is
// refilled with one atomic per chunk, the chunk shrinking with the work left
// in the queue (guided self-scheduling: 4 * remaining / waves, clamped to
// [64, chunk_max]) so the tail stays balanced.
template <int MODE, int FMT, int SS>
__global__ __launch_bounds__(kBlock) void k_trace_persistent(
    const DevJob *__restrict__ jobs, int n_jobs, WorkQueues *queues, int refill_min, int chunk_max,
    float *__restrict__ out_range, int32_t *__restrict__ out_hit,
    int32_t *__restrict__ out_nodes, int32_t *__restrict__ out_tris)
{
    __shared__ uint64_t s_stk[SS > 0 ? SS * kBlock : 1];
    const int lane = threadIdx.x & 63;
    const unsigned long long lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const unsigned long long n_waves = (unsigned long long)gridDim.x * (kBlock / 64);
    LaneRay L;
    LaneStack<SS, FMT == FMT_Q8 ? kStackQ8 : kStack, kBlock> S;
    S.lw = s_stk + threadIdx.x;
    int xq = blockIdx.x % kQueues;
    bool exhausted = false;   // wave-uniform
    bool active = false;
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
    while (true) {
        unsigned long long am = __ballot(active);
        if (!exhausted && 64 - __popcll(am) >= refill_min) {
            unsigned long long idle = ~am;
            for (int round = 0; round < 2 && idle != 0 && !exhausted; ++round) {
                if (pool_next >= pool_end) {
                    // new chunk: own XCD's range first, then steal
                    bool got = false;
                    for (int tries = 0; tries < kQueues && !got; ++tries) {
                        const int x = (xq + tries) % kQueues;
                        const unsigned long long e = queues->end[x];
                        const unsigned long long h = __hip_atomic_load(
                            &queues->head[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (h >= e) continue;
                        unsigned long long chunk = 4 * (e - h) / n_waves;
                        chunk = (chunk + 63) & ~63ull;
                        if (chunk < 64) chunk = 64;
                        if (chunk > (unsigned long long)chunk_max) chunk = chunk_max;
                        unsigned long long b = 0;
                        if (lane == 0) b = atomicAdd(&queues->head[x], chunk);
                        const unsigned int blo = __builtin_amdgcn_readfirstlane((unsigned int)b);
                        const unsigned int bhi =
                            __builtin_amdgcn_readfirstlane((unsigned int)(b >> 32));
                        b = ((unsigned long long)bhi << 32) | blo;
                        if (b < e) {
                            got = true;
                            pool_next = b;
                            pool_end = b + chunk < e ? b + chunk : e;
                            xq = x;
                        }
                    }
                    if (!got) {
                        exhausted = true;
                        break;
                    }
                }
                const unsigned long long avail = pool_end - pool_next;
                const unsigned long long want = (unsigned long long)__popcll(idle);
                const unsigned long long take = want < avail ? want : avail;
                const unsigned long long rank = __popcll(idle & lt_mask);
                const bool mine = ((idle >> lane) & 1ull) && rank < take;
                if (mine) {
                    active = setup_ray(jobs, n_jobs, (int64_t)(pool_next + rank), L);
                    if (!active) finish_ray<MODE>(L, out_range, out_hit, out_nodes, out_tris);
                }
                pool_next += take;
                idle &= ~__ballot(mine);
            }
            am = __ballot(active);
        }
        if (am == 0) {
            if (exhausted) break;
            continue;
        }
        while (true) {
            if (active) {
                if (visit_capped<FMT>(L, S)) {
                    finish_ray<MODE>(L, out_range, out_hit, out_nodes, out_tris);
                    active = false;
                }
            }
            am = __ballot(active);
            if (am == 0) break;
            if (!exhausted && 64 - __popcll(am) >= refill_min) break;
        }
    }
}

template <int MODE, int FMT, int SS>
hipError_t launch_persistent(const TraceConfig &cfg, const DevJob *jobs, int n_jobs,
                             WorkQueues *queues, float *out_range, int32_t *out_hit,
                             int32_t *out_nodes, int32_t *out_tris, hipStream_t s)
{
    static int cus = 0;
    static int occ = 0;
    if (cus == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
    }
    if (occ == 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void *>(k_trace_persistent<MODE, FMT, SS>), kBlock, 0);
        if (e != hipSuccess || occ < 1) occ = 1;
    }
    const int per_cu = cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : occ;
    int refill = cfg.refill_min < 1 ? 1 : (cfg.refill_min > 64 ? 64 : cfg.refill_min);
    const int chunk = cfg.chunk_max >= 64 ? cfg.chunk_max : 4096;
    hipLaunchKernelGGL((k_trace_persistent<MODE, FMT, SS>), dim3(cus * per_cu), dim3(kBlock), 0, s,
                       jobs, n_jobs, queues, refill, chunk, out_range, out_hit, out_nodes,
                       out_tris);
    return hipGetLastError();
}

template <int MODE, int FMT>
hipError_t launch_mode(const TraceConfig &cfg, const DevJob *jobs, int n_jobs, WorkQueues *queues,
                       int64_t total, float *out_range, int32_t *out_hit, int32_t *out_nodes,
                       int32_t *out_tris, hipStream_t s)
{
    if (cfg.persistent && MODE != TRACE_BRUTE) {
        switch (cfg.stack_lds) {
        case 8:
            return launch_persistent<MODE, FMT, 8>(cfg, jobs, n_jobs, queues, out_range, out_hit,
                                                   out_nodes, out_tris, s);
        case 24:
            return launch_persistent<MODE, FMT, 24>(cfg, jobs, n_jobs, queues, out_range, out_hit,
                                                    out_nodes, out_tris, s);
        default:
            return launch_persistent<MODE, FMT, 16>(cfg, jobs, n_jobs, queues, out_range, out_hit,
                                                    out_nodes, out_tris, s);
        }
    }
    // one thread per ray; a dispatch holds at most 2^32 work-items, so large
    // batches go out as several dispatches of kMaxRaysPerDispatch rays
    const int blk = cfg.group_waves == 4 ? 256 : 64;
    for (int64_t g0 = 0; g0 < total; g0 += kMaxRaysPerDispatch) {
        const int64_t n = total - g0 < kMaxRaysPerDispatch ? total - g0 : kMaxRaysPerDispatch;
        const dim3 grid((unsigned)((n + blk - 1) / blk));
#define RC_GRID2(SS_, W_, B_)                                                                \
        hipLaunchKernelGGL((k_trace<MODE, FMT, SS_, W_, B_>), grid, dim3(B_), 0, s, jobs,      \
                           n_jobs, g0, total, out_range, out_hit, out_nodes, out_tris)
#define RC_GRID(SS_, W_)                                                                     \
        if (blk == 256) RC_GRID2(SS_, W_, 256); else RC_GRID2(SS_, W_, 64)
#define RC_DEFER(W_, B_)                                                                     \
        hipLaunchKernelGGL((k_trace_defer<MODE, W_, B_>), grid, dim3(B_), 0, s, jobs, n_jobs,  \
                           g0, total, cfg.leaf_batch, out_range, out_hit, out_nodes, out_tris)
        if (MODE == TRACE_BRUTE) RC_GRID2(0, 1, 64);
        else if (FMT == FMT_Q8 && cfg.leaf_batch > 0) {
            if (blk == 256) { if (cfg.waves_cap) RC_DEFER(8, 256); else RC_DEFER(1, 256); }
            else { if (cfg.waves_cap) RC_DEFER(8, 64); else RC_DEFER(1, 64); }
        }
        else if (cfg.stack_lds == 0 && cfg.waves_cap) RC_GRID(0, 8);
        else if (cfg.stack_lds == 0) RC_GRID(0, 1);
        else if (cfg.stack_lds == 8 && cfg.waves_cap) RC_GRID(8, 8);
        else if (cfg.stack_lds == 8) RC_GRID(8, 1);
        else RC_GRID(16, 1);
#undef RC_DEFER
#undef RC_GRID
#undef RC_GRID2
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

namespace {
__global__ void k_queue_reset(WorkQueues *live, const WorkQueues *tmpl)
{
    const int i = threadIdx.x;
    if (i < kQueues) {
        live->head[i] = tmpl->head[i];
        live->end[i] = tmpl->end[i];
    }
}
}  // namespace

hipError_t queue_reset_launch(WorkQueues *live, const WorkQueues *tmpl, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, live, tmpl);
    return hipGetLastError();
}

void init_queues(WorkQueues &q, int64_t total_rays)
{
    for (int x = 0; x < kQueues; ++x) {
        q.head[x] = (unsigned long long)(total_rays * x / kQueues);
        q.end[x] = (unsigned long long)(total_rays * (x + 1) / kQueues);
    }
}

hipError_t trace_launch(int mode, int fmt, const TraceConfig &cfg, const DevJob *jobs,
                        int n_jobs, WorkQueues *queues, int64_t total_rays, float *out_range,
                        int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris, hipStream_t s)
{
    if (total_rays <= 0) return hipSuccess;
    if (mode == TRACE_BRUTE)
        return launch_mode<TRACE_BRUTE, FMT_BINARY>(cfg, jobs, n_jobs, queues, total_rays,
                                                    out_range, out_hit, out_nodes, out_tris, s);
    if (fmt == FMT_Q8) {
        if (mode == TRACE_BVH)
            return launch_mode<TRACE_BVH, FMT_Q8>(cfg, jobs, n_jobs, queues, total_rays,
                                                  out_range, out_hit, out_nodes, out_tris, s);
        return launch_mode<TRACE_STATS, FMT_Q8>(cfg, jobs, n_jobs, queues, total_rays, out_range,
                                                out_hit, out_nodes, out_tris, s);
    }
    if (mode == TRACE_BVH)
        return launch_mode<TRACE_BVH, FMT_BINARY>(cfg, jobs, n_jobs, queues, total_rays,
                                                  out_range, out_hit, out_nodes, out_tris, s);
    return launch_mode<TRACE_STATS, FMT_BINARY>(cfg, jobs, n_jobs, queues, total_rays, out_range,
                                                out_hit, out_nodes, out_tris, s);
}
