// trace.hip -- batched LiDAR ray casting kernels (gfx950).
//
// FGGS-LiDAR Sec. IV-C: one lane per beam; each ray r_j(t) = t_s + t R_s d_j
// walks the triangle LBVH near-child first and discards every node whose
// entry distance exceeds the best hit so far (and every triangle beyond it);
// the result is the nearest intersection t*_j over [t_min, t_max].
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
//    lowest id whatever the visit order: the BVH kernel and the brute-force
//    kernel agree bit for bit.
//  * The winner's range is recomputed in FP64 from the FP64 ray and the
//    triangle's plane, then rounded to FP32.
#include "rc_internal.h"

#include <math.h>

namespace {

constexpr int kBlock = 256;
constexpr int kStack = 64;           // >= depth of any Karras tree (62 key bits)
constexpr float kErrU = 2.384185791015625e-07f;  // 2^-22: sign certificate factor
constexpr float kBoxGrow = 1.0f + 3.5762786865234375e-07f * 2.0f;  // > 1 + 2 gamma_3
constexpr float kCullRel = 6.103515625e-05f;     // 2^-14 relative culling margin

struct RayW {
    float o[3];        // origin, permuted (kx, ky, kz)
    float Sx, Sy, Sz;  // shear constants
    int kx, ky, kz;
    float org[3];      // origin, world axes
    float inv[3];      // 1 / direction, world axes (clamped away from 0)
};

__device__ __forceinline__ float sel3(float a, float b, float c, int k)
{
    return k == 0 ? a : (k == 1 ? b : c);
}

__device__ __forceinline__ void make_ray(const DevJob &jb, int64_t local, RayW &r, float d32[3])
{
    const uint32_t nb = (uint32_t)jb.n_beams;
    const uint32_t e = (uint32_t)(local / nb);
    const uint32_t j = (uint32_t)(local - (int64_t)e * nb);
    const float *p = jb.poses + 12 * (int64_t)e;
    const float *b = jb.dirs + 3 * (int64_t)j;
    double bx = b[0], by = b[1], bz = b[2];
    double d[3];
    for (int i = 0; i < 3; ++i)
        d[i] = (double)p[4 * i + 0] * bx + (double)p[4 * i + 1] * by + (double)p[4 * i + 2] * bz;
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) d32[i] = (float)(d[i] / n);
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
__device__ __noinline__ bool woop64(float Ax, float Ay, float Bx, float By, float Cx, float Cy,
                                    float Az, float Bz, float Cz, float Sz, float *t_out)
{
    double U = (double)Cx * (double)By - (double)Cy * (double)Bx;
    double V = (double)Ax * (double)Cy - (double)Ay * (double)Cx;
    double W = (double)Bx * (double)Ay - (double)By * (double)Ax;
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return false;
    double det = U + V + W;
    if (det == 0.0) return false;
    double T = U * ((double)Sz * (double)Az) + V * ((double)Sz * (double)Bz) +
               W * ((double)Sz * (double)Cz);
    *t_out = (float)(T / det);
    return true;
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
    const float Ax = A_x - r.Sx * A_z, Ay = A_y - r.Sy * A_z;
    const float Bx = B_x - r.Sx * B_z, By = B_y - r.Sy * B_z;
    const float Cx = C_x - r.Sx * C_z, Cy = C_y - r.Sy * C_z;
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
    if (!((pU || nU) && (pV || nV) && (pW || nW)))
        return woop64(Ax, Ay, Bx, By, Cx, Cy, A_z, B_z, C_z, r.Sz, t_out);
    // all three signs certain and equal
    const float det = U + V + W;
    const float T = U * (r.Sz * A_z) + V * (r.Sz * B_z) + W * (r.Sz * C_z);
    *t_out = T / det;
    return true;
}

__device__ __forceinline__ bool better(float t, int id, float bt, int bid)
{
    return t < bt || (t == bt && id < bid);
}

// FP64 range of the winning triangle along the FP64 ray (plane equation).
__device__ float refine_range(const DevJob &jb, int64_t local, const TriRec &tr, float t32)
{
    const uint32_t nb = (uint32_t)jb.n_beams;
    const uint32_t e = (uint32_t)(local / nb);
    const uint32_t j = (uint32_t)(local - (int64_t)e * nb);
    const float *p = jb.poses + 12 * (int64_t)e;
    const float *b = jb.dirs + 3 * (int64_t)j;
    double d[3];
    for (int i = 0; i < 3; ++i)
        d[i] = (double)p[4 * i + 0] * (double)b[0] + (double)p[4 * i + 1] * (double)b[1] +
               (double)p[4 * i + 2] * (double)b[2];
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) d[i] /= n;
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
    const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * kBoxGrow;
    return (tn <= tf && tn <= t_hi) ? tn : INFINITY;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_trace(const DevJob *__restrict__ jobs, int n_jobs,
                                                  int64_t total, float *__restrict__ out_range,
                                                  int32_t *__restrict__ out_hit,
                                                  int32_t *__restrict__ out_nodes,
                                                  int32_t *__restrict__ out_tris)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const DevJob jb = jobs[find_job(jobs, n_jobs, g)];
    const int64_t local = g - jb.ray_begin;
    RayW r;
    float d32[3];
    make_ray(jb, local, r, d32);

    float best_t = INFINITY;
    int best_id = 0x7fffffff;
    int best_leaf = -1;
    int n_nodes = 0, n_tris = 0;
    bool corrupt = false;
    const float t_min = jb.t_min, t_max = jb.t_max;
    const float t_lo = t_min * (1.0f - kCullRel);
    float t_hi = t_max * (1.0f + kCullRel);

    auto test_leaf = [&](int leaf) {
        const TriRec tr = jb.tris[leaf];
        float t;
        ++n_tris;
        if (woop32(r, tr.a, tr.b, tr.c, &t) && t >= t_min && t <= t_max) {
            const int id = __float_as_int(tr.c.y);
            if (better(t, id, best_t, best_id)) {
                best_t = t;
                best_id = id;
                best_leaf = leaf;
                t_hi = best_t * (1.0f + kCullRel);
            }
        }
    };

    if (MODE == TRACE_BRUTE) {
        for (int k = 0; k < jb.n_tris; ++k) test_leaf(k);
    } else if (jb.n_tris > 0) {
        if (jb.root_leaf) {
            test_leaf(0);
        } else {
            int stack_node[kStack];
            float stack_t[kStack];
            int sp = 0;
            int node = 0;
            // a correct traversal fetches each of the n_tris - 1 records at
            // most once; the cap only guards against a corrupted tree
            const int max_fetch = jb.n_tris + 64;
            int fetched = 0;
            while (true) {
                if (++fetched > max_fetch) { corrupt = true; break; }
                const NodeRec nd = jb.nodes[node];
                ++n_nodes;
                const float tl = slab(r, nd.q0.x, nd.q0.y, nd.q1.x, nd.q1.y, nd.q2.x, nd.q2.y,
                                      t_lo, t_hi);
                const float tr = slab(r, nd.q0.z, nd.q0.w, nd.q1.z, nd.q1.w, nd.q2.z, nd.q2.w,
                                      t_lo, t_hi);
                int cl = nd.q3.x, cr = nd.q3.y;
                bool hl = tl < INFINITY, hr = tr < INFINITY;
                // leaves are tested on the spot, nearer one first
                if (hl && cl < 0 && hr && cr < 0) {
                    if (tl <= tr) { test_leaf(~cl); if (tr <= t_hi) test_leaf(~cr); }
                    else { test_leaf(~cr); if (tl <= t_hi) test_leaf(~cl); }
                    hl = hr = false;
                } else {
                    if (hl && cl < 0) { test_leaf(~cl); hl = false; }
                    if (hr && cr < 0) { test_leaf(~cr); hr = false; }
                }
                hl = hl && tl <= t_hi;
                hr = hr && tr <= t_hi;
                if (hl && hr) {
                    const bool lnear = tl <= tr;
                    node = lnear ? cl : cr;
                    if (sp == kStack) { corrupt = true; break; }  // deeper than any Karras tree
                    stack_node[sp] = lnear ? cr : cl;
                    stack_t[sp] = lnear ? tr : tl;
                    ++sp;
                    continue;
                }
                if (hl) { node = cl; continue; }
                if (hr) { node = cr; continue; }
                // pop the nearest pending subtree still in range
                bool found = false;
                while (sp > 0) {
                    --sp;
                    if (stack_t[sp] <= t_hi) { node = stack_node[sp]; found = true; break; }
                }
                if (!found) break;
            }
        }
    }
    const int64_t o = jb.out_offset + local;
    if (corrupt) {
        out_range[o] = NAN;  // never a valid result: flags a broken hierarchy
        out_hit[o] = -2;
    } else if (best_leaf >= 0) {
        const TriRec tr = jb.tris[best_leaf];
        out_range[o] = refine_range(jb, local, tr, best_t);
        out_hit[o] = best_id;
    } else {
        out_range[o] = INFINITY;
        out_hit[o] = -1;
    }
    if (MODE == TRACE_STATS) {
        out_nodes[o] = n_nodes;
        out_tris[o] = n_tris;
    }
}

}  // namespace

hipError_t trace_launch(int mode, const DevJob *jobs, int n_jobs, int64_t total_rays,
                        float *out_range, int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris,
                        hipStream_t s)
{
    if (total_rays <= 0) return hipSuccess;
    const dim3 grid((unsigned)((total_rays + kBlock - 1) / kBlock));
    if (mode == TRACE_BVH)
        hipLaunchKernelGGL(k_trace<TRACE_BVH>, grid, dim3(kBlock), 0, s, jobs, n_jobs, total_rays,
                           out_range, out_hit, out_nodes, out_tris);
    else if (mode == TRACE_BRUTE)
        hipLaunchKernelGGL(k_trace<TRACE_BRUTE>, grid, dim3(kBlock), 0, s, jobs, n_jobs,
                           total_rays, out_range, out_hit, out_nodes, out_tris);
    else
        hipLaunchKernelGGL(k_trace<TRACE_STATS>, grid, dim3(kBlock), 0, s, jobs, n_jobs,
                           total_rays, out_range, out_hit, out_nodes, out_tris);
    return hipGetLastError();
}
