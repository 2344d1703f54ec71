// meshopt.hip -- Taubin smoothing of a triangle mesh on gfx950 (FGGS-LiDAR
// Sec. IV-B, "Mesh optimization"; defaults of Sec. V).
//
//   N(i)   distinct vertices sharing an edge with i (never i itself)
//   L(x)_i (sum over N(i) of x_j) / |N(i)| - x_i  (umbrella operator)
//   x <- x + lambda L(x), then x <- x + mu L(x), per iteration; vertices on
//   an edge of a single triangle (the boundary) and vertices without
//   neighbours stay in place.
//
// Decimation: quadric-error vertex clustering (see decimate_emit below).
// Removal of tiny components: union-find labels, per-component face counts,
// stable compaction (see the components kernels below).
//
// Neighbour lists: every triangle appends its two other corners to each
// corner's slots (atomic slot counter, at most kNbrCap per vertex); each
// vertex then sorts its slots, keeps distinct entries and marks itself
// fixed when one of them occurred only once (a boundary edge).  Sorting
// makes the lists independent of the append order, and the half-steps sum
// neighbours in ascending index order, one rounded float32 operation at a
// time, so results are deterministic and reproducible on the CPU.
#include "mesh_internal.h"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Ascending sort of one vertex's n slot entries.  Up to 16 entries (nearly
// every vertex) are sorted in registers by a bitonic network, unrolled so
// that every index is a constant; longer lists are sorted in place in
// global memory (a per-thread array of kNbrCap entries would live in
// scratch memory).
constexpr int kRegSort = 16;

__device__ __forceinline__ void sort16(int32_t (&r)[kRegSort])
{
#pragma unroll
    for (int k = 2; k <= kRegSort; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < kRegSort; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t a = r[i], b = r[l];
                    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    const bool up = (i & k) == 0;
                    r[i] = up ? lo : hi;
                    r[l] = up ? hi : lo;
                }
            }
}

// sorts s[0..n) and returns true with the sorted values in r when n fits
// the registers; otherwise sorts s in place and returns false
__device__ __forceinline__ bool sort_slots(int32_t *__restrict__ s, int n, int32_t (&r)[kRegSort])
{
    if (n <= kRegSort) {
#pragma unroll
        for (int k = 0; k < kRegSort; ++k) r[k] = k < n ? s[k] : INT32_MAX;
        sort16(r);
        return true;
    }
    for (int k = 1; k < n; ++k) {
        const int32_t x = s[k];
        int j = k;
        while (j > 0 && s[j - 1] > x) {
            s[j] = s[j - 1];
            --j;
        }
        s[j] = x;
    }
    return false;
}

__global__ __launch_bounds__(kBlock) void k_nbr_fill(const int32_t *__restrict__ tris, int64_t nt,
                                                     int32_t *__restrict__ slots,
                                                     uint32_t *__restrict__ cnt,
                                                     int32_t *__restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const int32_t c[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    for (int k = 0; k < 3; ++k) {
        const int32_t v = c[k];
        const int32_t u0 = c[(k + 1) % 3], u1 = c[(k + 2) % 3];
        const bool w0 = u0 != v, w1 = u1 != v;
        const uint32_t nw = (w0 ? 1u : 0u) + (w1 ? 1u : 0u);
        if (!nw) continue;
        // one atomic reserves both slots of this corner
        uint32_t at = atomicAdd(&cnt[v], nw);
        if (at + nw > (uint32_t)kNbrCap) {
            atomicOr(flags, 1);
            continue;
        }
        int32_t *sv = slots + (int64_t)v * kNbrCap;
        if (w0) sv[at++] = u0;
        if (w1) sv[at] = u1;
    }
}

__global__ __launch_bounds__(kBlock) void k_nbr_finalize(int32_t *__restrict__ slots,
                                                         const uint32_t *__restrict__ cnt,
                                                         int64_t nv, int32_t *__restrict__ deg,
                                                         uint8_t *__restrict__ fixed)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const int n = cnt[v] < (uint32_t)kNbrCap ? (int)cnt[v] : kNbrCap;
    int32_t *s = slots + v * kNbrCap;
    int32_t r[kRegSort];
    int m = 0, run = 0;
    bool boundary = false;       // some neighbour occurs once: its edge lies in one triangle
    if (sort_slots(s, n, r)) {
#pragma unroll
        for (int k = 0; k < kRegSort; ++k) {
            if (k < n) {
                if (k == 0 || r[k] != r[k - 1]) {
                    if (run == 1) boundary = true;
                    s[m++] = r[k];
                    run = 1;
                } else {
                    ++run;
                }
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            const int32_t x = s[k];
            if (k == 0 || x != s[m - 1]) {
                if (run == 1) boundary = true;
                s[m++] = x;
                run = 1;
            } else {
                ++run;
            }
        }
    }
    if (run == 1) boundary = true;
    deg[v] = m;
    fixed[v] = (boundary || m == 0) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_umbrella(const float *__restrict__ src,
                                                     float *__restrict__ dst,
                                                     const int32_t *__restrict__ slots,
                                                     const int32_t *__restrict__ deg,
                                                     const uint8_t *__restrict__ fixed, int64_t nv,
                                                     float f)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const float x = src[3 * v], y = src[3 * v + 1], z = src[3 * v + 2];
    if (fixed[v]) {
        dst[3 * v] = x;
        dst[3 * v + 1] = y;
        dst[3 * v + 2] = z;
        return;
    }
    const int n = deg[v];
    const int32_t *s = slots + v * kNbrCap;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (int k = 0; k < n; ++k) {
        const int64_t u = s[k];
        ax = __fadd_rn(ax, src[3 * u]);
        ay = __fadd_rn(ay, src[3 * u + 1]);
        az = __fadd_rn(az, src[3 * u + 2]);
    }
    const float dn = (float)n;
    const float mx = __fdiv_rn(ax, dn), my = __fdiv_rn(ay, dn), mz = __fdiv_rn(az, dn);
    dst[3 * v] = __fadd_rn(x, __fmul_rn(f, __fsub_rn(mx, x)));
    dst[3 * v + 1] = __fadd_rn(y, __fmul_rn(f, __fsub_rn(my, y)));
    dst[3 * v + 2] = __fadd_rn(z, __fmul_rn(f, __fsub_rn(mz, z)));
}

}  // namespace

hipError_t nbr_build_launch(const int32_t *tris, int64_t nt, int64_t nv, int32_t *slots,
                            uint32_t *cnt, int32_t *deg, uint8_t *fixed, int32_t *flags,
                            hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * nv, s);
    if (e != hipSuccess) return e;
    if (nt > 0)
        hipLaunchKernelGGL(k_nbr_fill, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt,
                           slots, cnt, flags);
    hipLaunchKernelGGL(k_nbr_finalize, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, slots,
                           cnt, nv, deg, fixed);
    return hipGetLastError();
}

hipError_t taubin_launch(float *verts, float *tmp, const int32_t *slots, const int32_t *deg,
                         const uint8_t *fixed, int64_t nv, float lambda, float mu, int iterations,
                         hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    const unsigned g = grid_for(nv, kBlock);
    for (int it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(k_umbrella, dim3(g), dim3(kBlock), 0, s, verts, tmp, slots, deg, fixed,
                           nv, lambda);
        hipLaunchKernelGGL(k_umbrella, dim3(g), dim3(kBlock), 0, s, tmp, verts, slots, deg, fixed,
                           nv, mu);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quadric-error decimation by vertex clustering.
//
// Every vertex gets the sum Q of the area-weighted plane quadrics of its
// incident triangles (ascending triangle index).  For a cell size c, the
// vertices are keyed by their cell of a grid anchored at the mesh's box
// minimum (boundary vertices, on an edge of one triangle, keep groups of
// their own) and sorted stably by key, which puts every group's vertices
// together in ascending index order; a triangle survives when its corners
// lie in three groups.  Each surviving group becomes one vertex at the
// minimiser of its summed quadric (Cramer's rule when the matrix is well
// conditioned and the point stays within the group's cell widened by one
// cell), else at its members' mean.  All sums run in fixed orders in FP64,
// so the mesh is deterministic.
namespace {

__global__ __launch_bounds__(kBlock) void k_tri_fill(const int32_t *__restrict__ tris, int64_t nt,
                                                     int32_t *__restrict__ slots,
                                                     uint32_t *__restrict__ cnt,
                                                     int32_t *__restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const int32_t c[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    for (int k = 0; k < 3; ++k) {
        if ((k > 0 && c[k] == c[0]) || (k > 1 && c[k] == c[1])) continue;   // distinct corners
        const uint32_t at = atomicAdd(&cnt[c[k]], 1u);
        if (at < (uint32_t)kNbrCap) slots[(int64_t)c[k] * kNbrCap + at] = (int32_t)t;
        else atomicOr(flags, 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_tri_sort(int32_t *__restrict__ slots,
                                                     const uint32_t *__restrict__ cnt, int64_t nv,
                                                     int32_t *__restrict__ tdeg)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const int n = cnt[v] < (uint32_t)kNbrCap ? (int)cnt[v] : kNbrCap;
    int32_t *s = slots + v * kNbrCap;
    int32_t r[kRegSort];
    if (sort_slots(s, n, r)) {
#pragma unroll
        for (int k = 0; k < kRegSort; ++k)
            if (k < n) s[k] = r[k];
    }
    tdeg[v] = n;
}

// Boundary flags of the decimation from the sorted incident-triangle
// lists: a vertex is on the boundary when some neighbour is reached through
// exactly one of its triangles.  Per triangle t and vertex v the neighbour
// entries are the two other corners when v is one corner, the third corner
// twice when v is two corners, and none for three (the same multiset the
// neighbour lists of the smoothing collect).  Computed in
// k_vertex_quadrics: up to 8 triangles, the 16 entries sit in fixed
// register slots and are sorted by the bitonic network; larger fans count
// each entry's multiplicity by re-reading their triangles.  More than
// kNbrCap / 2 triangles set flags (the limit of the neighbour lists this
// replaces).
__device__ __forceinline__ void tri_entries(const int32_t *__restrict__ tris, int32_t t, int32_t v,
                                            int32_t &e0, int32_t &e1)
{
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    const int n = (a == v ? 1 : 0) + (b == v ? 1 : 0) + (c == v ? 1 : 0);
    if (n == 1) {
        if (a == v) { e0 = b; e1 = c; }
        else if (b == v) { e0 = c; e1 = a; }
        else { e0 = a; e1 = b; }
    } else if (n == 2) {
        const int32_t u = a != v ? a : (b != v ? b : c);
        e0 = u;
        e1 = u;
    } else {
        e0 = INT32_MAX;       // no entry (no vertex index reaches INT32_MAX)
        e1 = INT32_MAX;
    }
}

// area-weighted plane quadric of triangle t (upper triangle of the 4x4
// matrix, row by row), in a fixed operation order
__device__ void face_quadric(const float *__restrict__ verts, int64_t ia, int64_t ib, int64_t ic,
                             double K[10])
{
    const double ax = verts[3 * ia], ay = verts[3 * ia + 1], az = verts[3 * ia + 2];
    const double e1x = (double)verts[3 * ib] - ax, e1y = (double)verts[3 * ib + 1] - ay,
                 e1z = (double)verts[3 * ib + 2] - az;
    const double e2x = (double)verts[3 * ic] - ax, e2y = (double)verts[3 * ic + 1] - ay,
                 e2z = (double)verts[3 * ic + 2] - az;
    const double nx = e1y * e2z - e1z * e2y;
    const double ny = e1z * e2x - e1x * e2z;
    const double nz = e1x * e2y - e1y * e2x;
    const double ln = sqrt((nx * nx + ny * ny) + nz * nz);
    if (!(ln > 0.0)) {
        for (int k = 0; k < 10; ++k) K[k] = 0.0;
        return;
    }
    const double ux = nx / ln, uy = ny / ln, uz = nz / ln;
    const double d = -((ux * ax + uy * ay) + uz * az);
    const double w = 0.5 * ln;
    const double p[4] = {ux, uy, uz, d};
    int k = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) K[k++] = w * (p[i] * p[j]);
}

// the two neighbour entries of triangle (a, b, c) for vertex v (see
// tri_entries)
__device__ __forceinline__ void corner_entries(int32_t a, int32_t b, int32_t c, int32_t v,
                                               int32_t &e0, int32_t &e1)
{
    const int n = (a == v ? 1 : 0) + (b == v ? 1 : 0) + (c == v ? 1 : 0);
    if (n == 1) {
        if (a == v) { e0 = b; e1 = c; }
        else if (b == v) { e0 = c; e1 = a; }
        else { e0 = a; e1 = b; }
    } else if (n == 2) {
        const int32_t u = a != v ? a : (b != v ? b : c);
        e0 = u;
        e1 = u;
    } else {
        e0 = INT32_MAX;
        e1 = INT32_MAX;
    }
}

// Per vertex: the sum of its triangles' quadrics in ascending triangle
// order, and its boundary flag (the test described above), from one
// gather of each incident triangle.
__global__ __launch_bounds__(kBlock) void k_vertex_quadrics(const float *__restrict__ verts,
                                                            const int32_t *__restrict__ tris,
                                                            const int32_t *__restrict__ slots,
                                                            const int32_t *__restrict__ tdeg,
                                                            int64_t nv, double *__restrict__ Q,
                                                            uint8_t *__restrict__ bnd,
                                                            int32_t *__restrict__ flags)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    double q[10];
    for (int k = 0; k < 10; ++k) q[k] = 0.0;
    const int n = tdeg[v];
    const int32_t *s = slots + v * kNbrCap;
    const int32_t vv = (int32_t)v;
    if (n > kNbrCap / 2) atomicOr(flags, 1);
    int32_t r[kRegSort];
#pragma unroll
    for (int i = 0; i < kRegSort / 2; ++i) {
        int32_t e0 = INT32_MAX, e1 = INT32_MAX;
        if (i < n) {
            const int32_t t = s[i];
            const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
            double K[10];
            face_quadric(verts, a, b, c, K);
            for (int k = 0; k < 10; ++k) q[k] = q[k] + K[k];
            corner_entries(a, b, c, vv, e0, e1);
        }
        r[2 * i] = e0;
        r[2 * i + 1] = e1;
    }
    for (int j = kRegSort / 2; j < n; ++j) {
        const int32_t t = s[j];
        double K[10];
        face_quadric(verts, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2], K);
        for (int k = 0; k < 10; ++k) q[k] = q[k] + K[k];
    }
    for (int k = 0; k < 10; ++k) Q[10 * v + k] = q[k];
    bool boundary = false;
    if (n <= kRegSort / 2) {
        sort16(r);
        int run = 0;
#pragma unroll
        for (int k = 0; k < kRegSort; ++k) {
            if (r[k] == INT32_MAX) continue;
            if (k == 0 || r[k] != r[k - 1]) {
                if (run == 1) boundary = true;
                run = 1;
            } else {
                ++run;
            }
        }
        if (run == 1) boundary = true;
    } else if (n <= kNbrCap / 2) {
        const int E = 2 * n;
        for (int e = 0; e < E && !boundary; ++e) {
            int32_t x0, x1;
            tri_entries(tris, s[e >> 1], vv, x0, x1);
            const int32_t x = (e & 1) ? x1 : x0;
            if (x == INT32_MAX) continue;
            int cnt = 0;
            for (int f = 0; f < E && cnt < 2; ++f) {
                int32_t y0, y1;
                tri_entries(tris, s[f >> 1], vv, y0, y1);
                if (((f & 1) ? y1 : y0) == x) ++cnt;
            }
            if (cnt == 1) boundary = true;
        }
    }
    bnd[v] = boundary ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_points_minmax(const float *__restrict__ verts,
                                                          int64_t nv, float *__restrict__ partial)
{
    __shared__ float red[kBlock][6];
    float acc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * kBlock)
        for (int a = 0; a < 3; ++a) {
            acc[a] = fminf(acc[a], verts[3 * i + a]);
            acc[3 + a] = fmaxf(acc[3 + a], verts[3 * i + a]);
        }
    for (int a = 0; a < 6; ++a) red[threadIdx.x][a] = acc[a];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 6; ++a)
                red[threadIdx.x][a] = a < 3 ? fminf(red[threadIdx.x][a], red[threadIdx.x + w][a])
                                            : fmaxf(red[threadIdx.x][a], red[threadIdx.x + w][a]);
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void k_points_final(const float *__restrict__ partial, int nb, float *__restrict__ out)
{
    const int a = threadIdx.x;
    if (a >= 6) return;
    float v = partial[a];
    for (int b = 1; b < nb; ++b) v = a < 3 ? fminf(v, partial[6 * b + a]) : fmaxf(v, partial[6 * b + a]);
    out[a] = v;
}

__device__ __forceinline__ int64_t cell_of(double x, double lo, double c)
{
    return (int64_t)floor((x - lo) / c);
}

__global__ __launch_bounds__(kBlock) void k_cell_keys(const float *__restrict__ verts, int64_t nv,
                                                      const uint8_t *__restrict__ bnd,
                                                      const double *__restrict__ lo, double c,
                                                      int64_t n0, int64_t n1,
                                                      uint32_t *__restrict__ keys,
                                                      uint32_t *__restrict__ vals)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    uint32_t key = kBoundaryKey;
    if (!bnd[v]) {
        const int64_t ix = cell_of(verts[3 * v], lo[0], c), iy = cell_of(verts[3 * v + 1], lo[1], c),
                      iz = cell_of(verts[3 * v + 2], lo[2], c);
        key = (uint32_t)(ix + n0 * (iy + n1 * iz));
    }
    keys[v] = key;
    vals[v] = (uint32_t)v;
}

// Kept-triangle count for one cell size, without grouping: two corners
// share a group exactly when they are the same vertex, or when their cell
// keys are equal and not the boundary key (boundary vertices are groups of
// their own).  A triangle is kept when its three corners are in three
// groups.  Grid-stride blocks write partial counts and one block adds them
// (one atomic per block on a single counter serialised: 0.23 ms at 26k
// blocks).
constexpr int kCountBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_count_kept(const int32_t *__restrict__ tris, int64_t nt,
                                                       const uint32_t *__restrict__ keys,
                                                       uint32_t *__restrict__ partial)
{
    __shared__ uint32_t wsum[kBlock / 64];
    uint32_t n = 0;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nt;
         t += (int64_t)gridDim.x * kBlock) {
        const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
        const uint32_t ka = keys[a], kb = keys[b], kc = keys[c];
        const bool ab = a == b || (ka == kb && ka != kBoundaryKey);
        const bool bc = b == c || (kb == kc && kb != kBoundaryKey);
        const bool ca = c == a || (kc == ka && kc != kBoundaryKey);
        n += (!ab && !bc && !ca) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (int w = 0; w < kBlock / 64; ++w) sum += wsum[w];
        partial[blockIdx.x] = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_count_final(const uint32_t *__restrict__ partial,
                                                        int nb, uint32_t *__restrict__ count)
{
    __shared__ uint32_t wsum[kBlock / 64];
    uint32_t n = 0;
    for (int i = threadIdx.x; i < nb; i += kBlock) n += partial[i];
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (int w = 0; w < kBlock / 64; ++w) sum += wsum[w];
        *count = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_group_flags(const uint32_t *__restrict__ keys,
                                                        int64_t nv, uint32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nv) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1] || keys[i] == kBoundaryKey) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_group_ids(const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ flag,
                                                      const uint32_t *__restrict__ gpos, int64_t nv,
                                                      uint32_t *__restrict__ gid,
                                                      uint32_t *__restrict__ gstart)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nv) return;
    const uint32_t g = gpos[i] + flag[i] - 1u;
    gid[vals[i]] = g;
    if (flag[i]) gstart[g] = (uint32_t)i;
    if (i == nv - 1) gstart[g + 1] = (uint32_t)nv;
}

__global__ __launch_bounds__(kBlock) void k_keep(const int32_t *__restrict__ tris, int64_t nt,
                                                 const uint32_t *__restrict__ gid,
                                                 uint32_t *__restrict__ keep,
                                                 uint32_t *__restrict__ used)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const uint32_t a = gid[tris[3 * t]], b = gid[tris[3 * t + 1]], c = gid[tris[3 * t + 2]];
    const bool k = a != b && b != c && a != c;
    keep[t] = k ? 1u : 0u;
    if (k) {
        used[a] = 1u;
        used[b] = 1u;
        used[c] = 1u;
    }
}

__global__ __launch_bounds__(kBlock) void k_emit_groups(const float *__restrict__ verts,
                                                        const double *__restrict__ Q,
                                                        const uint8_t *__restrict__ bnd,
                                                        const uint32_t *__restrict__ vals,
                                                        const uint32_t *__restrict__ gstart,
                                                        int64_t ngroups,
                                                        const uint32_t *__restrict__ used,
                                                        const uint32_t *__restrict__ newid,
                                                        const double *__restrict__ lo, double c,
                                                        float *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= ngroups || !used[g]) return;
    const uint32_t b = gstart[g], e = gstart[g + 1];
    const int64_t v0 = vals[b];
    float *o = out + 3 * (int64_t)newid[g];
    if (bnd[v0]) {
        o[0] = verts[3 * v0];
        o[1] = verts[3 * v0 + 1];
        o[2] = verts[3 * v0 + 2];
        return;
    }
    double q[10];
    for (int k = 0; k < 10; ++k) q[k] = 0.0;
    for (uint32_t i = b; i < e; ++i) {
        const int64_t v = vals[i];
        for (int k = 0; k < 10; ++k) q[k] = q[k] + Q[10 * v + k];
    }
    const double a00 = q[0], a01 = q[1], a02 = q[2], b0 = -q[3];
    const double a11 = q[4], a12 = q[5], b1 = -q[6];
    const double a22 = q[7], b2 = -q[8];
    const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
                       a02 * (a01 * a12 - a11 * a02);
    const double tr = (a00 + a11) + a22;
    const double t3 = tr / 3.0;
    if (tr > 0.0 && fabs(det) > 1e-6 * ((t3 * t3) * t3)) {
        const double x0 = (b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2) +
                           a02 * (b1 * a12 - a11 * b2)) / det;
        const double x1 = (a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02) +
                           a02 * (a01 * b2 - b1 * a02)) / det;
        const double x2 = (a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02) +
                           b0 * (a01 * a12 - a11 * a02)) / det;
        const double x[3] = {x0, x1, x2};
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            const int64_t ci = cell_of(verts[3 * v0 + a], lo[a], c);
            const double cmin = lo[a] + (double)(ci - 1) * c;
            const double cmax = lo[a] + (double)(ci + 2) * c;
            inside = inside && x[a] >= cmin && x[a] <= cmax;
        }
        if (inside) {
            o[0] = (float)x0;
            o[1] = (float)x1;
            o[2] = (float)x2;
            return;
        }
    }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (uint32_t i = b; i < e; ++i) {
        const int64_t v = vals[i];
        sx = sx + (double)verts[3 * v];
        sy = sy + (double)verts[3 * v + 1];
        sz = sz + (double)verts[3 * v + 2];
    }
    const double m = (double)(e - b);
    o[0] = (float)(sx / m);
    o[1] = (float)(sy / m);
    o[2] = (float)(sz / m);
}

__global__ __launch_bounds__(kBlock) void k_emit_tris(const int32_t *__restrict__ tris, int64_t nt,
                                                      const uint32_t *__restrict__ gid,
                                                      const uint32_t *__restrict__ keep,
                                                      const uint32_t *__restrict__ tpos,
                                                      const uint32_t *__restrict__ newid,
                                                      int32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt || !keep[t]) return;
    const int64_t p = tpos[t];
    for (int k = 0; k < 3; ++k) out[3 * p + k] = (int32_t)newid[gid[tris[3 * t + k]]];
}


// ---- connected components and removal of tiny ones ------------------------
// Lock-free union-find over the vertices, one thread per triangle joining
// its corners.  Roots are ranked by a bijective hash of their index, and a
// root is only ever hooked under a root of lower rank (CAS on its own parent
// slot): ranks strictly decrease along every chain, so every loop ends, and
// a failed CAS means another thread hooked that root.  Hashed ranks behave
// like random linking and keep trees shallow; ranking by index instead
// builds chains as long as the mesh on spatially ordered vertices.  Which
// vertex ends up as a root depends on thread timing, but the partition does
// not, and only the partition reaches the output.
//
// Parent loads are plain (cached) loads.  A stale value is an earlier
// parent, still an ancestor of lower rank, so walks still end; the CAS
// compares against the current value and hands back a fresh one when it
// fails.  Coherent loads sent every find of the giant component to the one
// L2 line holding its root.

__device__ __forceinline__ uint32_t cc_load(const uint32_t *p) { return *p; }

// a bijection of 32-bit integers (odd multiplies and xor-shifts)
__device__ __forceinline__ uint32_t cc_rank(uint32_t x)
{
    x *= 0x9E3779B1u;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    return x;
}

// root of x.  Read-only: linking by random rank keeps the expected depth
// logarithmic without compression, and path-halving stores from thousands
// of threads kept rewriting the same slots near the giant component's root.
__device__ __forceinline__ uint32_t cc_find(const uint32_t *parent, uint32_t x)
{
    for (;;) {
        const uint32_t p = cc_load(parent + x);
        if (p == x) return x;
        x = p;
    }
}

__device__ __forceinline__ void cc_unite(uint32_t *parent, uint32_t a, uint32_t b)
{
    uint32_t ra = cc_find(parent, a), rb = cc_find(parent, b);
    while (ra != rb) {
        if (cc_rank(ra) > cc_rank(rb)) {
            const uint32_t t = ra;
            ra = rb;
            rb = t;
        }
        const uint32_t old = atomicCAS(parent + rb, rb, ra);
        if (old == rb) return;
        rb = cc_find(parent, old);
        ra = cc_find(parent, ra);
    }
}

__global__ __launch_bounds__(kBlock) void k_cc_init(uint32_t *__restrict__ parent, int64_t nv)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < nv) parent[v] = (uint32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_cc_union(const int32_t *__restrict__ tris, int64_t nt,
                                                     uint32_t *parent)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const uint32_t a = (uint32_t)tris[3 * t], b = (uint32_t)tris[3 * t + 1],
                   c = (uint32_t)tris[3 * t + 2];
    if (a != b) cc_unite(parent, a, b);
    if (b != c) cc_unite(parent, b, c);
}

// label = root; per-root face counts
__global__ __launch_bounds__(kBlock) void k_cc_label(uint32_t *parent, int64_t nv,
                                                     uint32_t *__restrict__ label)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < nv) label[v] = cc_find(parent, (uint32_t)v);
}

// Most triangles of a mesh lie in one component and atomics on one counter
// serialise, so each thread counts runs of equal labels over kFacesRun
// consecutive triangles, and the wave then adds the counts of each distinct
// final label with one atomic (one ballot and one reduction per label).
constexpr int kFacesRun = 16;

__global__ __launch_bounds__(kBlock) void k_cc_faces(const int32_t *__restrict__ tris, int64_t nt,
                                                     const uint32_t *__restrict__ label,
                                                     uint32_t *__restrict__ faces)
{
    const int64_t t0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kFacesRun;
    uint32_t key = 0, cnt = 0;
    for (int k = 0; k < kFacesRun; ++k) {
        const int64_t t = t0 + k;
        if (t >= nt) break;
        const uint32_t L = label[tris[3 * t]];
        if (cnt && L != key) {
            atomicAdd(&faces[key], cnt);
            cnt = 0;
        }
        key = L;
        ++cnt;
    }
    const bool act = cnt > 0;
    const int lane = (int)__lane_id();
    unsigned long long pending = __ballot(act);
    while (pending) {
        const int first = __ffsll(pending) - 1;
        const uint32_t k0 = __shfl(key, first, 64);
        const bool mine = act && key == k0 && ((pending >> lane) & 1ull);
        uint32_t sum = mine ? cnt : 0u;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (lane == first) atomicAdd(&faces[k0], sum);
        pending &= ~__ballot(mine);
    }
}

__global__ __launch_bounds__(kBlock) void k_cc_keep(const int32_t *__restrict__ tris, int64_t nt,
                                                    const uint32_t *__restrict__ label,
                                                    const uint32_t *__restrict__ faces,
                                                    uint32_t min_faces, uint32_t *__restrict__ keep,
                                                    uint32_t *__restrict__ used)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt) return;
    const int32_t a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    const uint32_t k = faces[label[a]] >= min_faces ? 1u : 0u;
    keep[t] = k;
    if (k) {
        used[a] = 1u;
        used[b] = 1u;
        used[c] = 1u;
    }
}

__global__ __launch_bounds__(kBlock) void k_cc_emit_verts(const float *__restrict__ verts,
                                                          int64_t nv,
                                                          const uint32_t *__restrict__ used,
                                                          const uint32_t *__restrict__ newid,
                                                          float *__restrict__ out)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv || !used[v]) return;
    const int64_t o = newid[v];
    out[3 * o] = verts[3 * v];
    out[3 * o + 1] = verts[3 * v + 1];
    out[3 * o + 2] = verts[3 * v + 2];
}

__global__ __launch_bounds__(kBlock) void k_cc_emit_tris(const int32_t *__restrict__ tris,
                                                         int64_t nt,
                                                         const uint32_t *__restrict__ keep,
                                                         const uint32_t *__restrict__ tpos,
                                                         const uint32_t *__restrict__ newid,
                                                         int32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nt || !keep[t]) return;
    const int64_t o = tpos[t];
    for (int k = 0; k < 3; ++k) out[3 * o + k] = (int32_t)newid[tris[3 * t + k]];
}

}  // namespace

hipError_t tri_lists_launch(const int32_t *tris, int64_t nt, int64_t nv, int32_t *slots,
                            uint32_t *cnt, int32_t *tdeg, int32_t *flags, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * nv, s);
    if (e != hipSuccess) return e;
    if (nt > 0)
        hipLaunchKernelGGL(k_tri_fill, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt,
                           slots, cnt, flags);
    hipLaunchKernelGGL(k_tri_sort, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, slots, cnt, nv,
                       tdeg);
    return hipGetLastError();
}

hipError_t vertex_quadrics_launch(const float *verts, const int32_t *tris, const int32_t *slots,
                                  const int32_t *tdeg, int64_t nv, double *Q, uint8_t *bnd,
                                  int32_t *flags, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vertex_quadrics, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, verts,
                       tris, slots, tdeg, nv, Q, bnd, flags);
    return hipGetLastError();
}

hipError_t points_box_launch(const float *verts, int64_t nv, float *partial, float *out,
                             hipStream_t s)
{
    const unsigned nb = grid_for(nv, kBlock) < (unsigned)kMinmaxBlocks ? grid_for(nv, kBlock)
                                                                      : (unsigned)kMinmaxBlocks;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_points_minmax, dim3(nb), dim3(kBlock), 0, s, verts, nv, partial);
    hipLaunchKernelGGL(k_points_final, dim3(1), dim3(64), 0, s, partial, (int)nb, out);
    return hipGetLastError();
}

hipError_t cell_keys_launch(const float *verts, int64_t nv, const uint8_t *boundary,
                            const double *lo, double c, int64_t n0, int64_t n1, uint32_t *keys,
                            uint32_t *vals, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_keys, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, verts, nv,
                       boundary, lo, c, n0, n1, keys, vals);
    return hipGetLastError();
}

size_t count_kept_ws_bytes() { return sizeof(uint32_t) * kCountBlocks; }

hipError_t count_kept_launch(const int32_t *tris, int64_t nt, const uint32_t *keys,
                             uint32_t *partial, uint32_t *count, hipStream_t s)
{
    const unsigned g = grid_for(nt, kBlock);
    const int nb = (int)(g < (unsigned)kCountBlocks ? (g ? g : 1u) : (unsigned)kCountBlocks);
    hipLaunchKernelGGL(k_count_kept, dim3(nb), dim3(kBlock), 0, s, tris, nt, keys, partial);
    hipLaunchKernelGGL(k_count_final, dim3(1), dim3(kBlock), 0, s, partial, nb, count);
    return hipGetLastError();
}

hipError_t group_flags_launch(const uint32_t *keys, int64_t nv, uint32_t *flag, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, keys, nv,
                       flag);
    return hipGetLastError();
}

hipError_t group_ids_launch(const uint32_t *vals, const uint32_t *flag, const uint32_t *gpos,
                            int64_t nv, uint32_t *gid, uint32_t *gstart, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_group_ids, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, vals, flag,
                       gpos, nv, gid, gstart);
    return hipGetLastError();
}

hipError_t keep_launch(const int32_t *tris, int64_t nt, const uint32_t *gid, uint32_t *keep,
                       uint32_t *used, hipStream_t s)
{
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keep, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt, gid, keep,
                       used);
    return hipGetLastError();
}

hipError_t decimate_emit_launch(const float *verts, const double *Q, const uint8_t *boundary,
                                const uint32_t *vals, const uint32_t *gstart, int64_t ngroups,
                                int64_t nv, const uint32_t *used, const uint32_t *newid,
                                const double *lo, double c, const int32_t *tris, int64_t nt,
                                const uint32_t *gid, const uint32_t *keep, const uint32_t *tpos,
                                float *out_verts, int32_t *out_tris, hipStream_t s)
{
    (void)nv;
    if (ngroups > 0)
        hipLaunchKernelGGL(k_emit_groups, dim3(grid_for(ngroups, kBlock)), dim3(kBlock), 0, s,
                           verts, Q, boundary, vals, gstart, ngroups, used, newid, lo, c,
                           out_verts);
    if (nt > 0)
        hipLaunchKernelGGL(k_emit_tris, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt,
                           gid, keep, tpos, newid, out_tris);
    return hipGetLastError();
}

hipError_t components_launch(const int32_t *tris, int64_t nt, int64_t nv, uint32_t *parent,
                             uint32_t *label, uint32_t *faces, hipStream_t s)
{
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, parent, nv);
    if (nt > 0)
        hipLaunchKernelGGL(k_cc_union, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt,
                           parent);
    hipLaunchKernelGGL(k_cc_label, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, parent, nv,
                       label);
    hipError_t e = hipMemsetAsync(faces, 0, sizeof(uint32_t) * (size_t)nv, s);
    if (e != hipSuccess) return e;
    if (nt > 0)
        hipLaunchKernelGGL(k_cc_faces, dim3(grid_for((nt + kFacesRun - 1) / kFacesRun, kBlock)),
                           dim3(kBlock), 0, s, tris, nt, label, faces);
    return hipGetLastError();
}

hipError_t components_keep_launch(const int32_t *tris, int64_t nt, const uint32_t *label,
                                  const uint32_t *faces, uint32_t min_faces, uint32_t *keep,
                                  uint32_t *used, hipStream_t s)
{
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cc_keep, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris, nt, label,
                       faces, min_faces, keep, used);
    return hipGetLastError();
}

hipError_t components_emit_launch(const float *verts, int64_t nv, const uint32_t *used,
                                  const uint32_t *newid, const int32_t *tris, int64_t nt,
                                  const uint32_t *keep, const uint32_t *tpos, float *out_verts,
                                  int32_t *out_tris, hipStream_t s)
{
    if (nv > 0)
        hipLaunchKernelGGL(k_cc_emit_verts, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, verts,
                           nv, used, newid, out_verts);
    if (nt > 0)
        hipLaunchKernelGGL(k_cc_emit_tris, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tris,
                           nt, keep, tpos, newid, out_tris);
    return hipGetLastError();
}
