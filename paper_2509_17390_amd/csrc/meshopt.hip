// meshopt.hip -- Taubin smoothing of a triangle mesh on gfx950 (FGGS-LiDAR
// Sec. IV-B, "Mesh optimization"; defaults of Sec. V).
//
//   N(i)   distinct vertices sharing an edge with i (never i itself)
//   L(x)_i (sum over N(i) of x_j) / |N(i)| - x_i  (umbrella operator)
//   x <- x + lambda L(x), then x <- x + mu L(x), per iteration; vertices on
//   an edge of a single triangle (the boundary) and vertices without
//   neighbours stay in place.
//
// Neighbour lists: every triangle appends its two other corners to each
// corner's slots (atomic slot counter, at most kNbrCap per vertex); each
// vertex then sorts its slots, keeps distinct entries and marks itself
// fixed when one of them occurred only once (a boundary edge).  Sorting
// makes the lists independent of the append order, and the half-steps sum
// neighbours in ascending index order, one rounded float32 operation at a
// time, so results are deterministic and reproducible on the CPU.
#include "gauss_internal.h"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

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
        for (int j = 1; j < 3; ++j) {
            const int32_t u = c[(k + j) % 3];
            if (u == v) continue;
            const uint32_t at = atomicAdd(&cnt[v], 1u);
            if (at < (uint32_t)kNbrCap) slots[(int64_t)v * kNbrCap + at] = u;
            else atomicOr(flags, 1);
        }
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
    int32_t a[kNbrCap];
    for (int k = 0; k < n; ++k) {           // insertion sort, ascending
        const int32_t x = s[k];
        int j = k;
        while (j > 0 && a[j - 1] > x) {
            a[j] = a[j - 1];
            --j;
        }
        a[j] = x;
    }
    int m = 0;
    bool boundary = false;
    for (int k = 0; k < n;) {
        int e = k + 1;
        while (e < n && a[e] == a[k]) ++e;
        if (e - k == 1) boundary = true;    // the edge lies in one triangle
        s[m++] = a[k];
        k = e;
    }
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
