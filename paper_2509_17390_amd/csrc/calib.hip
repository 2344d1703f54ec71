// calib.hip -- calibration kernels for the measured ceilings against which
// the traversal is reported (see include/rcast_calib.h).
//
//  * k_calib_gather: random 64-byte record gathers (four 16-byte loads each,
//    the access the traversal makes for one node record) over a working set
//    of a chosen size, four independent records in flight per lane.  With a
//    working set that fits one XCD's L2 it measures the L2 gather ceiling,
//    with one of the size of a scene's records the cache-hierarchy ceiling
//    the traversal actually meets, and with several GiB the HBM ceiling.
//  * k_calib_valu: independent FP32 vector operations, eight chains per
//    lane, so the vector ALUs never wait on a result.  Mix 0 issues only
//    FMAs; mix 1 the instruction classes of a node test (byte-to-float
//    conversions, FMAs, minimum/maximum, compares and selects).  The vector
//    instruction count comes from the hardware counters of a profiled run;
//    divided by the kernel's time it is the issue ceiling.
#include "rc_internal.h"
#include "rcast_calib.h"

#include "ctx.h"

namespace {

typedef float gvec4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const gvec4 gvec4_g;

__device__ __forceinline__ uint32_t step_lcg(uint32_t x)
{
    return x * 1664525u + 1013904223u;   // Numerical Recipes LCG
}

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void k_calib_gather(const gvec4 *__restrict__ buf,
                                                      uint32_t n_records, int iters,
                                                      uint32_t *__restrict__ sink)
{
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    uint32_t s0 = mix32(gid * 4u + 1u), s1 = mix32(gid * 4u + 2u);
    uint32_t s2 = mix32(gid * 4u + 3u), s3 = mix32(gid * 4u + 4u);
    uint32_t acc = 0;
    const gvec4_g *g = (const gvec4_g *)buf;
    for (int it = 0; it < iters; ++it) {
        s0 = step_lcg(s0); s1 = step_lcg(s1); s2 = step_lcg(s2); s3 = step_lcg(s3);
        const uint64_t r0 = (uint64_t)__umulhi(s0, n_records) * 4u;
        const uint64_t r1 = (uint64_t)__umulhi(s1, n_records) * 4u;
        const uint64_t r2 = (uint64_t)__umulhi(s2, n_records) * 4u;
        const uint64_t r3 = (uint64_t)__umulhi(s3, n_records) * 4u;
        gvec4 a[4], b[4], c[4], d[4];
        for (int k = 0; k < 4; ++k) {
            a[k] = g[r0 + k];
            b[k] = g[r1 + k];
            c[k] = g[r2 + k];
            d[k] = g[r3 + k];
        }
        for (int k = 0; k < 4; ++k) {
            acc ^= __float_as_uint(a[k].x) ^ __float_as_uint(b[k].y) ^ __float_as_uint(c[k].z) ^
                   __float_as_uint(d[k].w) ^ __float_as_uint(a[k].w) ^ __float_as_uint(b[k].x) ^
                   __float_as_uint(c[k].y) ^ __float_as_uint(d[k].z);
        }
    }
    // one store per lane keeps the loads live; nearly never taken
    if (acc == 0x9e3779b9u) sink[gid & 1023u] = acc;
}

template <int MIX>
__global__ __launch_bounds__(256) void k_calib_valu(int iters, float seed, float *__restrict__ sink)
{
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    float x[8];
    for (int k = 0; k < 8; ++k) x[k] = seed + (float)((gid + k) & 255u) * 0.00390625f;
    const float a = 0.99951171875f, b = 0.000244140625f;
    uint32_t w = gid * 0x01010101u;
    for (int it = 0; it < iters; ++it) {
        if (MIX == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // byte to float, a plane distance, an entry/exit bound, a
                // compare and a select -- the shape of one child-plane test
                const float q = (float)((w >> (8 * (k & 3))) & 0xffu);
                const float t = fmaf(q, a, x[k]);
                const float lo = fmaxf(t, b);
                const float hi = fminf(t, 1.0f);
                x[k] = lo <= hi ? lo * a : hi;
            }
            w = w + 0x01030507u;
        }
    }
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == 12345.678f) sink[gid & 1023u] = s;
}

}  // namespace

extern "C" rc_status rc_calib_gather(const void *records, uint64_t n_records, int64_t n_lanes,
                                     int32_t iters, uint32_t *sink, void *stream)
{
    if (!records || !sink || n_records == 0 || n_records > 0xffffffffull || n_lanes <= 0 ||
        n_lanes % 256 != 0 || n_lanes / 256 > 0x7fffffff || iters <= 0)
        return rc::fail(RC_E_INVAL, "rc_calib_gather: bad arguments (records %p, n_records %llu, "
                        "n_lanes %lld, iters %d)", records, (unsigned long long)n_records,
                        (long long)n_lanes, iters);
    if (((uintptr_t)records & 63u) != 0)
        return rc::fail(RC_E_INVAL, "rc_calib_gather: records must be 64-byte aligned");
    hipLaunchKernelGGL(k_calib_gather, dim3((unsigned)(n_lanes / 256)), dim3(256), 0,
                       (hipStream_t)stream, (const gvec4 *)records, (uint32_t)n_records, iters,
                       sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return rc::fail(RC_E_DEVICE, "rc_calib_gather: launch failed: %s", hipGetErrorString(e));
    return RC_OK;
}

extern "C" rc_status rc_calib_valu(int64_t n_lanes, int32_t iters, int32_t mix, float *sink,
                                   void *stream)
{
    if (!sink || n_lanes <= 0 || n_lanes % 256 != 0 || n_lanes / 256 > 0x7fffffff ||
        iters <= 0 || (mix != 0 && mix != 1))
        return rc::fail(RC_E_INVAL, "rc_calib_valu: bad arguments (n_lanes %lld, iters %d, "
                        "mix %d)", (long long)n_lanes, iters, mix);
    const dim3 grid((unsigned)(n_lanes / 256));
    if (mix == 0)
        hipLaunchKernelGGL(k_calib_valu<0>, grid, dim3(256), 0, (hipStream_t)stream, iters,
                           1.0f, sink);
    else
        hipLaunchKernelGGL(k_calib_valu<1>, grid, dim3(256), 0, (hipStream_t)stream, iters,
                           1.0f, sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return rc::fail(RC_E_DEVICE, "rc_calib_valu: launch failed: %s", hipGetErrorString(e));
    return RC_OK;
}
