// gauss.hip -- Gaussian-to-occupancy conversion on gfx950.
//
// FGGS-LiDAR Sec. IV-A ("Grid query and occupancy evaluation") on the
// Gaussian model of Sec. III-A:
//   b_i     box of the k-sigma ellipsoid of G_i: mu +- k sqrt(diag Sigma),
//           Sigma = R S S^T R^T
//   C_tile  the Gaussians whose box meets the box of a tile of 8^3 voxels,
//           found by querying the LBVH built over the b_i (build.hip)
//   D(v)    sum over C_tile of exp(-1/2 (v - mu)^T Sigma^-1 (v - mu)) alpha^2
//   V_occ   D > theta;  Surf = V_occ and not (all six face neighbours occupied)
//
// Kernels:
//   k_gauss_pack      the uploaded arrays interleaved, 48 bytes per Gaussian
//   k_gauss_validate  input checks at upload
//   k_gauss_boxes     b_i: FP64 in one fixed operation order (the library is
//                     built without contraction), each end rounded to the
//                     nearest float32, so that membership in C_tile is an
//                     exact float32 comparison
//   k_gauss_records   64-byte evaluation records in leaf order: mu, the
//                     whitening matrix M = c0 S^-1 R^T and alpha^2 * 2^31
//   k_voxelize        one wave per tile.  Query: breadth-first from the root
//                     until 64 subtrees are pending, then one depth-first
//                     walk per lane; culling-set members go to an LDS ring.
//                     Every 64 members the wave stages their records in LDS
//                     (in the tile's voxel-unit frame) and each lane
//                     evaluates one 8-voxel column of the tile against them.
//   k_surface         6-neighbour test on the occupancy bytes
//
// The density is accumulated in 64-bit fixed point (units of 2^-31 per
// term), so the result does not depend on the order in which the query
// returns culling-set members: it is deterministic and needs no sorting.
// A term with w alpha^2 2^31 < 1/4 rounds to zero, so voxels where the
// exponent exceeds 33 skip the exponential exactly.
#include "gauss_internal.h"

#include <math.h>

namespace {

constexpr int kBlock = 256;
constexpr int kRing = 256;        // LDS ring of culling-set members (<= 191 pending)
constexpr int kFront = 128;       // breadth-first frontier (< 64 nodes, 2 children each)
constexpr int kDfs = 64;          // per-lane stack; the tree depth is at most 62
constexpr float kQSkip = 33.0f;   // exp2(-q) * 2^31 < 1/4 beyond this
constexpr double kC0 = 0.8493218002880191;   // sqrt(log2(e) / 2)
constexpr double kFix = 2147483648.0;        // 2^31: fixed-point unit of one term

// R of q / |q| for q = (w, x, y, z); every step one FP64 operation, in the
// order the Gaussian boxes are defined with.
__device__ __forceinline__ void rotation64(const float4 q4, double R[3][3])
{
    const double w = q4.x, x = q4.y, y = q4.z, z = q4.w;
    const double n = ((w * w + x * x) + y * y) + z * z;
    const double s = 2.0 / n;
    R[0][0] = 1.0 - s * (y * y + z * z);
    R[0][1] = s * (x * y - w * z);
    R[0][2] = s * (x * z + w * y);
    R[1][0] = s * (x * y + w * z);
    R[1][1] = 1.0 - s * (x * x + z * z);
    R[1][2] = s * (y * z - w * x);
    R[2][0] = s * (x * z - w * y);
    R[2][1] = s * (y * z + w * x);
    R[2][2] = 1.0 - s * (x * x + y * y);
}

__global__ __launch_bounds__(kBlock) void k_gauss_pack(GaussArrays a, float4 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    out[3 * i + 0] = make_float4(a.mean[3 * i], a.mean[3 * i + 1], a.mean[3 * i + 2], a.opacity[i]);
    out[3 * i + 1] = make_float4(a.quat[4 * i], a.quat[4 * i + 1], a.quat[4 * i + 2], a.quat[4 * i + 3]);
    out[3 * i + 2] = make_float4(a.scale[3 * i], a.scale[3 * i + 1], a.scale[3 * i + 2], 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_gauss_validate(GaussParams p, int32_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const float4 m = p.g[3 * i], q = p.g[3 * i + 1], s = p.g[3 * i + 2];
    int f = 0;
    const float v[11] = {m.x, m.y, m.z, m.w, q.x, q.y, q.z, q.w, s.x, s.y, s.z};
    for (int k = 0; k < 11; ++k)
        if (!isfinite(v[k])) f |= 1;
    const double qn = (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z + (double)q.w * q.w;
    if (!(qn > 0.0)) f |= 4;
    if (!(s.x > 0.0f) || !(s.y > 0.0f) || !(s.z > 0.0f)) f |= 2;
    if (isfinite(m.w) && (m.w < 0.0f || m.w > 1.0f)) f |= 8;
    if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kBlock) void k_gauss_boxes(GaussParams p, double k,
                                                        float *__restrict__ boxes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const float4 m = p.g[3 * i], sc = p.g[3 * i + 2];
    double R[3][3];
    rotation64(p.g[3 * i + 1], R);
    const double s0 = sc.x, s1 = sc.y, s2 = sc.z;
    const double mu[3] = {m.x, m.y, m.z};
    for (int a = 0; a < 3; ++a) {
        const double c0 = R[a][0] * s0, c1 = R[a][1] * s1, c2 = R[a][2] * s2;
        const double saa = (c0 * c0 + c1 * c1) + c2 * c2;
        const double e = k * sqrt(saa);
        boxes[6 * i + a] = (float)(mu[a] - e);
        boxes[6 * i + 3 + a] = (float)(mu[a] + e);
    }
}

__global__ __launch_bounds__(kBlock) void k_gauss_records(GaussParams p,
                                                          const uint32_t *__restrict__ sorted,
                                                          GaussRec *__restrict__ recs)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n) return;
    const int64_t i = sorted[k];
    const float4 m = p.g[3 * i], sc = p.g[3 * i + 2];
    double R[3][3];
    rotation64(p.g[3 * i + 1], R);
    const double inv[3] = {kC0 / (double)sc.x, kC0 / (double)sc.y, kC0 / (double)sc.z};
    float M[9];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) M[3 * r + j] = (float)(R[j][r] * inv[r]);   // (S^-1 R^T)_rj
    const double al = m.w;
    GaussRec g;
    g.r0 = make_float4(m.x, m.y, m.z, (float)(al * al * kFix));
    g.r1 = make_float4(M[0], M[1], M[2], M[3]);
    g.r2 = make_float4(M[4], M[5], M[6], M[7]);
    g.r3 = make_float4(M[8], __int_as_float((int32_t)i), 0.0f, 0.0f);
    recs[k] = g;
}

__device__ __forceinline__ bool meets(float lx, float hx, float ly, float hy, float lz, float hz,
                                      const float tb[6])
{
    return lx <= tb[3] && hx >= tb[0] && ly <= tb[4] && hy >= tb[1] && lz <= tb[5] &&
           hz >= tb[2];
}

__device__ __forceinline__ uint32_t below(uint64_t m, int lane)
{
    return (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Test both children of internal node `node` against the tile box.
__device__ __forceinline__ void test_children(const NodeRec *__restrict__ nodes, int32_t node,
                                              const float tb[6], int32_t &cl, int32_t &cr,
                                              bool &hl, bool &hr)
{
    const NodeRec nr = nodes[node];
    cl = nr.q3.x;
    cr = nr.q3.y;
    hl = meets(nr.q0.x, nr.q0.y, nr.q1.x, nr.q1.y, nr.q2.x, nr.q2.y, tb);
    hr = meets(nr.q0.z, nr.q0.w, nr.q1.z, nr.q1.w, nr.q2.z, nr.q2.w, tb);
}

// MODE 0: density and occupancy.  MODE 1: |C_tile| per tile only.
template <int MODE>
__global__ __launch_bounds__(64) void k_voxelize(const NodeRec *__restrict__ nodes,
                                                 const GaussRec *__restrict__ recs,
                                                 const float *__restrict__ boxes, int64_t n_gauss,
                                                 VoxGrid g, float *__restrict__ density,
                                                 uint8_t *__restrict__ occ,
                                                 int32_t *__restrict__ counts)
{
    __shared__ int32_t ring[kRing];
    __shared__ int32_t front[kFront];
    __shared__ float4 stage[64 * 4];

    // Workgroups are dealt to the 8 XCDs in turn (workgroup b on XCD b % 8):
    // give each XCD one contiguous run of tiles so that neighbouring tiles,
    // which share most of their culling sets, share an L2.
    const int64_t per = (int64_t)gridDim.x / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= g.n_tiles) return;
    const int lane = threadIdx.x;
    const int ti = (int)(tile % g.tx);
    const int tj = (int)((tile / g.tx) % g.ty);
    const int tk = (int)(tile / ((int64_t)g.tx * g.ty));
    const int i0 = ti * kVoxTile, j0 = tj * kVoxTile, k0 = tk * kVoxTile;
    const int ie = min(i0 + kVoxTile, g.nx), je = min(j0 + kVoxTile, g.ny),
              ke = min(k0 + kVoxTile, g.nz);
    float tb[6];
    tb[0] = (float)(g.o[0] + (double)i0 * g.h);
    tb[1] = (float)(g.o[1] + (double)j0 * g.h);
    tb[2] = (float)(g.o[2] + (double)k0 * g.h);
    tb[3] = (float)(g.o[0] + (double)ie * g.h);
    tb[4] = (float)(g.o[1] + (double)je * g.h);
    tb[5] = (float)(g.o[2] + (double)ke * g.h);

    // evaluation frame: voxel units, origin at the tile's first voxel centre
    const double v0x = g.o[0] + ((double)i0 + 0.5) * g.h;
    const double v0y = g.o[1] + ((double)j0 + 0.5) * g.h;
    const double v0z = g.o[2] + ((double)k0 + 0.5) * g.h;
    const double inv_h = 1.0 / g.h;
    const float hf = (float)g.h;
    const int cy = lane & 7, cz = lane >> 3;   // this lane's column of 8 voxels along x
    const float py = (float)cy, pz = (float)cz;

    uint64_t acc[kVoxTile];
#pragma unroll
    for (int x = 0; x < kVoxTile; ++x) acc[x] = 0;
    uint32_t head = 0, tail = 0;   // ring positions (wave-uniform)
    int64_t total = 0;

    // Evaluate the next m (<= 64) members of the ring against this lane's
    // column and drop them from the ring.
    auto flush = [&](uint32_t m) {
        if (MODE == 1) {
            total += m;
            head += m;
            return;
        }
        if ((uint32_t)lane < m) {
            const GaussRec r = recs[ring[(head + lane) & (kRing - 1)]];
            const float M[9] = {r.r1.x * hf, r.r1.y * hf, r.r1.z * hf, r.r1.w * hf, r.r2.x * hf,
                                r.r2.y * hf, r.r2.z * hf, r.r2.w * hf, r.r3.x * hf};
            const double c0 = ((double)r.r0.x - v0x) * inv_h;
            const double c1 = ((double)r.r0.y - v0y) * inv_h;
            const double c2 = ((double)r.r0.z - v0z) * inv_h;
            float a[3];
            for (int k = 0; k < 3; ++k)
                a[k] = (float)(((double)M[3 * k] * c0 + (double)M[3 * k + 1] * c1) +
                               (double)M[3 * k + 2] * c2);
            stage[4 * lane + 0] = make_float4(M[0], M[1], M[2], a[0]);
            stage[4 * lane + 1] = make_float4(M[3], M[4], M[5], a[1]);
            stage[4 * lane + 2] = make_float4(M[6], M[7], M[8], a[2]);
            stage[4 * lane + 3] = make_float4(r.r0.w, 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
        for (uint32_t r = 0; r < m; ++r) {
            const float4 s0 = stage[4 * r + 0], s1 = stage[4 * r + 1], s2 = stage[4 * r + 2];
            const float A = stage[4 * r + 3].x;
            // u = M (p - c) = M p - a with p = (x, cy, cz) in voxel units
            const float b0 = fmaf(s0.y, py, fmaf(s0.z, pz, -s0.w));
            const float b1 = fmaf(s1.y, py, fmaf(s1.z, pz, -s1.w));
            const float b2 = fmaf(s2.y, py, fmaf(s2.z, pz, -s2.w));
#pragma unroll
            for (int x = 0; x < kVoxTile; ++x) {
                const float u0 = fmaf(s0.x, (float)x, b0);
                const float u1 = fmaf(s1.x, (float)x, b1);
                const float u2 = fmaf(s2.x, (float)x, b2);
                const float q = fmaf(u0, u0, fmaf(u1, u1, u2 * u2));
                if (q <= kQSkip) {
                    const float w = __builtin_amdgcn_exp2f(-q);
                    acc[x] += (uint32_t)fmaf(w, A, 0.5f);
                }
            }
        }
        __syncthreads();
        head += m;
    };

    // Append the leaves among this lane's two children to the ring
    // (ballot compaction; the order within a step is irrelevant).
    auto append = [&](bool ll, int32_t cl, bool lr, int32_t cr) {
        const uint64_t bl = __ballot(ll), br = __ballot(lr);
        if (ll) ring[(tail + below(bl, lane)) & (kRing - 1)] = ~cl;
        if (lr) ring[(tail + (uint32_t)__popcll(bl) + below(br, lane)) & (kRing - 1)] = ~cr;
        tail += (uint32_t)(__popcll(bl) + __popcll(br));
    };

    if (n_gauss == 1) {
        if (meets(boxes[0], boxes[3], boxes[1], boxes[4], boxes[2], boxes[5], tb)) {
            if (lane == 0) ring[0] = 0;
            tail = 1;
        }
        __syncthreads();
    } else if (n_gauss > 1) {
        // breadth-first from the root while fewer than 64 nodes are pending
        int nf = 1;
        if (lane == 0) front[0] = 0;
        __syncthreads();
        while (nf > 0 && nf < 64) {
            const int32_t node = lane < nf ? front[lane] : -1;
            __syncthreads();
            int32_t cl = 0, cr = 0;
            bool hl = false, hr = false;
            if (node >= 0) test_children(nodes, node, tb, cl, cr, hl, hr);
            append(hl && cl < 0, cl, hr && cr < 0, cr);
            const bool il = hl && cl >= 0, ir = hr && cr >= 0;
            const uint64_t bil = __ballot(il), bir = __ballot(ir);
            if (il) front[below(bil, lane)] = cl;
            if (ir) front[(uint32_t)__popcll(bil) + below(bir, lane)] = cr;
            nf = __popcll(bil) + __popcll(bir);
            __syncthreads();
            while (tail - head >= 64) flush(64);
        }
        // then one depth-first walk per lane over its (at most two) subtrees
        int32_t stk[kDfs];
        int sp = 0;
        if (lane < nf) stk[sp++] = front[lane];
        if (lane + 64 < nf) stk[sp++] = front[lane + 64];
        while (__ballot(sp > 0)) {
            int32_t cl = 0, cr = 0;
            bool hl = false, hr = false;
            if (sp > 0) {
                const int32_t node = stk[--sp];
                test_children(nodes, node, tb, cl, cr, hl, hr);
                if (hl && cl >= 0 && sp < kDfs) stk[sp++] = cl;
                if (hr && cr >= 0 && sp < kDfs) stk[sp++] = cr;
            }
            append(hl && cl < 0, cl, hr && cr < 0, cr);
            __syncthreads();
            while (tail - head >= 64) flush(64);
        }
    }
    if (tail > head) flush(tail - head);

    if (MODE == 1) {
        if (lane == 0) counts[tile] = (int32_t)total;
        return;
    }
    const int y = j0 + cy, z = k0 + cz;
    if (y < je && z < ke) {
        const int64_t row = ((int64_t)z * g.ny + y) * g.nx;
#pragma unroll
        for (int x = 0; x < kVoxTile; ++x) {
            if (i0 + x < ie) {
                const float d = (float)((double)acc[x] * (1.0 / kFix));
                if (density) density[row + i0 + x] = d;
                if (occ) occ[row + i0 + x] = d > g.theta ? 1 : 0;
            }
        }
    }
}

__device__ __forceinline__ uint32_t udiv32(uint32_t n, UDiv d)
{
    const uint32_t t = __umulhi(n, d.m);
    return (t + ((n - t) >> (d.sh & 0xffu))) >> (d.sh >> 8);
}

// Four consecutive voxels of a row per thread; rows are (z, y) pairs.
__global__ __launch_bounds__(kBlock) void k_surface(const uint8_t *__restrict__ occ,
                                                    uint8_t *__restrict__ surf, int nx, int ny,
                                                    int nz, uint32_t n_threads, int quads,
                                                    UDiv div_quads, UDiv div_ny)
{
    const uint32_t t = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
    if (t >= n_threads) return;
    const uint32_t row = udiv32(t, div_quads);
    const int x0 = 4 * (int)(t - row * (uint32_t)quads);
    const uint32_t zz = udiv32(row, div_ny);
    const int y = (int)(row - zz * (uint32_t)ny), z = (int)zz;
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t base = (int64_t)row * nx;
    const bool ym = y > 0, yp = y < ny - 1, zm = z > 0, zp = z < nz - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = x0 + k;
        if (x >= nx) break;
        const int64_t i = base + x;
        uint8_t s = 0;
        if (occ[i]) {
            const bool interior = x > 0 && x < nx - 1 && ym && yp && zm && zp && occ[i - 1] &&
                                  occ[i + 1] && occ[i - nx] && occ[i + nx] && occ[i - sxy] &&
                                  occ[i + sxy];
            s = interior ? 0 : 1;
        }
        surf[i] = s;
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t gauss_pack_launch(const GaussArrays &a, float4 *out, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_pack, dim3(grid_for(a.n, kBlock)), dim3(kBlock), 0, s, a, out);
    return hipGetLastError();
}

hipError_t gauss_validate_launch(const GaussParams &p, int32_t *flags, hipStream_t s)
{
    if (p.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_validate, dim3(grid_for(p.n, kBlock)), dim3(kBlock), 0, s, p,
                       flags);
    return hipGetLastError();
}

hipError_t gauss_boxes_launch(const GaussParams &p, float k, float *boxes, hipStream_t s)
{
    if (p.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_boxes, dim3(grid_for(p.n, kBlock)), dim3(kBlock), 0, s, p,
                       (double)k, boxes);
    return hipGetLastError();
}

hipError_t gauss_records_launch(const GaussParams &p, const uint32_t *sorted, GaussRec *recs,
                                hipStream_t s)
{
    if (p.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_records, dim3(grid_for(p.n, kBlock)), dim3(kBlock), 0, s, p,
                       sorted, recs);
    return hipGetLastError();
}

hipError_t voxelize_launch(int mode, const NodeRec *nodes, const GaussRec *recs,
                           const float *boxes, int64_t n_gauss, const VoxGrid &g,
                           float *density, uint8_t *occ, int32_t *tile_counts, hipStream_t s)
{
    if (g.n_tiles <= 0) return hipSuccess;
    const int64_t blocks = (g.n_tiles + 7) / 8 * 8;   // a multiple of the XCD count
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (mode == 0)
        hipLaunchKernelGGL(k_voxelize<0>, dim3((unsigned)blocks), dim3(64), 0, s, nodes, recs,
                           boxes, n_gauss, g, density, occ, tile_counts);
    else
        hipLaunchKernelGGL(k_voxelize<1>, dim3((unsigned)blocks), dim3(64), 0, s, nodes, recs,
                           boxes, n_gauss, g, density, occ, tile_counts);
    return hipGetLastError();
}

hipError_t surface_launch(const uint8_t *occ, uint8_t *surf, const VoxGrid &g, hipStream_t s)
{
    const int quads = (g.nx + 3) / 4;
    const int64_t rows = (int64_t)g.ny * g.nz;
    const int64_t threads = (int64_t)quads * rows;
    if (threads <= 0) return hipSuccess;
    if (threads > 0xffffff00LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_surface, dim3(grid_for(threads, kBlock)), dim3(kBlock), 0, s, occ, surf,
                       g.nx, g.ny, g.nz, (uint32_t)threads, quads, udiv_magic((uint32_t)quads),
                       udiv_magic((uint32_t)g.ny));
    return hipGetLastError();
}
