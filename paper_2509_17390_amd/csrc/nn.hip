// nn.hip -- exact nearest neighbours between point clouds and the fidelity
// metrics of FGGS-LiDAR Sec. V (symmetric Chamfer distance, F-score at a
// distance threshold), gfx950.
//
// The reference cloud gets an LBVH (the shared build kernels over degenerate
// point boxes); one thread per query walks it nearest child first.  Every
// distance is evaluated in FP64 from the float32 coordinates: a box's
// distance is computed with the same rounded operations as the distance to
// any point inside it, and rounding is monotone, so the box bound never
// exceeds a contained point's distance and pruning is exact.  Ties go to the
// lowest reference index.  The sums of the metrics are reduced in a fixed
// order (per-block partials, then one block), so results repeat exactly.
#include "mesh_internal.h"

#include <math.h>

namespace {

constexpr int kBlock = 256;
constexpr int kStack = 64;   // the Karras tree depth is at most 62

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

__global__ __launch_bounds__(kBlock) void k_point_boxes(const float *__restrict__ p, int64_t n,
                                                        float *__restrict__ boxes)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
    float *b = boxes + 6 * i;
    b[0] = x; b[1] = y; b[2] = z;
    b[3] = x; b[4] = y; b[5] = z;
}

// leaf-order points: (x, y, z, reference index)
__global__ __launch_bounds__(kBlock) void k_leaf_points(const float *__restrict__ p,
                                                        const uint32_t *__restrict__ sorted,
                                                        int64_t n, float4 *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t i = sorted[k];
    out[k] = make_float4(p[3 * i], p[3 * i + 1], p[3 * i + 2], __int_as_float((int32_t)i));
}

__device__ __forceinline__ double axis_gap(double q, float lo, float hi)
{
    const double a = (double)lo - q, b = q - (double)hi;
    return a > 0.0 ? a : (b > 0.0 ? b : 0.0);
}

__device__ __forceinline__ double box_d2(double qx, double qy, double qz, float lx, float hx,
                                         float ly, float hy, float lz, float hz)
{
    const double dx = axis_gap(qx, lx, hx), dy = axis_gap(qy, ly, hy), dz = axis_gap(qz, lz, hz);
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ void leaf_test(const float4 *__restrict__ pts, int32_t leaf, double qx,
                                          double qy, double qz, double &best, int32_t &best_i)
{
    const float4 p = pts[leaf];
    const double dx = (double)p.x - qx, dy = (double)p.y - qy, dz = (double)p.z - qz;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const int32_t id = __float_as_int(p.w);
    if (d2 < best || (d2 == best && id < best_i)) {
        best = d2;
        best_i = id;
    }
}

__global__ __launch_bounds__(kBlock) void k_nearest(const NodeRec *__restrict__ nodes,
                                                    const float4 *__restrict__ pts, int64_t n_ref,
                                                    const float *__restrict__ q, int64_t n_q,
                                                    double *__restrict__ out_d,
                                                    int32_t *__restrict__ out_i)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_q) return;
    const double qx = q[3 * t], qy = q[3 * t + 1], qz = q[3 * t + 2];
    double best = INFINITY;
    int32_t best_i = 0x7fffffff;
    if (n_ref == 1) {
        leaf_test(pts, 0, qx, qy, qz, best, best_i);
    } else if (n_ref > 1) {
        int32_t stk[kStack];
        int sp = 0;
        stk[sp++] = 0;
        while (sp > 0) {
            const int32_t node = stk[--sp];
            const NodeRec nr = nodes[node];
            const double dl = box_d2(qx, qy, qz, nr.q0.x, nr.q0.y, nr.q1.x, nr.q1.y, nr.q2.x, nr.q2.y);
            const double dr = box_d2(qx, qy, qz, nr.q0.z, nr.q0.w, nr.q1.z, nr.q1.w, nr.q2.z, nr.q2.w);
            const int32_t cl = nr.q3.x, cr = nr.q3.y;
            // children within the best distance (ties kept: an equally near
            // point with a lower index may lie inside)
            const bool vl = dl <= best, vr = dr <= best;
            if (vl && cl < 0) leaf_test(pts, ~cl, qx, qy, qz, best, best_i);
            if (vr && cr < 0) leaf_test(pts, ~cr, qx, qy, qz, best, best_i);
            const bool il = vl && cl >= 0, ir = vr && cr >= 0;
            if (il && ir) {
                // the nearer child is taken next
                const bool lfirst = dl <= dr;
                if (sp + 2 <= kStack) {
                    stk[sp++] = lfirst ? cr : cl;
                    stk[sp++] = lfirst ? cl : cr;
                }
            } else if (il) {
                if (sp < kStack) stk[sp++] = cl;
            } else if (ir) {
                if (sp < kStack) stk[sp++] = cr;
            }
        }
    }
    // (a node pushed before the best improved has its children tested
    // against the improved best when it is popped)
    out_d[t] = n_ref > 0 ? sqrt(best) : INFINITY;
    out_i[t] = n_ref > 0 ? best_i : -1;
}

// per-block partial sums of d and of [d <= tau], fixed order
__global__ __launch_bounds__(kBlock) void k_metric_partials(const double *__restrict__ d,
                                                            int64_t n, double tau,
                                                            double *__restrict__ sum_out,
                                                            unsigned long long *__restrict__ cnt_out)
{
    __shared__ double ss[kBlock];
    __shared__ unsigned long long sc[kBlock];
    double s = 0.0;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        s += d[i];
        c += d[i] <= tau ? 1ull : 0ull;
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sc[threadIdx.x] += sc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sum_out[blockIdx.x] = ss[0];
        cnt_out[blockIdx.x] = sc[0];
    }
}

__global__ void k_metric_final(const double *__restrict__ sums,
                               const unsigned long long *__restrict__ cnts, int nb,
                               double *__restrict__ out_sum, unsigned long long *__restrict__ out_cnt)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    unsigned long long c = 0;
    for (int b = 0; b < nb; ++b) {
        s += sums[b];
        c += cnts[b];
    }
    *out_sum = s;
    *out_cnt = c;
}

}  // namespace

constexpr int kMetricBlocks = 1024;

size_t nn_scratch_bytes(int64_t n_ref)
{
    const int64_t ni = n_ref > 1 ? n_ref - 1 : 1;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(24 * (size_t)n_ref) + 2 * al(4 * (size_t)n_ref) + al(12 * (size_t)ni) +
           al(sizeof(NodeRec) * (size_t)ni) + al(16 * (size_t)n_ref) + al(64) +
           al(sizeof(double) * kMetricBlocks) + al(8 * kMetricBlocks) + al(16);
}

size_t nn_workspace_bytes(int64_t n_ref) { return lbvh_workspace_bytes(n_ref > 0 ? n_ref : 1); }

hipError_t nearest_launch(const float *ref, int64_t n_ref, const float *query, int64_t n_q,
                          double *out_d, int32_t *out_i, void *scratch, void *ws, size_t ws_bytes,
                          hipStream_t s)
{
    const int64_t ni = n_ref > 1 ? n_ref - 1 : 1;
    char *w = static_cast<char *>(scratch);
    auto take = [&](size_t bytes) {
        char *p = w;
        w += (bytes + 255) & ~(size_t)255;
        return p;
    };
    float *boxes = reinterpret_cast<float *>(take(24 * (size_t)n_ref));
    uint32_t *morton = reinterpret_cast<uint32_t *>(take(4 * (size_t)n_ref));
    uint32_t *sorted = reinterpret_cast<uint32_t *>(take(4 * (size_t)n_ref));
    int32_t *topo = reinterpret_cast<int32_t *>(take(12 * (size_t)ni));
    NodeRec *nodes = reinterpret_cast<NodeRec *>(take(sizeof(NodeRec) * (size_t)ni));
    float4 *pts = reinterpret_cast<float4 *>(take(16 * (size_t)n_ref));
    float *box_dev = reinterpret_cast<float *>(take(64));
    if (n_ref > 0) {
        hipLaunchKernelGGL(k_point_boxes, dim3(grid_for(n_ref, kBlock)), dim3(kBlock), 0, s, ref,
                           n_ref, boxes);
        BuildBuffers b;
        b.verts = nullptr;
        b.tris = nullptr;
        b.nv = 0;
        b.nt = n_ref;
        b.morton_bits = 10;
        b.ws = ws;
        b.ws_bytes = ws_bytes;
        b.morton = morton;
        b.sorted = sorted;
        b.topo = topo;
        b.nodes = nodes;
        b.trirecs = nullptr;
        b.scene_box = box_dev;
        b.depth_out = reinterpret_cast<int32_t *>(box_dev + 6);
        b.q8nodes = nullptr;
        b.q8_count = nullptr;
        hipError_t e = lbvh_build_boxes_launch(b, boxes, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_leaf_points, dim3(grid_for(n_ref, kBlock)), dim3(kBlock), 0, s, ref,
                           sorted, n_ref, pts);
    }
    if (n_q > 0)
        hipLaunchKernelGGL(k_nearest, dim3(grid_for(n_q, kBlock)), dim3(kBlock), 0, s, nodes, pts,
                           n_ref, query, n_q, out_d, out_i);
    return hipGetLastError();
}

hipError_t metric_sums_launch(const double *d, int64_t n, double tau, void *scratch, size_t off,
                              double *out_sum, unsigned long long *out_cnt, hipStream_t s)
{
    char *w = static_cast<char *>(scratch) + off;
    double *sums = reinterpret_cast<double *>(w);
    unsigned long long *cnts =
        reinterpret_cast<unsigned long long *>(w + ((sizeof(double) * kMetricBlocks + 255) & ~(size_t)255));
    const int nb = (int)(grid_for(n, kBlock) < (unsigned)kMetricBlocks ? grid_for(n, kBlock)
                                                                       : (unsigned)kMetricBlocks);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_metric_partials, dim3(nb), dim3(kBlock), 0, s, d, n, tau, sums, cnts);
    hipLaunchKernelGGL(k_metric_final, dim3(1), dim3(64), 0, s, sums, cnts, nb, out_sum, out_cnt);
    return hipGetLastError();
}

size_t nn_metric_offset(int64_t n_ref)
{
    const int64_t ni = n_ref > 1 ? n_ref - 1 : 1;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(24 * (size_t)n_ref) + 2 * al(4 * (size_t)n_ref) + al(12 * (size_t)ni) +
           al(sizeof(NodeRec) * (size_t)ni) + al(16 * (size_t)n_ref) + al(64);
}
