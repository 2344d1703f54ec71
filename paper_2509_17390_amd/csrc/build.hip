// build.hip -- GPU linear BVH over primitive boxes (gfx950): triangle boxes
// for ray casting, or ready-made Gaussian boxes.
//
// FGGS-LiDAR Sec. IV-A "LBVH construction" (reused for triangles in
// Sec. IV-C): every primitive centre is quantised inside the scene box,
//   u_i = floor(2^b (c_i - o) / L),  m_i = Morton(u_i),
// the primitives are radix-sorted by m_i, the hierarchy follows from the
// longest common prefix of the sorted codes (Karras 2012: ties between equal
// codes are broken by the index, so every internal node splits on a distinct
// bit of the 3b + 32 bit augmented key), and node boxes are reduced bottom-up.
//
// Stages, one kernel each (radix sort: three per 8-bit digit):
//   tri_bounds   triangle boxes + per-block partial scene boxes, folded by
//                one more block (or: union of ready-made primitive boxes)
//   morton       centre of the triangle box -> 3b-bit code
//   radix sort   per-tile digit histogram / per-digit scan of tile counts /
//                stable scatter ranked in LDS with wave64 ballots
//   karras       children and parent of every internal node
//   refit        bottom-up: each leaf walks up; the second arrival at a node
//                merges both child boxes into the parent's record (LDS
//                counters inside a block's leaf chunk, agent-scope counters
//                across chunks); node heights give the tree depth
//   tri_records  triangles reordered into leaf order (48-byte records; not
//                for ready-made boxes)
//   collapse     optional: 4-wide nodes with 8-bit child boxes in each node's
//                frame (node depths, prefix count of even-depth nodes, then
//                one thread per 4-wide node)
#include "mesh_internal.h"

#include <math.h>

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

constexpr int kBoundBlocks = 512;   // blocks of the box reductions

// Block-wide min/max of acc[0..2] / acc[3..5]; thread 0 writes out[6].
__device__ __forceinline__ void block_box(float acc[6], float *out)
{
    __shared__ float red[kBlock / 64][6];
    for (int a = 0; a < 3; ++a) {
        acc[a] = wave_min(acc[a]);
        acc[3 + a] = wave_max(acc[3 + a]);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 6; ++a) red[w][a] = acc[a];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        float v = red[0][a];
        for (int ww = 1; ww < kBlock / 64; ++ww) v = a < 3 ? fminf(v, red[ww][a]) : fmaxf(v, red[ww][a]);
        out[a] = v;
    }
}

// Triangle boxes (AoS lo.xyz hi.xyz) and one partial scene box per block
// (grid-stride loop; the partials are folded by k_bounds_final, so no
// atomics: min/max are exact in any order).
__global__ __launch_bounds__(kBlock) void k_tri_bounds(const float *__restrict__ verts,
                                                       const int32_t *__restrict__ tris,
                                                       int64_t nt, float *__restrict__ bounds,
                                                       float *__restrict__ partial)
{
    float acc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt;
         i += (int64_t)gridDim.x * blockDim.x) {
        float lo[3] = {INFINITY, INFINITY, INFINITY};
        float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < 3; ++k) {
            const float *v = verts + 3 * (int64_t)tris[3 * i + k];
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], v[a]);
                hi[a] = fmaxf(hi[a], v[a]);
            }
        }
        float *b = bounds + 6 * i;
        b[0] = lo[0]; b[1] = lo[1]; b[2] = lo[2];
        b[3] = hi[0]; b[4] = hi[1]; b[5] = hi[2];
        for (int a = 0; a < 3; ++a) {
            acc[a] = fminf(acc[a], lo[a]);
            acc[3 + a] = fmaxf(acc[3 + a], hi[a]);
        }
    }
    block_box(acc, partial + 6 * blockIdx.x);
}

// Partial unions of ready-made primitive boxes.
__global__ __launch_bounds__(kBlock) void k_box_union(const float *__restrict__ bounds, int64_t n,
                                                      float *__restrict__ partial)
{
    float acc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float *b = bounds + 6 * i;
        for (int a = 0; a < 3; ++a) {
            acc[a] = fminf(acc[a], b[a]);
            acc[3 + a] = fmaxf(acc[3 + a], b[3 + a]);
        }
    }
    block_box(acc, partial + 6 * blockIdx.x);
}

// One block: the scene box from the per-block partials.
__global__ __launch_bounds__(kBlock) void k_bounds_final(const float *__restrict__ partial,
                                                         int nparts, float *__restrict__ box)
{
    float acc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int p = threadIdx.x; p < nparts; p += kBlock)
        for (int a = 0; a < 3; ++a) {
            acc[a] = fminf(acc[a], partial[6 * p + a]);
            acc[3 + a] = fmaxf(acc[3 + a], partial[6 * p + 3 + a]);
        }
    block_box(acc, box);
}

__device__ __forceinline__ uint32_t expand_bits(uint32_t v)
{
    // spread the low 10 bits of v so that bit k moves to bit 3k
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Morton code of each triangle-box centre; x takes the most significant
// position of every 3-bit group
__global__ __launch_bounds__(kBlock) void k_morton(const float *__restrict__ bounds,
                                                   const float *__restrict__ scene_box,
                                                   int64_t nt, int bits,
                                                   uint32_t *__restrict__ morton,
                                                   uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const float *b = bounds + 6 * i;
    const float cells = (float)(1u << bits);
    uint32_t u[3];
    for (int a = 0; a < 3; ++a) {
        float o = scene_box[a];
        float L = scene_box[3 + a] - o;
        float scale = L > 0.0f ? cells / L : 0.0f;
        float c = (b[a] + b[3 + a]) * 0.5f;
        float q = floorf((c - o) * scale);
        q = fminf(fmaxf(q, 0.0f), cells - 1.0f);
        u[a] = (uint32_t)q;
    }
    uint32_t m = (expand_bits(u[0]) << 2) | (expand_bits(u[1]) << 1) | expand_bits(u[2]);
    morton[i] = m;
    keys[i] = m;
    vals[i] = (uint32_t)i;
}

// ---- radix sort ------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                 int shift, uint32_t *__restrict__ hist,
                                                 int nblocks)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// block-wide exclusive scan of one value per thread (kBlock threads);
// returns the exclusive prefix, *total receives the block sum
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int ww = 0; ww < kBlock / 64; ++ww) {
        if (ww < w) off += wsum[ww];
        tot += wsum[ww];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// one block per digit: exclusive scan of that digit's per-tile counts
// (in place) and the digit's total
__global__ __launch_bounds__(kBlock) void k_scan_digits(uint32_t *__restrict__ hist, int nblocks,
                                                        uint32_t *__restrict__ digit_tot)
{
    uint32_t *h = hist + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int base = 0; base < nblocks; base += kBlock) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nblocks ? h[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nblocks) h[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// stable scatter: tile order is (round, thread); ranks come from ballots
__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t *__restrict__ keys_in,
                                                    const uint32_t *__restrict__ vals_in,
                                                    uint32_t *__restrict__ keys_out,
                                                    uint32_t *__restrict__ vals_out, int64_t n,
                                                    int shift, const uint32_t *__restrict__ offs,
                                                    const uint32_t *__restrict__ digit_tot,
                                                    int nblocks)
{
    __shared__ uint32_t base_of[kRadix];
    __shared__ uint32_t running[kRadix];
    __shared__ uint32_t wcount[kBlock / 64][kRadix];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    {
        uint32_t tot;
        const uint32_t digit_base = block_exclusive_scan(digit_tot[tid], &tot);
        base_of[tid] = digit_base + offs[(int64_t)tid * nblocks + blockIdx.x];
    }
    running[tid] = 0;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        for (int j = tid; j < (kBlock / 64) * kRadix; j += kBlock) (&wcount[0][0])[j] = 0;
        __syncthreads();
        int64_t i = base + r * kBlock + tid;
        bool valid = i < n;
        uint32_t key = valid ? keys_in[i] : 0u;
        uint32_t val = valid ? vals_in[i] : 0u;
        uint32_t d = (key >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < kRadixBits; ++bit) {
            bool set = (d >> bit) & 1u;
            uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcount[w][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t run = running[tid];
            for (int ww = 0; ww < kBlock / 64; ++ww) {
                uint32_t c = wcount[ww][tid];
                wcount[ww][tid] = run;
                run += c;
            }
            running[tid] = run;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = base_of[d] + wcount[w][d] + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
    }
}

// ---- hierarchy -------------------------------------------------------------
__device__ __forceinline__ int delta(const uint32_t *keys, int64_t n, int64_t i, int64_t j)
{
    if (j < 0 || j >= n) return -1;
    uint32_t a = keys[i], b = keys[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

// Internal node i of the radix tree over sorted keys (Karras 2012, Sec. 4):
// the direction of its range, the range end, then the split position.
__global__ __launch_bounds__(kBlock) void k_karras(const uint32_t *__restrict__ keys, int64_t n,
                                                   int32_t *__restrict__ topo,
                                                   int32_t *__restrict__ leaf_parent,
                                                   int2 *__restrict__ range,
                                                   NodeRec *__restrict__ nodes)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t left = (lo == gamma) ? ~(int32_t)gamma : (int32_t)gamma;
    int32_t right = (hi == gamma + 1) ? ~(int32_t)(gamma + 1) : (int32_t)(gamma + 1);
    topo[3 * i + 0] = left;
    topo[3 * i + 1] = right;
    if (left >= 0) topo[3 * left + 2] = (int32_t)i; else leaf_parent[~left] = (int32_t)i;
    if (right >= 0) topo[3 * right + 2] = (int32_t)i; else leaf_parent[~right] = (int32_t)i;
    if (i == 0) topo[2] = -1;
    range[i] = make_int2((int32_t)lo, (int32_t)hi);
    nodes[i].q3 = make_int4(left, right, 0, 0);
}

__device__ __forceinline__ void store_child_box(NodeRec *node, int slot, const float lo[3],
                                                const float hi[3])
{
    float2 *q = reinterpret_cast<float2 *>(node);
    // q0..q2 hold (L.lo, L.hi, R.lo, R.hi) per axis: float2 index 2*axis + slot
    q[0 + slot] = make_float2(lo[0], hi[0]);
    q[2 + slot] = make_float2(lo[1], hi[1]);
    q[4 + slot] = make_float2(lo[2], hi[2]);
}

// Bottom-up box reduction in two kernels.
//
// k_refit: a thread walks up from kRefitLeavesPerThread leaves in turn.
// A block owns a chunk of kRefitChunk consecutive leaves; a node whose leaf
// range lies inside the chunk has both children finished by this block, so its arrival counter lives in LDS and
// workgroup-scope ordering suffices.  A thread whose walk reaches a node
// spanning chunks writes its child box there and leaves the node on a list.
//
// k_refit_top: one block finishes the spanning nodes (a few per chunk
// boundary and level) with arrival counters in global memory.  The kernel
// boundary publishes the first kernel's records, and inside one block
// workgroup-scope ordering suffices again, so no step needs the agent-scope
// release/acquire that would write back and invalidate whole L2 caches
// (one per XCD) on every arrival.
constexpr int kRefitBlock = 1024;
constexpr int kRefitLeavesPerThread = 4;   // larger chunks: fewer spanning nodes
constexpr int kRefitChunk = kRefitBlock * kRefitLeavesPerThread;   // leaves per block

__global__ __launch_bounds__(kRefitBlock) void k_refit(const float *__restrict__ bounds,
                                                       const uint32_t *__restrict__ sorted,
                                                       int64_t n, const int32_t *__restrict__ topo,
                                                       const int32_t *__restrict__ leaf_parent,
                                                       const int2 *__restrict__ range,
                                                       int32_t *__restrict__ height,
                                                       NodeRec *nodes, int32_t *depth_out,
                                                       int32_t *__restrict__ pend,
                                                       uint32_t *__restrict__ pend_count)
{
    __shared__ uint32_t local_arrive[kRefitChunk];
    for (int i = threadIdx.x; i < kRefitChunk; i += kRefitBlock) local_arrive[i] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kRefitChunk;
    const int64_t c1 = c0 + kRefitChunk < n ? c0 + kRefitChunk : n;
    for (int64_t k = c0 + threadIdx.x; k < c1; k += kRefitBlock) {
        const float *b = bounds + 6 * (int64_t)sorted[k];
        float lo[3] = {b[0], b[1], b[2]};
        float hi[3] = {b[3], b[4], b[5]};
        int32_t child = ~(int32_t)k;
        int32_t h = 0;
        int32_t p = leaf_parent[k];
        bool root = true;
        while (p >= 0) {
            int slot = (topo[3 * p + 0] == child) ? 0 : 1;
            store_child_box(nodes + p, slot, lo, hi);
            if (slot == 0) height[2 * p + 0] = h; else height[2 * p + 1] = h;
            const int2 rg = range[p];
            if (rg.x < c0 || rg.y >= c0 + kRefitChunk) {
                // spans chunks: finished by k_refit_top (a unique list slot is
                // all this counter provides, so no ordering is asked of it)
                const uint32_t at = __hip_atomic_fetch_add(pend_count, 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                pend[at] = p;
                root = false;
                break;
            }
            const uint32_t prev = __hip_atomic_fetch_add(local_arrive + (p - c0), 1u,
                                                         __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == 0) {   // first arrival: the sibling finishes the node
                root = false;
                break;
            }
            const NodeRec nr = nodes[p];
            lo[0] = fminf(nr.q0.x, nr.q0.z); hi[0] = fmaxf(nr.q0.y, nr.q0.w);
            lo[1] = fminf(nr.q1.x, nr.q1.z); hi[1] = fmaxf(nr.q1.y, nr.q1.w);
            lo[2] = fminf(nr.q2.x, nr.q2.z); hi[2] = fmaxf(nr.q2.y, nr.q2.w);
            int32_t h0 = height[2 * p + 0], h1 = height[2 * p + 1];
            h = 1 + (h0 > h1 ? h0 : h1);
            child = p;
            p = topo[3 * p + 2];
        }
        if (root) depth_out[0] = h;   // the root lies inside this chunk (n <= kRefitChunk)
    }
}

__global__ __launch_bounds__(kRefitBlock) void k_refit_top(const int32_t *__restrict__ topo,
                                                           uint32_t *__restrict__ arrive,
                                                           int32_t *__restrict__ height,
                                                           NodeRec *nodes, int32_t *depth_out,
                                                           const int32_t *__restrict__ pend,
                                                           const uint32_t *__restrict__ pend_count)
{
    const uint32_t cnt = *pend_count;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        int32_t p = pend[i];
        while (true) {
            const uint32_t prev = __hip_atomic_fetch_add(arrive + p, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == 0) break;   // first arrival: the sibling finishes the node
            const NodeRec nr = nodes[p];
            float lo[3], hi[3];
            lo[0] = fminf(nr.q0.x, nr.q0.z); hi[0] = fmaxf(nr.q0.y, nr.q0.w);
            lo[1] = fminf(nr.q1.x, nr.q1.z); hi[1] = fmaxf(nr.q1.y, nr.q1.w);
            lo[2] = fminf(nr.q2.x, nr.q2.z); hi[2] = fmaxf(nr.q2.y, nr.q2.w);
            const int32_t h0 = height[2 * p + 0], h1 = height[2 * p + 1];
            const int32_t h = 1 + (h0 > h1 ? h0 : h1);
            const int32_t pp = topo[3 * p + 2];
            if (pp < 0) {
                depth_out[0] = h;   // the root
                break;
            }
            const int slot = (topo[3 * pp + 0] == p) ? 0 : 1;
            store_child_box(nodes + pp, slot, lo, hi);
            height[2 * pp + slot] = h;
            p = pp;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_tri_records(const float *__restrict__ verts,
                                                        const int32_t *__restrict__ tris,
                                                        const uint32_t *__restrict__ sorted,
                                                        int64_t n, TriRec *__restrict__ out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t t = sorted[k];
    const float *a = verts + 3 * (int64_t)tris[3 * (int64_t)t + 0];
    const float *b = verts + 3 * (int64_t)tris[3 * (int64_t)t + 1];
    const float *c = verts + 3 * (int64_t)tris[3 * (int64_t)t + 2];
    TriRec r;
    r.a = make_float4(a[0], a[1], a[2], b[0]);
    r.b = make_float4(b[1], b[2], c[0], c[1]);
    r.c = make_float4(c[2], __int_as_float((int32_t)t), 0.0f, 0.0f);
    out[k] = r;
}

// ---- quantised 4-wide nodes ------------------------------------------------
// Depth of every internal node (edges from the root), by walking up.
__global__ __launch_bounds__(kBlock) void k_node_depth(const int32_t *__restrict__ topo,
                                                       int64_t ni, int32_t *__restrict__ depth)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    int32_t d = 0;
    for (int32_t p = topo[3 * i + 2]; p >= 0 && d <= 64; p = topo[3 * p + 2]) ++d;
    depth[i] = d;
}

// Nodes at even depth become 4-wide nodes; their compact index is the
// exclusive prefix count of even-depth nodes (three-kernel scan).
__global__ __launch_bounds__(kBlock) void k_even_local(const int32_t *__restrict__ depth,
                                                       int64_t ni, uint32_t *__restrict__ qidx,
                                                       uint32_t *__restrict__ bsum)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = (i < ni && (depth[i] & 1) == 0) ? 1u : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, &tot);
    if (i < ni) qidx[i] = ex;
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t *__restrict__ bsum, int nb,
                                                      uint32_t *__restrict__ total)
{
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) total[0] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *__restrict__ qidx, int64_t ni,
                                                     const uint32_t *__restrict__ bsum)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ni) qidx[i] += bsum[blockIdx.x];
}

__device__ __forceinline__ void slot_box(const NodeRec &nd, int slot, float lo[3], float hi[3])
{
    if (slot == 0) {
        lo[0] = nd.q0.x; hi[0] = nd.q0.y; lo[1] = nd.q1.x; hi[1] = nd.q1.y;
        lo[2] = nd.q2.x; hi[2] = nd.q2.y;
    } else {
        lo[0] = nd.q0.z; hi[0] = nd.q0.w; lo[1] = nd.q1.z; hi[1] = nd.q1.w;
        lo[2] = nd.q2.z; hi[2] = nd.q2.w;
    }
}

// One 4-wide node per even-depth binary node: its children are the binary
// node's children, with every internal (odd-depth) child replaced by that
// child's own two children.  Boxes are quantised to 8 bits in the node's
// frame: scale_a = smallest power of two with 255 * scale_a >= extent_a,
// qlo = floor((lo - origin) / scale), qhi = ceil((hi - origin) / scale),
// computed in FP64 (exact here), so every decoded box contains its child.
__global__ __launch_bounds__(kBlock) void k_collapse4(const NodeRec *__restrict__ nodes,
                                                      const int32_t *__restrict__ depth,
                                                      const uint32_t *__restrict__ qidx,
                                                      int64_t ni, NodeRec *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || (depth[i] & 1)) return;
    int32_t ref[4] = {kEmptyChild, kEmptyChild, kEmptyChild, kEmptyChild};
    float clo[4][3], chi[4][3];
    int m = 0;
    const NodeRec nd = nodes[i];
    for (int s = 0; s < 2; ++s) {
        const int32_t c = s == 0 ? nd.q3.x : nd.q3.y;
        if (c < 0) {
            slot_box(nd, s, clo[m], chi[m]);
            ref[m++] = c;
        } else {
            const NodeRec cd = nodes[c];
            for (int s2 = 0; s2 < 2; ++s2) {
                const int32_t g = s2 == 0 ? cd.q3.x : cd.q3.y;
                slot_box(cd, s2, clo[m], chi[m]);
                ref[m++] = g < 0 ? g : (int32_t)qidx[g];
            }
        }
    }
    float olo[3], ohi[3];
    for (int a = 0; a < 3; ++a) {
        olo[a] = clo[0][a];
        ohi[a] = chi[0][a];
        for (int k = 1; k < m; ++k) {
            olo[a] = fminf(olo[a], clo[k][a]);
            ohi[a] = fmaxf(ohi[a], chi[k][a]);
        }
    }
    float scale[3];
    uint32_t qlo[3] = {0u, 0u, 0u}, qhi[3] = {0u, 0u, 0u};
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)ohi[a] - (double)olo[a];
        double sc = 0.0;
        if (ext > 0.0) {
            int e = (int)ceil(log2(ext / 255.0));
            if (e < -100) e = -100;
            sc = ldexp(1.0, e);
            while (255.0 * sc < ext) sc *= 2.0;
        }
        scale[a] = (float)sc;
        for (int k = 0; k < m; ++k) {
            double lo = 0.0, hi = 0.0;
            if (sc > 0.0) {
                lo = floor(((double)clo[k][a] - (double)olo[a]) / sc);
                hi = ceil(((double)chi[k][a] - (double)olo[a]) / sc);
            }
            lo = fmin(fmax(lo, 0.0), 255.0);
            hi = fmin(fmax(hi, 0.0), 255.0);
            qlo[a] |= (uint32_t)lo << (8 * k);
            qhi[a] |= (uint32_t)hi << (8 * k);
        }
    }
    NodeRec r;
    r.q0 = make_float4(olo[0], olo[1], olo[2], scale[0]);
    r.q1 = make_float4(scale[1], scale[2], __uint_as_float(qlo[0]), __uint_as_float(qhi[0]));
    r.q2 = make_float4(__uint_as_float(qlo[1]), __uint_as_float(qhi[1]), __uint_as_float(qlo[2]),
                       __uint_as_float(qhi[2]));
    r.q3 = make_int4(ref[0], ref[1], ref[2], ref[3]);
    out[qidx[i]] = r;
}

__global__ void k_single_tri_depth(int32_t *depth_out) { depth_out[0] = 0; }

__global__ __launch_bounds__(kBlock) void k_validate(const float *__restrict__ verts, int64_t nv,
                                                     const int32_t *__restrict__ tris, int64_t nt,
                                                     int32_t *flags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (i < nt) {
        for (int k = 0; k < 3; ++k) {
            int32_t v = tris[3 * i + k];
            if (v < 0 || v >= nv) f |= 1;
        }
    }
    if (i < nv) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(verts[3 * i + a])) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t lbvh_workspace_bytes(int64_t nt)
{
    int64_t nblocks = (nt + kTile - 1) / kTile;
    if (nblocks < 1) nblocks = 1;
    size_t s = 0;
    s += align_up(sizeof(float) * 6 * (size_t)nt);       // bounds
    s += 4 * align_up(sizeof(uint32_t) * (size_t)nt);     // keys/vals ping-pong
    s += align_up(sizeof(uint32_t) * kRadix * (size_t)nblocks);  // histograms
    s += align_up(sizeof(int32_t) * (size_t)nt);          // leaf parents
    s += align_up(sizeof(uint32_t) * (size_t)nt);         // arrival counters
    s += align_up(sizeof(int32_t) * 2 * (size_t)nt);      // child heights
    s += align_up(sizeof(int32_t) * 2 * (size_t)nt);      // node leaf ranges
    s += align_up(sizeof(uint32_t) * kRadix);             // digit totals
    s += align_up(sizeof(int32_t) * (size_t)nt);          // node depths
    s += align_up(sizeof(uint32_t) * (size_t)nt);         // 4-wide node index
    s += align_up(sizeof(uint32_t) * ((size_t)nt / kBlock + 2));  // scan block sums
    s += align_up(sizeof(float) * 6 * kBoundBlocks);      // partial scene boxes
    s += align_up(sizeof(int32_t) * (size_t)nt);          // spanning nodes left to refit
    s += align_up(sizeof(uint32_t) * 1);                  // their count
    return s;
}

hipError_t validate_mesh_launch(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                                int32_t *flags, hipStream_t s)
{
    int64_t n = nv > nt ? nv : nt;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, verts, nv, tris,
                       nt, flags);
    return hipGetLastError();
}

namespace {

hipError_t lbvh_build_any(const BuildBuffers &b, const float *prim_boxes, hipStream_t s)
{
    const int64_t n = b.nt;
    if (n <= 0) return hipSuccess;
    const int64_t nblocks = (n + kTile - 1) / kTile;
    char *w = static_cast<char *>(b.ws);
    auto take = [&](size_t bytes) {
        char *p = w;
        w += align_up(bytes);
        return p;
    };
    float *bounds = reinterpret_cast<float *>(take(sizeof(float) * 6 * n));
    uint32_t *keys0 = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    uint32_t *keys1 = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    uint32_t *vals0 = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    uint32_t *vals1 = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    uint32_t *hist = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * kRadix * nblocks));
    int32_t *leaf_parent = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * n));
    uint32_t *arrive = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    int32_t *height = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 2 * n));
    int2 *range = reinterpret_cast<int2 *>(take(sizeof(int32_t) * 2 * n));
    uint32_t *digit_tot = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * kRadix));
    int32_t *ndepth = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * n));
    uint32_t *qidx = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
    uint32_t *bsum = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * (n / kBlock + 2)));
    float *partial = reinterpret_cast<float *>(take(sizeof(float) * 6 * kBoundBlocks));
    int32_t *pend = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * n));
    uint32_t *pend_count = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t)));
    if ((size_t)(w - static_cast<char *>(b.ws)) > b.ws_bytes) return hipErrorInvalidValue;

    const unsigned bgrid = grid_for(n, kBlock) < (unsigned)kBoundBlocks ? grid_for(n, kBlock)
                                                                         : (unsigned)kBoundBlocks;
    if (prim_boxes) {
        bounds = const_cast<float *>(prim_boxes);
        hipLaunchKernelGGL(k_box_union, dim3(bgrid), dim3(kBlock), 0, s, prim_boxes, n, partial);
    } else {
        hipLaunchKernelGGL(k_tri_bounds, dim3(bgrid), dim3(kBlock), 0, s, b.verts, b.tris, n,
                           bounds, partial);
    }
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBlock), 0, s, partial, (int)bgrid,
                       b.scene_box);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, bounds,
                       b.scene_box, n, b.morton_bits, b.morton, keys0, vals0);
    const int key_bits = 3 * b.morton_bits;
    uint32_t *kin = keys0, *kout = keys1, *vin = vals0, *vout = vals1;
    for (int shift = 0; shift < key_bits; shift += kRadixBits) {
        hipLaunchKernelGGL(k_hist, dim3((unsigned)nblocks), dim3(kBlock), 0, s, kin, n, shift,
                           hist, (int)nblocks);
        hipLaunchKernelGGL(k_scan_digits, dim3(kRadix), dim3(kBlock), 0, s, hist, (int)nblocks,
                           digit_tot);
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)nblocks), dim3(kBlock), 0, s, kin, vin,
                           kout, vout, n, shift, hist, digit_tot, (int)nblocks);
        uint32_t *t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    hipError_t e = hipMemcpyAsync(b.sorted, vin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (b.trirecs)
        hipLaunchKernelGGL(k_tri_records, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, b.verts,
                           b.tris, b.sorted, n, b.trirecs);
    if (n == 1) {
        hipLaunchKernelGGL(k_single_tri_depth, dim3(1), dim3(1), 0, s, b.depth_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_karras, dim3(grid_for(n - 1, kBlock)), dim3(kBlock), 0, s, kin, n,
                       b.topo, leaf_parent, range, b.nodes);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, arrive, n, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, pend_count, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_refit, dim3(grid_for(n, kRefitChunk)), dim3(kRefitBlock), 0, s, bounds,
                       b.sorted, n, b.topo, leaf_parent, range, height, b.nodes, b.depth_out,
                       pend, pend_count);
    hipLaunchKernelGGL(k_refit_top, dim3(1), dim3(kRefitBlock), 0, s, b.topo, arrive, height,
                       b.nodes, b.depth_out, pend, pend_count);
    if (b.q8nodes) {
        const int64_t ni = n - 1;
        const unsigned g = grid_for(ni, kBlock);
        hipLaunchKernelGGL(k_node_depth, dim3(g), dim3(kBlock), 0, s, b.topo, ni, ndepth);
        hipLaunchKernelGGL(k_even_local, dim3(g), dim3(kBlock), 0, s, ndepth, ni, qidx, bsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, bsum, (int)g, b.q8_count);
        hipLaunchKernelGGL(k_scan_add, dim3(g), dim3(kBlock), 0, s, qidx, ni, bsum);
        hipLaunchKernelGGL(k_collapse4, dim3(g), dim3(kBlock), 0, s, b.nodes, ndepth, qidx, ni,
                           b.q8nodes);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t lbvh_build_launch(const BuildBuffers &b, hipStream_t s)
{
    return lbvh_build_any(b, nullptr, s);
}

hipError_t lbvh_build_boxes_launch(const BuildBuffers &b, const float *boxes, hipStream_t s)
{
    if (b.trirecs) return hipErrorInvalidValue;
    return lbvh_build_any(b, boxes, s);
}

size_t radix_sort_ws_bytes(int64_t n)
{
    const int64_t nblocks = n > 0 ? (n + kTile - 1) / kTile : 1;
    return align_up(sizeof(uint32_t) * kRadix * (size_t)nblocks) + align_up(sizeof(uint32_t) * kRadix);
}

hipError_t radix_sort_launch(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                             int64_t n, int key_bits, void *ws, hipStream_t s, int *in_tmp)
{
    *in_tmp = 0;
    if (n <= 0) return hipSuccess;
    const int64_t nblocks = (n + kTile - 1) / kTile;
    uint32_t *hist = static_cast<uint32_t *>(ws);
    uint32_t *digit_tot = reinterpret_cast<uint32_t *>(
        static_cast<char *>(ws) + align_up(sizeof(uint32_t) * kRadix * (size_t)nblocks));
    uint32_t *kin = keys, *kout = keys_tmp, *vin = vals, *vout = vals_tmp;
    for (int shift = 0; shift < key_bits; shift += kRadixBits) {
        hipLaunchKernelGGL(k_hist, dim3((unsigned)nblocks), dim3(kBlock), 0, s, kin, n, shift,
                           hist, (int)nblocks);
        hipLaunchKernelGGL(k_scan_digits, dim3(kRadix), dim3(kBlock), 0, s, hist, (int)nblocks,
                           digit_tot);
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)nblocks), dim3(kBlock), 0, s, kin, vin,
                           kout, vout, n, shift, hist, digit_tot, (int)nblocks);
        uint32_t *t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
        *in_tmp ^= 1;
    }
    return hipGetLastError();
}
