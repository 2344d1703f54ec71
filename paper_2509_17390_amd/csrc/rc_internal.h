// rc_internal.h -- shared declarations of librcast (device layouts, launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// ---------------------------------------------------------------------------
// Device data layouts.
//
// Binary BVH node record, 64 bytes = 4 x float4, child boxes stored
// coordinate-major so one float4 holds one axis of both children:
//   q0 = (L.lo.x, L.hi.x, R.lo.x, R.hi.x)
//   q1 = (L.lo.y, L.hi.y, R.lo.y, R.hi.y)
//   q2 = (L.lo.z, L.hi.z, R.lo.z, R.hi.z)
//   q3 = (ref L, ref R, -, -)   as int bits
// A child reference c >= 0 is an internal node index; c < 0 is the leaf
// holding triangle record ~c (leaf order).  Node 0 is the root.
//
// Triangle record, 48 bytes = 3 x float4, in leaf order:
//   (v0.x v0.y v0.z v1.x) (v1.y v1.z v2.x v2.y) (v2.z id - -)
// where id is the triangle's index in the uploaded mesh (int bits).
struct NodeRec {
    float4 q0, q1, q2;
    int4 q3;
};
static_assert(sizeof(NodeRec) == 64, "node record is 64 bytes");

struct TriRec {
    float4 a, b, c;
};
static_assert(sizeof(TriRec) == 48, "triangle record is 48 bytes");

// Quantised 4-wide node, 64 bytes (the binary tree collapsed two levels at a
// time).  Child k's box in the node's frame:
//   lo_a = origin_a + qlo_a[k] * scale_a,  hi_a = origin_a + qhi_a[k] * scale_a
// with 8-bit q (byte k of a packed word) and scale_a a power of two, rounded
// outward so the decoded box contains the child's exact FP32 box.
//   q0 = (origin.x, origin.y, origin.z, scale.x)
//   q1 = (scale.y, scale.z, qlo_x, qhi_x)        (q words as uint bits)
//   q2 = (qlo_y, qhi_y, qlo_z, qhi_z)
//   q3 = child refs: >= 0 Q8 node, < 0 leaf ~triangle record, INT_MIN empty
constexpr int32_t kEmptyChild = (int32_t)0x80000000;

// One job as the traversal kernels see it.
// Unsigned 32-bit division by a divisor fixed per launch, as a multiply and
// shifts (Granlund & Montgomery 1994, Fig. 4.1): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n):
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), for every n < 2^32.
struct UDiv {
    uint32_t m;
    uint32_t sh;   // min(l, 1) | max(l - 1, 0) << 8
};

inline UDiv udiv_magic(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    const uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1;
    UDiv u;
    u.m = (uint32_t)m;
    u.sh = (l > 0 ? 1u : 0u) | ((l > 0 ? l - 1 : 0u) << 8);
    return u;
}

struct DevJob {
    const NodeRec *nodes;   // null when the scene has no triangle
    const TriRec *tris;
    const float *dirs;      // [n_beams][3]
    const float *poses;     // [n_envs][12]
    int64_t ray_begin;      // first flattened ray of this job in the launch
    int64_t n_rays;         // n_envs * n_beams
    int64_t out_offset;
    int32_t n_beams;
    int32_t n_envs;
    int32_t n_tris;
    int32_t root_leaf;      // 1 when the scene is a single triangle (no nodes)
    float t_min, t_max;
    int32_t n_az;           // beams per elevation ring (n_beams % n_az == 0)
    int32_t tile_az;        // packet tile: tile_az x tile_el beams, row-major;
    int32_t tile_el;        //   tile_az | n_az and tile_el | n_beams / n_az
    int32_t tiles_az;       // n_az / tile_az
    UDiv div_beams;         // by n_beams
    UDiv div_tile;          // by tile_az * tile_el
    UDiv div_tiles_az;      // by n_az / tile_az
    UDiv div_tile_az;       // by tile_az
};
static_assert(sizeof(DevJob) == 128, "job record is 128 bytes");

// Work queues of the persistent traversal: the launch's flattened ray range
// is cut into kQueues contiguous parts, one per XCD; a wave takes rays from
// its XCD's part and steals from the others when that part is exhausted.
constexpr int kQueues = 8;
struct WorkQueues {
    unsigned long long head[kQueues];
    unsigned long long end[kQueues];
};

// Launch shape of the traversal (run-time tunable, see rc_tuning).
struct TraceConfig {
    int persistent;     // 1: persistent waves with refill; 0: one ray per thread
    int stack_lds;      // LDS stack entries per lane (8, 16 or 24)
    int refill_min;     // refill when at least this many lanes are idle (1..64)
    int blocks_per_cu;  // persistent grid = CUs x blocks_per_cu (0: occupancy limit)
    int chunk_max;      // largest ray chunk a persistent wave takes per atomic
    int waves_cap;      // 1: cap registers for 8 waves per SIMD (one-ray-per-thread kernel)
    int group_waves;    // waves per workgroup of the one-ray-per-thread grid (1 or 4)
    int leaf_batch;     // Q8 grid: 0 tests leaves on the spot; 1..64 queues them per wave
                        // and tests them once this many are queued (scenes < 2^26 tris)
};

// Largest scene (triangles) the queued-leaf traversal takes: a queued pair
// packs the lane (6 bits) and the leaf (26 bits) into one word.
constexpr int64_t kLeafBatchMaxTris = (int64_t)1 << 26;

// ---------------------------------------------------------------------------
// Launchers (implemented in build.hip / trace.hip).  All return hipError_t.

struct BuildBuffers {
    // inputs (a triangle mesh; lbvh_build_boxes_launch takes boxes instead)
    const float *verts;      // [nv][3]
    const int32_t *tris;     // [nt][3]
    int64_t nv, nt;
    int morton_bits;
    // workspace (caller-sized via lbvh_workspace_bytes)
    void *ws;
    size_t ws_bytes;
    // outputs (persistent per scene)
    uint32_t *morton;        // [nt]    input order
    uint32_t *sorted;        // [nt]    triangle index per leaf
    int32_t *topo;           // [nt-1][3] left, right, parent
    NodeRec *nodes;          // [max(nt-1,1)]
    TriRec *trirecs;         // [nt], or null (no triangle records)
    float *scene_box;        // [6] lo xyz, hi xyz (device)
    int32_t *depth_out;      // [1] device: tree depth
    NodeRec *q8nodes;        // [max(nt-1,1)] quantised 4-wide nodes, or null
    uint32_t *q8_count;      // [1] device: number of quantised nodes
};

size_t lbvh_workspace_bytes(int64_t nt);
hipError_t lbvh_build_launch(const BuildBuffers &b, hipStream_t s);

// validation of uploaded meshes: writes flags[0] |= 1 (bad index),
// |= 2 (non-finite vertex)
hipError_t validate_mesh_launch(const float *verts, int64_t nv, const int32_t *tris,
                                int64_t nt, int32_t *flags, hipStream_t s);

enum TraceMode { TRACE_BVH = 0, TRACE_BRUTE = 1, TRACE_STATS = 2 };

enum NodeFormat { FMT_BINARY = 0, FMT_Q8 = 1 };

hipError_t trace_launch(int mode, int fmt, const TraceConfig &cfg, const DevJob *jobs, int n_jobs,
                        WorkQueues *queues, int64_t total_rays, float *out_range,
                        int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris, hipStream_t s);

// Fill queue ranges for a launch of total_rays rays (host side).
void init_queues(WorkQueues &q, int64_t total_rays);

// Copy a queue template over the live queues (a kernel, so that it can be
// captured into a graph and replayed).
hipError_t queue_reset_launch(WorkQueues *live, const WorkQueues *tmpl, hipStream_t s);
