/*
 * rcast.h -- C ABI of librcast: batched LiDAR ray casting on one MI355X.
 *
 * The library implements the ray-casting stage of FGGS-LiDAR (Sec. IV-C):
 * a triangle mesh M = {(v_k0, v_k1, v_k2)}, per-environment sensor poses
 * T_s = [R_s | t_s] in SE(3) and a scan pattern of unit directions d_j go
 * in; for every (environment, beam) the nearest intersection
 *     t*_j = min_k eta(r_j, tri_k),  r_j(t) = t_s + t * R_s d_j,
 * over t in [t_min, t_max] comes out, as a range image plus the index of
 * the triangle hit.  The search runs over a linear BVH built on the GPU
 * (Sec. IV-A "LBVH construction": Morton codes of the primitives inside the
 * scene box, radix sort, hierarchy from longest common prefixes, bottom-up
 * box reduction; Sec. IV-C reuses it for triangle boxes) and prunes every
 * node whose entry distance exceeds the best hit so far.
 *
 * Conventions
 *   - Every call returns rc_status; nothing throws across the ABI.  On
 *     failure rc_last_error() gives a message for the calling thread.
 *   - Pointers are DEVICE pointers unless a parameter says "host".
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is
 *     stream-ordered: a call returns once the work is enqueued.
 *   - Handles are small integers owned by the context.
 *   - Scene and pattern calls on one context are serialised internally;
 *     rc_raycast_batch may be called from several threads.
 *   - Results: range in metres as float32, +INFINITY on a miss; hit id is
 *     the triangle's index in the uploaded index array, -1 on a miss.  The
 *     test is two-sided, [t_min, t_max] is closed, exact ties go to the
 *     lowest triangle index, and zero-area triangles are never hit.
 *   - Ray model: origin = translation column of the pose; direction =
 *     normalize(R * b_j) (computed in FP64, then rounded to FP32).  Pose
 *     layout: float32 [12], row-major [R | t] (3 rows of 4).
 */
#ifndef RCAST_H
#define RCAST_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rc_ctx rc_ctx;

typedef enum {
    RC_OK = 0,
    RC_PENDING = 1,
    RC_E_INVAL = -1,    /* bad argument, handle or input data             */
    RC_E_NOMEM = -2,    /* device memory or the context's budget exhausted */
    RC_E_NOTFOUND = -3, /* unknown handle or ticket                        */
    RC_E_BUSY = -4,     /* resource in use                                 */
    RC_E_DEVICE = -5,   /* a HIP runtime call failed                       */
    RC_E_STATE = -6     /* call not valid in the current state (e.g. no BVH) */
} rc_status;

enum { RC_NODE_FP32 = 0, RC_NODE_Q8 = 1 };

/* Message describing the last failing call made by this thread ("" if none).
 * The pointer stays valid until the next call on the same thread. */
const char *rc_last_error(void);

/* Library version, for the binding to check it loaded the right file. */
int32_t rc_version(void);

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold for scenes, patterns and internal
 * buffers (0 = no cap beyond the device itself).  *out receives the handle.
 * Errors: RC_E_INVAL (bad device or NULL out), RC_E_DEVICE. */
rc_status rc_create(int device, uint64_t hbm_budget_bytes, rc_ctx **out);

/* Wait for all work the context enqueued, then free everything it owns. */
void rc_destroy(rc_ctx *ctx);

/* Copy a triangle mesh (the mesh M of Sec. IV-C) into the context.
 *   verts_xyz : float32 [n_verts][3]
 *   tri_idx   : int32   [n_tris][3], indices into verts
 *   src_is_device : 1 if both arrays are device pointers, 0 if host
 * The caller keeps ownership of its arrays; the library copies them and
 * validates indices (0 <= i < n_verts) and that every vertex is finite.
 * n_tris may be 0 (every ray then misses).  The copy is complete when the
 * call returns.  *out_scene receives the scene handle.
 * Errors: RC_E_INVAL (bad sizes, index out of range, non-finite vertex),
 * RC_E_NOMEM (budget), RC_E_DEVICE. */
rc_status rc_scene_upload(rc_ctx *ctx, const float *verts_xyz, int64_t n_verts,
                          const int32_t *tri_idx, int64_t n_tris,
                          int src_is_device, void *stream, int32_t *out_scene);

/* Options for rc_lbvh_build.  Zero-initialised means the defaults. */
typedef struct {
    int32_t morton_bits; /* bits per axis, 1..10 (0 = 10)                    */
    int32_t node_format; /* RC_NODE_FP32 (binary nodes with FP32 child boxes)
                            or RC_NODE_Q8 (8-bit quantised child boxes)       */
    int32_t reserved[6];
} rc_build_opts;

/* Build (or rebuild) the BVH of `scene` on the GPU (Sec. IV-A LBVH
 * construction, applied to triangle boxes as in Sec. IV-C).  Runs on
 * `stream`; the BVH stays resident until the scene is released.  A later
 * raycast on any stream must be ordered after this call's stream work.
 * With node_format = RC_NODE_Q8 the binary tree is also collapsed into
 * 4-wide nodes whose child boxes are 8-bit offsets in the node's frame,
 * rounded outward; a launch whose scenes all carry them traverses those
 * (results are bit-identical to the FP32 nodes).
 * Errors: RC_E_NOTFOUND (scene), RC_E_INVAL (options), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_lbvh_build(rc_ctx *ctx, int32_t scene, const rc_build_opts *opts,
                        void *stream);

/* Drop a scene (the mesh M of Sec. IV-C stays resident for every cast that
 * uses it).  The handle is invalid from the moment the call returns: new
 * casts, builds and requests naming it fail with RC_E_NOTFOUND.  The
 * scene's memory is reference-counted and its free deferred while it is in
 * use: every cast, build or served batch that resolved the scene before the
 * release holds a reference until its device work has finished, and a graph
 * (rc_graph_create) holds one until it is destroyed.  When the last one
 * goes, the memory is freed by the next call into the context that reclaims
 * it (rc_scene_upload, rc_lbvh_build, rc_scene_release, rc_pattern_upload,
 * rc_scene_get_info, rc_device_bytes, rc_graph_destroy, rc_destroy) or by
 * the request server; a scene not in use is freed at once.  Never waits
 * for the device.  Casts enqueued on a stream that is being captured into
 * the caller's own graph hold no reference past the call: the caller keeps
 * their scenes until that graph is destroyed.  Errors: RC_E_NOTFOUND
 * (unknown or already released scene). */
rc_status rc_scene_release(rc_ctx *ctx, int32_t scene);

/* Copy a scan pattern (the unit directions d_j of Sec. IV-C) in.
 *   dirs_xyz : HOST float32 [n_beams][3]; the library normalises each
 *              direction after rotating it, so lengths need not be 1
 *   n_az_hint: beams per elevation ring (0 if unknown); used to shape
 *              coherent ray tiles
 * Errors: RC_E_INVAL (n_beams < 1, non-finite or zero direction),
 * RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_pattern_upload(rc_ctx *ctx, const float *dirs_xyz, int32_t n_beams,
                            int32_t n_az_hint, int32_t *out_pattern);

/* One job of a batch: n_envs sensor poses against one scene and pattern.
 * Its results occupy out[out_offset + e * n_beams + j]. */
typedef struct {
    int32_t scene;
    int32_t pattern;
    int32_t n_envs;
    int32_t reserved0;
    const float *poses_3x4; /* DEVICE float32 [n_envs][12], row-major [R|t] */
    float t_min, t_max;     /* closed range interval, 0 <= t_min <= t_max   */
    int64_t out_offset;
} rc_job;

/* Cast every ray of every job (Sec. IV-C nearest intersection, batched over
 * environments and scenes in one launch).  out_range (float32) and out_hit
 * (int32) are DEVICE arrays owned by the caller, large enough for every
 * job's slice.  Stream-ordered on `stream`.
 * Errors: RC_E_INVAL (bad job), RC_E_NOTFOUND (scene/pattern),
 * RC_E_STATE (scene has no BVH), RC_E_DEVICE. */
rc_status rc_raycast_batch(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs,
                           float *out_range, int32_t *out_hit, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): same contract and results
 * as rc_raycast_batch, with no device or host-pinned allocation.  The
 * launch's job table and work queues live in a fixed device array of 32,896
 * bytes (work queues + 256 job records of 128 bytes), one per GPU, held
 * until the process ends; the table reaches it through small kernel
 * launches (no copy, no memset).  At most 256 jobs per call (RC_E_INVAL
 * beyond).  Every call on one GPU shares that array and leaves the last
 * call's table in it: calls ordered one after another on one stream are
 * safe; calls that overlap on one GPU (on different streams, or from
 * threads racing on one stream) race on it and may corrupt each other's
 * launch.  Scenes are referenced as in rc_raycast_batch; at most 256 such
 * launches may be in flight per context (RC_E_BUSY beyond).
 * Errors: as rc_raycast_batch; RC_E_BUSY. */
rc_status rc_raycast_batch_noalloc(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs,
                                   float *out_range, int32_t *out_hit, void *stream);

/* Same contract as rc_raycast_batch, but every ray is tested against every
 * triangle (the naive O(N_r * N_tri) baseline of Sec. IV-C) with the same
 * FP32 triangle test.  A GPU cross-check of the BVH path: for rays that
 * are not near-ties its output is bit-identical to rc_raycast_batch. */
rc_status rc_raycast_bruteforce(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs,
                                float *out_range, int32_t *out_hit, void *stream);

/* Instrumented traversal: like rc_raycast_batch, and additionally writes
 * per-ray counts of BVH node records fetched (out_nodes) and triangles
 * tested (out_tris), DEVICE int32 arrays laid out like out_range.  These
 * are N_nodes(r_j) and K_j of the per-ray cost model of Sec. IV-C. */
rc_status rc_raycast_stats(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs,
                           float *out_range, int32_t *out_hit, int32_t *out_nodes,
                           int32_t *out_tris, void *stream);

/* Introspection of a built scene. */
typedef struct {
    int64_t n_verts, n_tris;
    int64_t n_nodes;        /* internal nodes of the binary BVH            */
    int64_t n_q8_nodes;     /* quantised 4-wide nodes (RC_NODE_Q8), else 0 */
    int32_t depth;          /* longest root-to-leaf path (edges)           */
    int32_t node_format;
    int32_t morton_bits;
    int32_t has_bvh;
    uint64_t device_bytes;  /* device memory held by the scene             */
    float scene_lo[3], scene_hi[3];
} rc_scene_info;

rc_status rc_scene_get_info(rc_ctx *ctx, int32_t scene, rc_scene_info *out);

/* Copy an internal array of a built scene to HOST memory (for tests of the
 * build kernels).  `what`:
 *   RC_DBG_MORTON   uint32 [n_tris]  Morton code of each triangle (input order)
 *   RC_DBG_SORTED   uint32 [n_tris]  triangle index in leaf (sorted) order
 *   RC_DBG_TOPOLOGY int32  [n_nodes][3]  left, right, parent of each internal
 *                   node; children >= 0 are internal nodes, a child c < 0 is
 *                   the leaf holding sorted triangle ~c; the root's parent is -1
 *   RC_DBG_NODES    raw node records (format-dependent bytes)
 *   RC_DBG_TRIS     raw triangle records (48 bytes each)
 *   RC_DBG_Q8NODES  quantised 4-wide node records, 64 bytes each, sized for
 *                   n_nodes records (the first n_q8_nodes are used)
 * `bytes` must equal the array's size.  Synchronises the device. */
enum { RC_DBG_MORTON = 1, RC_DBG_SORTED = 2, RC_DBG_TOPOLOGY = 3,
       RC_DBG_NODES = 4, RC_DBG_TRIS = 5, RC_DBG_Q8NODES = 6 };
rc_status rc_scene_debug_copy(rc_ctx *ctx, int32_t scene, int32_t what,
                              void *host_dst, uint64_t bytes);

/* Bytes the context currently holds on the device (a mock context counts
 * the host copies of its scenes' vertices).  Frees released scenes whose
 * last reference has gone first. */
uint64_t rc_device_bytes(rc_ctx *ctx);

/* Launch shape of the traversal.  Every setting gives bit-identical results
 * (the closest hit is the lexicographic minimum of (t, triangle id) and box
 * culling is conservative); they only change speed.
 *   persistent    1: persistent waves that take rays from per-XCD work
 *                 queues and refill idle lanes by wavefront ballot;
 *                 0: one ray per thread, one launch-wide grid (default)
 *   stack_lds     the top entries of each lane's traversal stack kept in
 *                 LDS, as a ring (deeper entries in scratch): 8, 16 or 24
 *                 for the persistent kernel; 0 (default), 8 or 16 otherwise
 *   refill_min    a persistent wave refills once this many of its 64 lanes
 *                 are idle (1..64, default 64)
 *   blocks_per_cu persistent grid = CUs x this (0 = occupancy limit)
 *   tile_az/el    packet tile: consecutive rays of an environment cover a
 *                 tile_az x tile_el block of (azimuth, elevation) beams; used
 *                 for a job when tile_az divides the pattern's n_az hint and
 *                 tile_el its ring count; 0 = plain beam order (default
 *                 16 x 4) */
typedef struct {
    int32_t persistent;
    int32_t stack_lds;
    int32_t refill_min;
    int32_t blocks_per_cu;
    int32_t tile_az;
    int32_t tile_el;
    int32_t chunk_max;     /* largest ray chunk a persistent wave claims per
                              atomic (64..2^20; 0 = 4096); chunks shrink as
                              the queue empties */
    int32_t waves_cap;     /* 1 (default): one-ray-per-thread kernel compiled
                              for at most 64 VGPRs (8 waves per SIMD) */
    int32_t group_waves;   /* waves per workgroup of the one-ray-per-thread
                              grid: 1 (default; a finished wave frees its slot
                              at once) or 4 (spreads a small launch over more
                              CUs) */
    int32_t leaf_batch;    /* one-ray-per-thread grid on quantised (RC_NODE_Q8)
                              trees: 0 tests each leaf's triangle when the
                              lane reaches it; 1..64 queues (lane, leaf) pairs
                              per wave and tests them 64 at a time, with every
                              lane busy, once this many are queued (lanes keep
                              traversing meanwhile).  Ignored for launches
                              with a scene of more than 2^26 triangles, for
                              plain FP32 trees and for persistent waves. */
} rc_tuning;

/* Set (NULL: reset to defaults) or read the context's traversal tuning.
 * Applies to launches enqueued after the call.  Errors: RC_E_INVAL. */
rc_status rc_set_tuning(rc_ctx *ctx, const rc_tuning *tuning);
rc_status rc_get_tuning(rc_ctx *ctx, rc_tuning *out);

/* Autotuner: launch the batch once per candidate launch shape (warm-up,
 * then the fastest of `reps` launches timed with HIP events on `stream`),
 * keep the fastest as the context's tuning and report it.  Candidates:
 * one-ray-per-thread with stack_lds {0, 8} x waves_cap {1, 0} x tiles
 * {16x4, 8x8, 32x2, plain} in one-wave workgroups, and with stack_lds
 * {0, 8} x waves_cap {1, 0} x tiles {16x4, plain} in four-wave workgroups;
 * queued leaf tests with leaf_batch {16, 32, 64} in one- and four-wave
 * workgroups (16x4 tiles, register cap);
 * persistent with stack_lds {8, 16} x refill_min {48, 64} x blocks_per_cu
 * {2, 4}.  Every candidate writes the same,
 * complete results into out_range / out_hit.  Synchronises `stream`.
 * Errors: as rc_raycast_batch. */
rc_status rc_autotune(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs, float *out_range,
                      int32_t *out_hit, void *stream, int32_t reps, rc_tuning *out_best,
                      float *out_ms);

/* Persisted autotuner results.  Once rc_tuning_cache_load has been called on
 * a context, rc_autotune first looks the batch up by its key -- the device
 * (architecture name and compute-unit count), the node format, the size
 * class of the largest scene (floor(log2(triangles))), the beam pattern
 * (rings x azimuths of the first job, or "mixed" when jobs differ), the
 * size class of the batch (floor(log2(rays))) and of its job count -- and on
 * a hit sets and reports the stored tuning without launching anything
 * (*out_ms = -1, outputs untouched); on a miss it tunes as above and stores
 * the result under the key.  The file (host path) is plain text, one entry
 * per line after a version line; a missing file loads as an empty cache.
 * rc_tuning_cache_save writes every entry (to `path`.tmp, then renames).
 * Errors: RC_E_INVAL (bad argument, malformed file or an entry whose tuning
 * is out of range: nothing is loaded), RC_E_DEVICE (file I/O failed). */
rc_status rc_tuning_cache_load(rc_ctx *ctx, const char *path);
rc_status rc_tuning_cache_save(rc_ctx *ctx, const char *path);

/* A batch captured in a hipGraph (queue reset + one traversal launch) for
 * replay, e.g. once per simulation frame.  The job table (scenes, patterns,
 * pose and output pointers, ranges, offsets) and the context's tuning are
 * fixed at creation; callers update pose contents in place between
 * replays.  The graph holds a reference to each of its scenes until it is
 * destroyed (a release meanwhile defers the free); rebuilding a scene's BVH
 * in place is allowed (ordered on the stream before the replay).  The graph holds no
 * hipMemset node.  Replays on one graph must not overlap (they share the
 * graph's work queues): order them on one stream.
 * Errors: as rc_raycast_batch; RC_E_DEVICE if capture fails. */
typedef struct rc_graph rc_graph;
rc_status rc_graph_create(rc_ctx *ctx, const rc_job *jobs, int32_t n_jobs, float *out_range,
                          int32_t *out_hit, rc_graph **out);
rc_status rc_graph_launch(rc_graph *graph, void *stream);
void rc_graph_destroy(rc_graph *graph);

/* ---------------------------------------------------------------------
 * Serving: requests of different scenes, environment counts and beam
 * patterns arrive at any time and are batched continuously.  Requests are
 * admitted in arrival order as soon as their footprint (8 bytes of output
 * per ray + 48 bytes of pose per environment) fits in the server's arenas;
 * the requests admitted at one moment share one batched launch (up to
 * max_batch_rays_m million rays), and up to max_inflight launches run at
 * once on separate streams.  Each request's
 * results are bit-identical to casting it alone with rc_raycast_batch.
 * A request whose scene is released while it is still queued fails with
 * RC_E_NOTFOUND; once its batch has been launched, the release defers the
 * scene's free until the batch has finished and the request completes
 * normally.  Patterns stay resident until rc_destroy. */
typedef struct {
    int32_t scene;
    int32_t pattern;
    int32_t n_envs;           /* >= 1                                        */
    int32_t reserved0;
    const float *poses_3x4;   /* HOST float32 [n_envs][12]; copied by submit */
    float t_min, t_max;       /* closed range interval                       */
} rc_request;

typedef struct {
    uint64_t arena_bytes;     /* device memory for admitted requests
                                 (0 = 4 GiB; >= 1 MiB); 1/64 holds poses     */
    int32_t max_inflight;     /* launches in flight at once, 1..8 (0 = 2);
                                 each has its own stream, but a process gets
                                 4 hardware queues by default, so launches
                                 beyond 4 share queues and wait in them */
    int32_t max_batch_rays_m; /* cap on rays per launch, millions (0 = none):
                                 admission stops before a request that would
                                 exceed it; a larger request runs alone     */
    int32_t mock_ns_per_ray;  /* mock context: simulated device time per ray */
    int32_t mock_fail_scene;  /* mock context: requests on scene
                                 (mock_fail_scene - 1) fail with RC_E_DEVICE
                                 (0 = none)                                  */
    int32_t policy;           /* admission order: 0 = arrival order, never
                                 overtaking (default); 1 = fewest rays first
                                 among requests queued less than max_wait_ms,
                                 older ones first in arrival order           */
    int32_t max_wait_ms;      /* policy 1: age after which a request goes
                                 ahead of younger ones (0 = 200 ms)          */
    int32_t mock_launch_delay_us; /* mock context: pause between resolving a
                                 batch's scenes and handing it to the
                                 simulated device (tests of a release racing
                                 a launch; 0 = none)                         */
    int32_t reserved[1];
} rc_serve_opts;

typedef struct {
    uint64_t submitted, completed, failed, rejected, cancelled;
    uint64_t launches;            /* batched launches issued                 */
    uint64_t max_batch_requests;  /* most requests folded into one launch    */
    uint64_t bytes_in_use, peak_bytes;  /* arena bytes held by requests      */
    uint64_t out_capacity_bytes;
    uint64_t pending, inflight, peak_inflight;
} rc_serve_stats;

/* Start / stop the context's server (one per context).  Stop waits for
 * launched work and invalidates every ticket. Errors: RC_E_INVAL (options),
 * RC_E_STATE (already running / not running), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_serve_start(rc_ctx *ctx, const rc_serve_opts *opts);
rc_status rc_serve_stop(rc_ctx *ctx);

/* Queue a request; never blocks on the device.  *out_ticket identifies it.
 * Errors: RC_E_STATE (server not running, scene without BVH),
 * RC_E_NOTFOUND (scene/pattern), RC_E_INVAL (sizes, non-finite pose),
 * RC_E_NOMEM (the request could never fit in the arenas). */
rc_status rc_serve_submit(rc_ctx *ctx, const rc_request *request, uint64_t *out_ticket);

/* Wait up to timeout_us (0: just check, < 0: forever) for a ticket.
 * RC_OK: *out_range / *out_hit point at its results (DEVICE memory for a
 * GPU context, host memory for a mock context; n_envs * n_beams entries,
 * [env][beam]) and *latency_ms is completion minus submission time.
 * RC_PENDING: not finished yet.  A failed request returns its error status.
 * Errors: RC_E_NOTFOUND (ticket), RC_E_STATE. */
rc_status rc_serve_poll(rc_ctx *ctx, uint64_t ticket, int64_t timeout_us,
                        const float **out_range, const int32_t **out_hit, double *latency_ms);

/* Drop a ticket: frees its results (or cancels it if still queued).
 * Errors: RC_E_NOTFOUND, RC_E_BUSY (currently on the device). */
rc_status rc_serve_release(rc_ctx *ctx, uint64_t ticket);

/* Copy a finished ticket's results (n_envs * n_beams floats and int32s)
 * into caller buffers, host (dst_is_host = 1) or device; either may be NULL.
 * Synchronous.  RC_PENDING if the ticket has not finished; a failed request
 * returns its error status.  Errors: RC_E_NOTFOUND, RC_E_STATE, RC_E_DEVICE. */
rc_status rc_serve_copy(rc_ctx *ctx, uint64_t ticket, float *range_dst, int32_t *hit_dst,
                        int dst_is_host);

/* Counters of the running server. */
rc_status rc_serve_get_stats(rc_ctx *ctx, rc_serve_stats *out);

/* ------------------------------------------------------------------------
 * Gaussian-to-occupancy conversion (Sec. IV-A, "Grid query and occupancy
 * evaluation", on the Gaussian model of Sec. III-A).
 *
 * A Gaussian G_i has mean mu_i, covariance Sigma_i = R_i S_i S_i^T R_i^T and
 * opacity alpha_i; its box b_i is the axis-aligned box of the k-sigma
 * ellipsoid, mu_i +- k sqrt(diag Sigma_i).  On a voxel grid (origin o,
 * spacing h, voxel (i, j, k) = the cell o + [i, i+1] x [j, j+1] x [k, k+1] h
 * with centre v = o + (i + 1/2, j + 1/2, k + 1/2) h) cut into tiles of 8^3
 * voxels, each voxel receives
 *     D(v) = sum over G_i in C_tile of
 *            exp(-1/2 (v - mu_i)^T Sigma_i^-1 (v - mu_i)) alpha_i^2,
 *     C_tile = { G_i : b_i meets the tile's box }  (closed boxes),
 * then V_occ = [D(v) > theta] and Surf = V_occ and not (V_occ on all six
 * face neighbours), neighbours outside the grid counting as unoccupied.
 * C_tile is found by querying an LBVH over the boxes (Morton codes of the
 * box centres, radix sort, Karras hierarchy, bottom-up box reduction).
 * Box ends and tile-box ends are evaluated in FP64 and rounded to the
 * nearest float32, so membership is an exact float32 comparison.
 * ---------------------------------------------------------------------- */

/* Copy n Gaussians in (3DGS parameterisation, with activations applied):
 *   means_xyz  float32 [n][3]
 *   quats_wxyz float32 [n][4]  rotation quaternion (w, x, y, z); need not be
 *                              unit length (R is the rotation of q / |q|)
 *   scales_xyz float32 [n][3]  linear scales, > 0 (S = diag(s))
 *   opacity    float32 [n]     alpha in [0, 1]
 *   src_is_device: 1 if all four arrays are device pointers, 0 if host.
 * The caller keeps ownership; the copy is complete when the call returns.
 * n may be 0 (every density is then 0).  *out_set receives the handle.
 * Errors: RC_E_INVAL (sizes, non-finite value, scale <= 0, zero quaternion,
 * opacity outside [0, 1]), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_gauss_upload(rc_ctx *ctx, const float *means_xyz, const float *quats_wxyz,
                          const float *scales_xyz, const float *opacity, int64_t n,
                          int src_is_device, void *stream, int32_t *out_set);

/* Options for rc_gauss_build.  Zero-initialised means the defaults. */
typedef struct {
    float cutoff_sigma;   /* k of the k-sigma boxes, > 0 (0 = 3)            */
    int32_t morton_bits;  /* bits per axis, 1..10 (0 = 10)                  */
    int32_t reserved[6];
} rc_gauss_opts;

/* Compute the Gaussian boxes and build the LBVH over them (Sec. IV-A LBVH
 * construction) plus the per-leaf evaluation records, on `stream`.  A later
 * rc_voxelize on any stream must be ordered after this call's work.
 * Errors: RC_E_NOTFOUND (set), RC_E_INVAL (options), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_gauss_build(rc_ctx *ctx, int32_t set, const rc_gauss_opts *opts, void *stream);

/* Drop a Gaussian set.  Waits for the device, then frees its memory.
 * Errors: RC_E_NOTFOUND. */
rc_status rc_gauss_release(rc_ctx *ctx, int32_t set);

/* Voxel grid of one conversion. */
typedef struct {
    float origin[3];     /* o, metres                                        */
    float spacing;       /* h > 0, metres                                    */
    int32_t dims[3];     /* nx, ny, nz >= 1; at most 2^30 voxels per axis    */
    int32_t tile;        /* tile edge B in voxels: 8 (0 = 8)                 */
    float theta;         /* density threshold (finite)                       */
    int32_t reserved[3];
} rc_grid;

/* Convert a built set on `grid`.  Outputs are DEVICE arrays owned by the
 * caller, laid out [nz][ny][nx] (x fastest):
 *   out_density float32 D(v), or NULL
 *   out_occ     uint8   V_occ (0/1), or NULL
 *   out_surf    uint8   Surf (0/1), or NULL; needs out_occ
 * At least one output must be given.  Stream-ordered on `stream`.  The
 * density is accumulated in fixed point with units of 2^-31 per term, so
 * results are identical from run to run; V_occ is taken on the float32 D.
 * Errors: RC_E_INVAL (grid, outputs), RC_E_NOTFOUND (set), RC_E_STATE (set
 * not built), RC_E_DEVICE. */
rc_status rc_voxelize(rc_ctx *ctx, int32_t set, const rc_grid *grid, float *out_density,
                      uint8_t *out_occ, uint8_t *out_surf, void *stream);

/* |C_tile| of every tile, DEVICE int32 [tz][ty][tx] with t = ceil(n / 8)
 * per axis (the query of rc_voxelize without the evaluation).  Same errors. */
rc_status rc_voxelize_counts(rc_ctx *ctx, int32_t set, const rc_grid *grid,
                             int32_t *out_tile_counts, void *stream);

/* Copy an internal array of a built set to HOST memory (for tests):
 *   RC_GDBG_BOXES     float32 [n][6]  Gaussian boxes lo xyz, hi xyz (input order)
 *   RC_GDBG_SORTED    uint32 [n]      Gaussian index in leaf order
 *   RC_GDBG_TOPOLOGY  int32 [n-1][3]  as RC_DBG_TOPOLOGY
 *   RC_GDBG_RECORDS   64 bytes per leaf: mu xyz, alpha^2 2^31, the whitening
 *                     matrix c0 S^-1 R^T (row-major, c0 = sqrt(log2(e) / 2)),
 *                     the Gaussian's index (int bits), 2 unused
 * `bytes` must equal the array's size.  Synchronises the device. */
enum { RC_GDBG_BOXES = 1, RC_GDBG_SORTED = 2, RC_GDBG_TOPOLOGY = 3, RC_GDBG_RECORDS = 4 };
rc_status rc_gauss_debug_copy(rc_ctx *ctx, int32_t set, int32_t what, void *host_dst,
                              uint64_t bytes);

/* ------------------------------------------------------------------------
 * Narrow-band TSDF and marching cubes (Sec. IV-B), from a surface mask V on
 * a grid (origin, spacing, dims of rc_grid; its tile and theta are unused):
 *   V'    = G * V, G the binomial kernel of n = max(1, round(2 sigma^2))
 *           steps (sigma in voxels, halves rounded up): integer weights
 *           C(2n, n + k), k = -n..n, separable, zero outside the grid;
 *           V~ = [V' >= tau] (or the quantile form, see rc_tsdf_opts),
 *           decided exactly on the integer sums
 *   O     = free voxels (V~ = 0) 6-connected to a free frame around the grid;
 *           s = +1 on O, -1 elsewhere
 *   S_0   = voxels with a 6-neighbour of the other V~ value (frame = 0)
 *   p     = first shell of a 6-neighbour expansion from S_0 reaching the
 *           voxel, counted up to ceil(band / h)
 *   phi   = clip(s p h, -band, band) (band where p was not reached)
 * Marching cubes runs on the lattice of voxel centres: a corner is inside
 * when phi < iso; each crossed lattice edge carries one vertex at
 * t = (iso - phi_a) / (phi_b - phi_a) from its lower end; vertices are
 * numbered by (voxel, axis x/y/z), triangles by (cell, position in the case
 * table); triangles face the region phi >= iso.
 * ---------------------------------------------------------------------- */
typedef struct {
    float sigma_smooth;   /* smoothing scale, metres, > 0 (n <= 10)          */
    float tau;            /* fixed re-threshold (finite; mode 0)             */
    float band;           /* r, metres, > 0; band / spacing <= 250           */
    int32_t threshold_mode; /* 0: V~ = [V' >= tau]; 1: V~ = [V' >= Quantile_q(V')]
                               (Sec. IV-B quantile re-threshold eq.): over all
                               N voxels, the quantile interpolated linearly
                               between the order statistics x_k and x_(k+1),
                               k = floor(q (N - 1)); decided exactly on the
                               integer sums (sum >= x_k when q (N - 1) is an
                               integer, else sum >= x_(k+1))               */
    float quantile;       /* q in [0, 1] (mode 1)                            */
    int32_t reserved[3];
} rc_tsdf_opts;

/* TSDF of the DEVICE uint8 surface mask `surf` [nz][ny][nx] into the DEVICE
 * float32 `out_phi` (same layout); `out_vtilde` (DEVICE uint8, or NULL)
 * receives V~.  Runs on `stream` and returns when phi is complete (the
 * outside labelling repeats until it settles, reading a flag each round).
 * Scratch device memory of about 14 bytes per voxel (22 with the quantile
 * re-threshold, which keeps the smoothing's integer sums) is kept by the context
 * (grown on demand, reused by later calls, freed by rc_destroy).
 * Errors: RC_E_INVAL (grid, options), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_tsdf(rc_ctx *ctx, const rc_grid *grid, const uint8_t *surf,
                  const rc_tsdf_opts *opts, float *out_phi, uint8_t *out_vtilde, void *stream);

/* Marching cubes of the DEVICE float32 field `phi` [nz][ny][nx] at `iso`.
 * Always writes the mesh size to *n_verts / *n_tris.  With out_verts (DEVICE
 * float32 [cap_verts][3]) and out_tris (DEVICE int32 [cap_tris][3]) given
 * and large enough, also writes the mesh; with both NULL only counts (call
 * once to size, once to fill; a capacity already large enough fills in one
 * call).  out_normals (DEVICE float32 [cap_verts][3], or NULL; needs
 * out_verts) receives the unit vertex normals from the gradient of phi
 * (Sec. IV-B isosurface extraction): per lattice point the central
 * difference, one-sided on the grid's faces, interpolated along the
 * vertex's edge like its position; they point toward growing phi, out of
 * the solid; (0, 0, 0) where the gradient vanishes.  Synchronous.  Scratch
 * of about 4 bytes per voxel is kept by the context like rc_tsdf's.  Grids
 * up to 2^29 voxels.
 * Errors: RC_E_INVAL, RC_E_NOMEM (capacity too small: sizes still written),
 * RC_E_DEVICE. */
rc_status rc_marching_cubes(rc_ctx *ctx, const rc_grid *grid, const float *phi, float iso,
                            float *out_verts, int32_t *out_tris, float *out_normals,
                            int64_t cap_verts, int64_t cap_tris, int64_t *n_verts,
                            int64_t *n_tris, void *stream);

/* Marching cubes with the step-size parameter mc_step of Sec. IV-B
 * ("Isosurface extraction"): the same extraction on the lattice of every
 * step-th voxel centre along each axis -- points (i, j, k) * step with
 * i <= (nx - 1) / step and so on, as a grid of spacing fl32(step * h) and
 * origin fl32(o - (step - 1) h / 2) per axis (FP64, rounded once), whose
 * voxel centres fall on the fine centres -- so vertex and triangle
 * numbering follow that coarser lattice.
 * step = 1 is rc_marching_cubes.  Other arguments, sizes and errors as
 * rc_marching_cubes, plus RC_E_INVAL for step < 1; a temporary device
 * buffer of 4 bytes per coarse point is allocated and freed by the call. */
rc_status rc_marching_cubes_step(rc_ctx *ctx, const rc_grid *grid, const float *phi, float iso,
                                 int32_t step, float *out_verts, int32_t *out_tris,
                                 float *out_normals, int64_t cap_verts, int64_t cap_tris,
                                 int64_t *n_verts, int64_t *n_tris, void *stream);

/* The marching-cubes case table, HOST arrays: count[256] triangles per case
 * (corner k inside sets bit k; corner k = (k & 1, k >> 1 & 1, k >> 2 & 1))
 * and tris[256][15] cube-edge ids, -1 padded (edge 4 a + j joins the j-th
 * corner, ascending, with bit a clear to its neighbour along axis a). */
rc_status rc_marching_cubes_table(uint8_t *count, int8_t *tris);

/* ------------------------------------------------------------------------
 * Point-cloud fidelity (Sec. V "Metrics"): between a simulated LiDAR cloud P
 * and a ground-truth cloud G,
 *   d(p, G) = min over g of |p - g| (Euclidean, FP64 from float32 points),
 *   CD = (mean over P of d(p, G) + mean over G of d(g, P)) / 2,
 *   precision = share of P with d(p, G) <= tau, recall = share of G with
 *   d(g, P) <= tau, F = 2 precision recall / (precision + recall).
 * Nearest neighbours are exact (an LBVH over the reference points, FP64
 * distances, exact box pruning); ties go to the lowest reference index.
 * ---------------------------------------------------------------------- */

/* For every query point, the distance to and index of its nearest reference
 * point.  ref_xyz, query_xyz: DEVICE float32 [n][3]; out_dist: DEVICE float64
 * [n_query]; out_idx: DEVICE int32 [n_query].  n_ref = 0 gives +INFINITY and
 * -1.  Synchronous; scratch is kept by the context.
 * Errors: RC_E_INVAL, RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_nearest(rc_ctx *ctx, const float *ref_xyz, int64_t n_ref, const float *query_xyz,
                     int64_t n_query, double *out_dist, int32_t *out_idx, void *stream);

typedef struct {
    double chamfer;     /* CD, metres                                       */
    double mean_pg;     /* mean over P of d(p, G)                           */
    double mean_gp;     /* mean over G of d(g, P)                           */
    double precision, recall, fscore;
    int64_t n_p, n_g;
} rc_fidelity;

/* CD and F-score at `tau` (metres; the paper uses 0.05) of DEVICE float32
 * clouds P [n_p][3] and G [n_g][3], both non-empty.  Synchronous.
 * Errors: RC_E_INVAL, RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_chamfer_fscore(rc_ctx *ctx, const float *p_xyz, int64_t n_p, const float *g_xyz,
                            int64_t n_g, float tau, rc_fidelity *out, void *stream);

/* Taubin smoothing (Sec. IV-B "Mesh optimization"; the paper's defaults are
 * lambda = 0.5, mu = -0.53), in place on the DEVICE float32 vertex array
 * verts_xyz [n_verts][3] of the mesh tri_idx (DEVICE int32 [n_tris][3]).
 * Each iteration moves every vertex by lambda, then by mu, times the
 * umbrella operator (mean of its distinct edge neighbours minus itself);
 * vertices on an edge of a single triangle and vertices without neighbours
 * stay in place.  Float32, neighbours summed in ascending index order.
 * Synchronous.  At most 64 triangles per vertex.
 * Errors: RC_E_INVAL (sizes, indices, non-finite vertex or parameters,
 * valence), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_taubin_smooth(rc_ctx *ctx, float *verts_xyz, int64_t n_verts, const int32_t *tri_idx,
                           int64_t n_tris, float lambda, float mu, int32_t iterations,
                           void *stream);

/* Quadric-error decimation (Sec. IV-B "Mesh optimization") by vertex
 * clustering: vertices are grouped by a uniform grid of cell size c
 * anchored at the mesh's box minimum (vertices on an edge of one triangle
 * keep groups of their own); each group becomes one vertex at the minimiser
 * of the sum of its vertices' quadrics (area-weighted planes of the
 * incident triangles) when that is well posed and lies within the group's
 * cell widened by one cell, else at its vertices' mean; triangles whose
 * corners fall into three groups are kept in input order.  c is the
 * smallest of a geometric bisection (12 steps, between extent / 1023 and
 * the extent) whose face count is at most floor(ratio * n_tris).
 * verts_xyz, tri_idx: DEVICE input mesh; out_verts (DEVICE float32
 * [n_verts][3]) and out_tris (DEVICE int32 [n_tris][3]) receive the result
 * (never larger than the input); sizes in *n_verts_out / *n_tris_out and
 * the cell size in *cell_out (may be NULL).  Synchronous.  At most 64
 * triangles per vertex.  Errors: RC_E_INVAL, RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_decimate(rc_ctx *ctx, const float *verts_xyz, int64_t n_verts, const int32_t *tri_idx,
                      int64_t n_tris, float ratio, float *out_verts, int32_t *out_tris,
                      int64_t *n_verts_out, int64_t *n_tris_out, float *cell_out, void *stream);

/* Quadric-error decimation by rounds of parallel edge contraction
 * (Sec. IV-B "Mesh optimization": quadric-error decimation to a face ratio;
 * Sec. V "Implementation": ratio 0.1, three rounds, boundary protected).
 * Faces with a repeated corner are dropped first; F0 faces remain.  Round
 * k = 1..rounds runs until at most ceil(F0 * ratio^(k / rounds)) faces
 * remain or no edge can contract; at its start every vertex's quadric is
 * the sum of its faces' plane quadrics (Garland and Heckbert 1997; squared
 * distance to the plane, faces weighted equally) and the vertices on an
 * edge that is not on exactly two faces are protected (never moved, their
 * edges never contracted).  A step contracts, at once, every edge that
 * (a) lies on exactly two faces, (b) has two unprotected ends, (c) has
 * exactly two common neighbours (link condition), (d) flips no face when
 * both ends move to its point x* (the minimiser of Q_u + Q_v when well
 * conditioned and within twice the edge length of the midpoint, else the
 * cheapest of the ends and the midpoint), (e) is among the
 * ceil((F - target) / 2) smallest keys (float32 cost, pi(e)) -- e the
 * edge's rank among all edges (u < v) in lexicographic order, pi the
 * "lowbias32" bijection of 32-bit integers, so equal costs (flat regions)
 * are ordered pseudo-randomly and many edges contract per step -- and (f) has
 * the smallest key among those at every vertex of its two closed
 * one-rings; the contracted vertex takes x* and Q_u + Q_v.  FP64 inside,
 * positions rounded to float32 at the end; the result is deterministic.
 * Output: the vertices a remaining face uses, in ascending input order,
 * renumbered densely, and the remaining faces in ascending input order.
 * verts_xyz (float32 [n_verts][3]) and tri_idx (int32 [n_tris][3]) are
 * DEVICE arrays; out_verts / out_tris are DEVICE arrays of at least
 * n_verts / n_tris entries (never larger than the input; must not alias
 * it); *n_steps_out (may be NULL) receives the number of contraction
 * steps.  Synchronous.  Scratch of about 900 bytes per vertex and 120 per
 * triangle is kept by the context.  Errors: RC_E_INVAL (sizes, null
 * arrays, an index out of range or a non-finite vertex, ratio outside
 * (0, 1], rounds outside 1..64, a vertex with more than 64 incident faces
 * or 64 neighbours at some step), RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_decimate_qem(rc_ctx *ctx, const float *verts_xyz, int64_t n_verts,
                          const int32_t *tri_idx, int64_t n_tris, float ratio, int32_t rounds,
                          float *out_verts, int32_t *out_tris, int64_t *n_verts_out,
                          int64_t *n_tris_out, int32_t *n_steps_out, void *stream);

/* Removal of tiny components (Sec. IV-B "Mesh optimization": decimation
 * also removes tiny components).  Two triangles are connected when they
 * share a vertex; components with fewer than min_faces triangles are
 * dropped (exactly min_faces is kept; min_faces <= 1 keeps every
 * triangle).  The kept triangles keep their input order; the vertices
 * they reference keep their input order and are renumbered densely;
 * vertices no kept triangle references are dropped.  verts_xyz, tri_idx:
 * DEVICE input mesh (float32 [n_verts][3], int32 [n_tris][3]); out_verts
 * (DEVICE float32 [n_verts][3]) and out_tris (DEVICE int32 [n_tris][3])
 * receive the result (never larger than the input; must not alias the
 * input); sizes in *n_verts_out / *n_tris_out.  Synchronous.  Scratch of
 * 20 bytes per vertex and 8 per triangle is kept by the context.
 * Errors: RC_E_INVAL (sizes, null arrays, an index out of range),
 * RC_E_NOMEM, RC_E_DEVICE. */
rc_status rc_remove_small_components(rc_ctx *ctx, const float *verts_xyz, int64_t n_verts,
                                     const int32_t *tri_idx, int64_t n_tris, int64_t min_faces,
                                     float *out_verts, int32_t *out_tris, int64_t *n_verts_out,
                                     int64_t *n_tris_out, void *stream);

/* Device id of a host-only context for rc_create: no HIP calls; scenes and
 * patterns hold their sizes only (rc_scene_upload needs host arrays);
 * rc_raycast_* report RC_E_STATE; the server runs requests on a simulated
 * device that writes range = ray index within the request and
 * hit = scene id.  For testing the scheduler without a GPU. */
#define RC_DEVICE_MOCK (-1)

#ifdef __cplusplus
}
#endif

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#endif /* RCAST_H */
