// ctx.h -- host-side context of librcast, shared by the C ABI (api.hip) and
// the serving scheduler (serve.hip).  Not part of the public interface.
#pragma once

#include "rcast.h"
#include "rc_internal.h"
#include "mesh_internal.h"

#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace rc {

// Set the calling thread's error text and return `s`.
rc_status fail(rc_status s, const char *fmt, ...);

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::rc::fail(RC_E_DEVICE, "%s failed: %s (%s:%d)", #expr,                  \
                              hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

// A scene's life: upload makes it alive; rc_scene_release makes it dead
// (no new work may resolve it) and its memory is freed once `refs` is zero.
// Every launch, build or captured graph that resolved the scene holds one
// reference until its device work has finished (graphs: until destroyed).
// `refs` and `dead` are guarded by rc_ctx::ref_mu, the rest by rc_ctx::mu.
struct Scene {
    bool alive = false;   // the slot holds a scene and its memory
    bool dead = false;    // released; freed when refs drops to zero
    int refs = 0;
    int64_t nv = 0, nt = 0;
    float *verts = nullptr;
    int32_t *tris = nullptr;
    bool has_bvh = false;
    int morton_bits = 10;
    int node_format = RC_NODE_FP32;
    uint32_t *morton = nullptr;
    uint32_t *sorted = nullptr;
    int32_t *topo = nullptr;
    NodeRec *nodes = nullptr;
    TriRec *trirecs = nullptr;
    NodeRec *q8nodes = nullptr;  // quantised 4-wide nodes (node_format == RC_NODE_Q8)
    float *box_dev = nullptr;    // [8]: box (6) + depth (int bits) + quantised node count
    uint64_t bytes = 0;
    // mock context: a host copy of the vertices stands in for the device
    // arrays, so the simulated device reads real scene memory
    float *host_verts = nullptr;
    double host_sum = 0.0;
};

struct Pattern {
    bool alive = false;
    float *dirs = nullptr;
    int32_t n_beams = 0, n_az = 0;
    uint64_t bytes = 0;
};

// A set of Gaussians (Sec. III-A) and its LBVH (Sec. IV-A).
struct GaussSet {
    bool alive = false;
    int64_t n = 0;
    float4 *params = nullptr;    // [n][3]: (mu, alpha) (quaternion) (scale, 0)
    float *boxes = nullptr;      // [n][6] Gaussian boxes (input order)
    bool has_bvh = false;
    float cutoff = 3.0f;         // k of the k-sigma boxes
    int morton_bits = 10;
    uint32_t *morton = nullptr;
    uint32_t *sorted = nullptr;
    int32_t *topo = nullptr;
    NodeRec *nodes = nullptr;
    GaussRec *recs = nullptr;    // [n] evaluation records in leaf order
    float *box_dev = nullptr;    // [8]: box (6) + depth (int bits) + unused
    uint64_t bytes = 0;

    GaussParams view() const
    {
        GaussParams p;
        p.g = params;
        p.n = n;
        return p;
    }
};

constexpr int kSlots = 8;

// A slot holds one launch's job table followed by its work queues.
struct JobSlot {
    DevJob *host = nullptr;  // pinned: DevJob[cap] then WorkQueues
    DevJob *dev = nullptr;
    int cap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};

struct ServeState;  // serve.hip

// References dropped by a host function once the work enqueued before it on
// a stream has finished.  Records with slot >= 0 belong to the context's
// pool, preallocated for the launch entry point that allocates nothing.
struct DropRec {
    rc_ctx *c = nullptr;
    std::vector<Scene *> held;
    int slot = -1;
};

// rc_raycast_batch_noalloc: jobs per call (its job table lives in a fixed
// device array of WorkQueues + kNoAllocJobs DevJob records) and pooled drop
// records per context (launches of it in flight at once).
constexpr int kNoAllocJobs = 256;
constexpr int kDropPool = 256;

}  // namespace rc

struct rc_ctx {
    int device = 0;
    bool mock = false;    // host-only context (no HIP): serving runs on a simulated device
    uint64_t budget = 0;
    uint64_t used = 0;
    std::mutex mu;        // scenes, patterns, workspace
    std::mutex job_mu;    // job slots, tuning
    std::deque<rc::Scene> scenes;  // elements never move: holds keep Scene pointers
    std::vector<rc::Pattern> patterns;
    std::vector<rc::GaussSet> gsets;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ws_event = nullptr;
    bool ws_event_recorded = false;
    rc::JobSlot slots[rc::kSlots];
    int next_slot = 0;
    int32_t *flags_dev = nullptr;
    rc_tuning tuning{};
    rc::ServeState *serve = nullptr;
    uint8_t *mc_table = nullptr;   // marching-cubes case table on the device (256 + 256 * 15 bytes)
    // scene references (never held across a HIP call that waits for the
    // device, so host functions on a stream can always take it)
    std::mutex ref_mu;
    std::condition_variable ref_cv;
    std::vector<rc::Scene *> reap;       // dead scenes without references, freed under mu
    int pending_drops = 0;               // drop host functions enqueued and not yet run
    std::vector<rc::DropRec> drop_pool;  // kDropPool records, each with room for
    std::vector<int> drop_free;          //   kNoAllocJobs scenes; indices of free ones
    char *scratch = nullptr;             // this device's fixed launch array (api.hip)
    bool tune_cache_on = false;    // rc_tuning_cache_load was called (guarded by job_mu)
    std::map<std::string, rc_tuning> tune_cache;
    std::mutex mesh_mu;            // TSDF / marching-cubes calls and their scratch
    void *mesh_ws = nullptr;       // grow-only scratch of those calls
    size_t mesh_ws_bytes = 0;
};

namespace rc {

// Scene references (see Scene).  hold_scene: caller holds c->mu.
// drop_holds: any thread, makes no HIP call; a dead scene left without
// references goes to c->reap.  reap_locked: caller holds c->mu; frees the
// scenes on c->reap.  drop_after: drops `held` once the work enqueued so
// far on `s` has finished (a host function; at once when `s` is being
// captured into a graph, whose owner keeps the scenes alive); empties `held`.
void hold_scene(rc_ctx *c, Scene *s);
void drop_holds(rc_ctx *c, Scene *const *s, size_t n);
void reap_locked(rc_ctx *c);
rc_status drop_after(rc_ctx *c, hipStream_t s, std::vector<Scene *> &held);

rc_status dev_alloc(rc_ctx *c, void **p, size_t bytes);
void dev_free(rc_ctx *c, void *p, size_t bytes);
Scene *get_scene(rc_ctx *c, int32_t id);      // caller holds c->mu
Pattern *get_pattern(rc_ctx *c, int32_t id);  // caller holds c->mu
void free_gauss_set(rc_ctx *c, GaussSet &g);  // caller holds c->mu

// Grow the shared LBVH build workspace to at least `need` bytes and order
// `s` after the previous build that used it.  Caller holds c->mu.
rc_status ensure_build_ws(rc_ctx *c, size_t need, hipStream_t s);
rc_tuning default_tuning();

// Job table staging owned by one caller stream (the request server keeps
// one per stream).  Device layout: WorkQueues, then DevJob[cap].  The caller
// guarantees that no launch still reads `dev` when it stages the next batch
// and keeps `host` unchanged until the launch has completed.
struct StageBuf {
    char *dev = nullptr;
    int cap = 0;
    std::vector<char> host;
};

// Stage one batch and launch it on `stream`; `forced` overrides the
// context's tuning; `own` replaces the context's shared staging ring.
// Thread-safe.
// Jobs whose scene or pattern is gone are skipped and listed in `skipped`
// when it is given (else the call fails with RC_E_NOTFOUND).
rc_status trace_common(rc_ctx *c, int mode, const rc_job *jobs, int32_t n_jobs, float *out_range,
                       int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris, void *stream,
                       const rc_tuning *forced = nullptr, StageBuf *own = nullptr,
                       std::vector<int> *skipped = nullptr);
void stage_free(rc_ctx *c, StageBuf &b);

// Serving scheduler hooks (serve.hip).
void serve_shutdown(rc_ctx *c);  // stop the scheduler, wait for in-flight work

}  // namespace rc
