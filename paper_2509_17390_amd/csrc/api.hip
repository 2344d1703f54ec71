// api.hip -- the C ABI of librcast (see include/rcast.h).
//
// Host-side runtime: a context per device owns scene and pattern tables, the
// LBVH build workspace and a ring of job-table slots (pinned staging buffer
// + device buffer + completion event), so a batch call only enqueues one
// small host-to-device copy and one traversal launch on the caller's stream.
#include "ctx.h"

#include <errno.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

namespace rc {

thread_local std::string g_err;

rc_status fail(rc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

rc_status dev_alloc(rc_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (c->budget && c->used + bytes > c->budget)
        return fail(RC_E_NOMEM, "device budget exceeded: %llu + %llu > %llu bytes",
                    (unsigned long long)c->used, (unsigned long long)bytes,
                    (unsigned long long)c->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RC_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    c->used += bytes;
    return RC_OK;
}

void dev_free(rc_ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    if (bytes == 0) bytes = 256;
    (void)hipFree(p);
    c->used -= bytes;
}

size_t scene_bvh_bytes(int64_t nt)
{
    int64_t ni = nt > 1 ? nt - 1 : 1;
    return sizeof(uint32_t) * nt * 2 + sizeof(int32_t) * 3 * ni + sizeof(NodeRec) * ni +
           sizeof(TriRec) * nt;
}

void free_bvh(rc_ctx *c, Scene &s)
{
    int64_t nt = s.nt, ni = nt > 1 ? nt - 1 : 1;
    dev_free(c, s.morton, sizeof(uint32_t) * nt);
    dev_free(c, s.sorted, sizeof(uint32_t) * nt);
    dev_free(c, s.topo, sizeof(int32_t) * 3 * ni);
    dev_free(c, s.nodes, sizeof(NodeRec) * ni);
    dev_free(c, s.trirecs, sizeof(TriRec) * nt);
    dev_free(c, s.q8nodes, sizeof(NodeRec) * ni);
    s.q8nodes = nullptr;
    s.morton = s.sorted = nullptr;
    s.topo = nullptr;
    s.nodes = nullptr;
    s.trirecs = nullptr;
    s.has_bvh = false;
}

void free_scene(rc_ctx *c, Scene &s)
{
    if (c->mock) {
        free(s.host_verts);
        c->used -= s.bytes;
        s = Scene();
        return;
    }
    free_bvh(c, s);
    dev_free(c, s.verts, sizeof(float) * 3 * s.nv);
    dev_free(c, s.tris, sizeof(int32_t) * 3 * s.nt);
    dev_free(c, s.box_dev, sizeof(float) * 8);
    s = Scene();
}

// A live (uploaded, not released) scene, or null.
Scene *get_scene(rc_ctx *c, int32_t id)
{
    if (id < 0 || id >= (int32_t)c->scenes.size()) return nullptr;
    Scene &s = c->scenes[id];
    return s.alive && !s.dead ? &s : nullptr;
}

// ---------------------------------------------------------------------------
// Scene references.  `dead` is written with both c->mu and c->ref_mu held,
// so it may be read under either; `refs` only under c->ref_mu.

void hold_scene(rc_ctx *c, Scene *s)
{
    std::lock_guard<std::mutex> lk(c->ref_mu);
    ++s->refs;
}

void drop_holds(rc_ctx *c, Scene *const *s, size_t n)
{
    std::lock_guard<std::mutex> lk(c->ref_mu);
    for (size_t i = 0; i < n; ++i)
        if (--s[i]->refs == 0 && s[i]->dead) c->reap.push_back(s[i]);
}

void reap_locked(rc_ctx *c)
{
    std::vector<Scene *> r;
    {
        std::lock_guard<std::mutex> lk(c->ref_mu);
        if (c->reap.empty()) return;
        r.swap(c->reap);
    }
    for (Scene *s : r) free_scene(c, *s);
}

namespace {

// Host function behind a launch or build: no HIP call, no c->mu.  A pooled
// record goes back to the pool (clear() keeps its capacity).
void drop_host_fn(void *arg)
{
    DropRec *d = static_cast<DropRec *>(arg);
    rc_ctx *c = d->c;
    drop_holds(c, d->held.data(), d->held.size());
    const int slot = d->slot;
    if (slot < 0) delete d;
    std::lock_guard<std::mutex> lk(c->ref_mu);
    if (slot >= 0) {
        d->held.clear();
        c->drop_free.push_back(slot);
    }
    --c->pending_drops;
    c->ref_cv.notify_all();
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

}  // namespace

// Drop the references of record d once the work enqueued so far on s has
// finished (at once while s is being captured).
rc_status enqueue_drop(rc_ctx *c, hipStream_t s, DropRec *d)
{
    {
        std::lock_guard<std::mutex> lk(c->ref_mu);
        ++c->pending_drops;
    }
    if (stream_capturing(s)) {
        drop_host_fn(d);
        return RC_OK;
    }
    hipError_t e = hipLaunchHostFunc(s, drop_host_fn, d);
    if (e != hipSuccess) {
        // no host function: wait for the stream, then drop here
        (void)hipStreamSynchronize(s);
        drop_host_fn(d);
        return fail(RC_E_DEVICE, "hipLaunchHostFunc failed: %s", hipGetErrorString(e));
    }
    return RC_OK;
}

rc_status drop_after(rc_ctx *c, hipStream_t s, std::vector<Scene *> &held)
{
    if (held.empty()) return RC_OK;
    DropRec *d = new DropRec();
    d->c = c;
    d->held.swap(held);
    return enqueue_drop(c, s, d);
}

Pattern *get_pattern(rc_ctx *c, int32_t id)
{
    if (id < 0 || id >= (int32_t)c->patterns.size() || !c->patterns[id].alive) return nullptr;
    return &c->patterns[id];
}

// Packet tile of a job: the tuned tile when it divides the pattern, else
// one elevation ring at a time (plain beam order).
void pick_tile(const rc_tuning &t, int32_t n_beams, int32_t n_az, DevJob &d)
{
    if (n_az < 1 || n_beams % n_az != 0) n_az = n_beams;
    const int32_t n_el = n_beams / n_az;
    d.n_az = n_az;
    d.tile_az = n_az;
    d.tile_el = 1;
    if (t.tile_az > 0 && t.tile_el > 0 && n_az % t.tile_az == 0 && n_el % t.tile_el == 0) {
        d.tile_az = t.tile_az;
        d.tile_el = t.tile_el;
    }
    d.tiles_az = n_az / d.tile_az;
    d.div_beams = udiv_magic((uint32_t)(n_beams > 0 ? n_beams : 1));
    d.div_tile = udiv_magic((uint32_t)(d.tile_az * d.tile_el));
    d.div_tiles_az = udiv_magic((uint32_t)(n_az / d.tile_az));
    d.div_tile_az = udiv_magic((uint32_t)d.tile_az);
}

rc_status check_tuning(const rc_tuning *t);

rc_tuning default_tuning()
{
    rc_tuning t;
    memset(&t, 0, sizeof t);
    t.persistent = 0;
    t.stack_lds = 0;
    t.refill_min = 64;
    t.blocks_per_cu = 0;
    t.tile_az = 16;
    t.tile_el = 4;
    t.chunk_max = 4096;
    t.waves_cap = 1;
    t.group_waves = 1;
    t.leaf_batch = 0;
    return t;
}

// Build the device job table for a batch; shared by every trace entry point.
// out[] and held[] have room for n_jobs entries; *n_out jobs are written,
// and held[k] is the scene of out[k], referenced on return (the caller drops
// the references, also when this call fails: *n_out says how many).  With
// `skipped`, a job whose scene or pattern is gone (or has no BVH) is left
// out and its index listed instead of failing the call.
rc_status prepare_jobs(rc_ctx *c, const rc_tuning &tuning, const rc_job *jobs, int32_t n_jobs,
                       DevJob *out, Scene **held, int *n_out, int64_t &total, int &fmt,
                       std::vector<int> *skipped)
{
    *n_out = 0;
    total = 0;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(RC_E_INVAL, "bad job list");
    bool all_q8 = true;
    std::lock_guard<std::mutex> lk(c->mu);
    for (int i = 0; i < n_jobs; ++i) {
        const rc_job &j = jobs[i];
        Scene *s = get_scene(c, j.scene);
        Pattern *p = get_pattern(c, j.pattern);
        if (skipped && (!s || !p || (s->nt > 0 && !s->has_bvh))) {
            skipped->push_back(i);
            continue;
        }
        if (!s) return fail(RC_E_NOTFOUND, "job %d: unknown scene %d", i, j.scene);
        if (!p) return fail(RC_E_NOTFOUND, "job %d: unknown pattern %d", i, j.pattern);
        if (s->nt > 0 && !s->has_bvh)
            return fail(RC_E_STATE, "job %d: scene %d has no BVH (call rc_lbvh_build)", i, j.scene);
        if (j.n_envs < 0) return fail(RC_E_INVAL, "job %d: n_envs < 0", i);
        if (j.n_envs > 0 && !j.poses_3x4) return fail(RC_E_INVAL, "job %d: poses is NULL", i);
        if (!(j.t_min >= 0.0f) || !(j.t_max >= j.t_min) || !isfinite(j.t_min))
            return fail(RC_E_INVAL, "job %d: need 0 <= t_min <= t_max", i);
        if (j.out_offset < 0) return fail(RC_E_INVAL, "job %d: out_offset < 0", i);
        int64_t nr = (int64_t)j.n_envs * p->n_beams;
        if (nr > (int64_t)0x7fffffff) return fail(RC_E_INVAL, "job %d: more than 2^31-1 rays", i);
        const int k = (*n_out)++;
        hold_scene(c, s);
        held[k] = s;
        DevJob &d = out[k];
        d.nodes = s->nodes;
        if (s->node_format != RC_NODE_Q8) all_q8 = false;
        d.tris = s->trirecs;
        d.dirs = p->dirs;
        d.poses = j.poses_3x4;
        d.ray_begin = total;
        d.n_rays = nr;
        d.out_offset = j.out_offset;
        d.n_beams = p->n_beams;
        d.n_envs = j.n_envs;
        d.n_tris = (int32_t)s->nt;
        d.root_leaf = s->nt == 1 ? 1 : 0;
        d.t_min = j.t_min;
        d.t_max = j.t_max;
        pick_tile(tuning, p->n_beams, p->n_az, d);
        total += nr;
    }
    // quantised nodes only when every scene of the launch has them
    fmt = (all_q8 && *n_out > 0) ? FMT_Q8 : FMT_BINARY;
    if (fmt == FMT_Q8)
        for (int k = 0; k < *n_out; ++k) out[k].nodes = held[k]->q8nodes;
    return RC_OK;
}

// Copy a job table into the next ring slot; returns the device pointer.
size_t slot_bytes(int cap) { return sizeof(DevJob) * cap + sizeof(WorkQueues); }

rc_status stage_jobs(rc_ctx *c, const std::vector<DevJob> &dj, int64_t total, hipStream_t stream,
                     DevJob **dev, WorkQueues **queues, JobSlot **slot_out)
{
    JobSlot &sl = c->slots[c->next_slot];
    c->next_slot = (c->next_slot + 1) % kSlots;
    if (sl.used) HIP_TRY(hipEventSynchronize(sl.done));
    int need = (int)dj.size() > 0 ? (int)dj.size() : 1;
    if (need > sl.cap) {
        int cap = 64;
        while (cap < need) cap *= 2;
        if (sl.host) (void)hipHostFree(sl.host);
        // c->used is guarded by c->mu (taken inside job_mu, never the other way)
        std::lock_guard<std::mutex> lk(c->mu);
        if (sl.dev) dev_free(c, sl.dev, slot_bytes(sl.cap));
        sl.host = nullptr;
        sl.dev = nullptr;
        sl.cap = 0;
        HIP_TRY(hipHostMalloc((void **)&sl.host, slot_bytes(cap), hipHostMallocDefault));
        rc_status st = dev_alloc(c, (void **)&sl.dev, slot_bytes(cap));
        if (st != RC_OK) return st;
        sl.cap = cap;
    }
    memcpy(sl.host, dj.data(), sizeof(DevJob) * dj.size());
    WorkQueues *hq = reinterpret_cast<WorkQueues *>(sl.host + sl.cap);
    init_queues(*hq, total);
    HIP_TRY(hipMemcpyAsync(sl.dev, sl.host, sizeof(DevJob) * dj.size(), hipMemcpyHostToDevice,
                           stream));
    WorkQueues *dq = reinterpret_cast<WorkQueues *>(sl.dev + sl.cap);
    HIP_TRY(hipMemcpyAsync(dq, hq, sizeof(WorkQueues), hipMemcpyHostToDevice, stream));
    *dev = sl.dev;
    *queues = dq;
    *slot_out = &sl;
    return RC_OK;
}

// Launch configuration of a batch: the tuning, with queued leaf tests off
// when a scene is too large for the queue's packed (lane, leaf) words.
TraceConfig config_of(const rc_tuning &t, const DevJob *jobs, int n_jobs)
{
    TraceConfig cfg;
    cfg.leaf_batch = t.leaf_batch;
    for (int k = 0; k < n_jobs; ++k)
        if ((int64_t)jobs[k].n_tris > kLeafBatchMaxTris) cfg.leaf_batch = 0;
    cfg.persistent = t.persistent;
    cfg.stack_lds = t.stack_lds;
    cfg.refill_min = t.refill_min;
    cfg.blocks_per_cu = t.blocks_per_cu;
    cfg.chunk_max = t.chunk_max;
    cfg.waves_cap = t.waves_cap;
    cfg.group_waves = t.group_waves;
    return cfg;
}

size_t stage_bytes(int cap) { return sizeof(WorkQueues) + sizeof(DevJob) * (size_t)cap; }

void stage_free(rc_ctx *c, StageBuf &b)
{
    std::lock_guard<std::mutex> lk(c->mu);
    dev_free(c, b.dev, stage_bytes(b.cap));
    b.dev = nullptr;
    b.cap = 0;
}

// Copy a job table into caller-owned staging (no host wait: the caller
// orders reuse, see StageBuf).
rc_status stage_own(rc_ctx *c, StageBuf &b, const std::vector<DevJob> &dj, int64_t total,
                    hipStream_t stream, DevJob **dev, WorkQueues **queues)
{
    const int need = (int)dj.size() > 0 ? (int)dj.size() : 1;
    if (need > b.cap) {
        int cap = 64;
        while (cap < need) cap *= 2;
        std::lock_guard<std::mutex> lk(c->mu);
        dev_free(c, b.dev, stage_bytes(b.cap));
        b.dev = nullptr;
        b.cap = 0;
        rc_status st = dev_alloc(c, (void **)&b.dev, stage_bytes(cap));
        if (st != RC_OK) return st;
        b.cap = cap;
    }
    const size_t bytes = sizeof(WorkQueues) + sizeof(DevJob) * dj.size();
    b.host.resize(bytes);
    init_queues(*reinterpret_cast<WorkQueues *>(b.host.data()), total);
    memcpy(b.host.data() + sizeof(WorkQueues), dj.data(), sizeof(DevJob) * dj.size());
    HIP_TRY(hipMemcpyAsync(b.dev, b.host.data(), bytes, hipMemcpyHostToDevice, stream));
    *queues = reinterpret_cast<WorkQueues *>(b.dev);
    *dev = reinterpret_cast<DevJob *>(b.dev + sizeof(WorkQueues));
    return RC_OK;
}

// Stage and launch one batch; `forced` overrides the context's tuning.  The
// batch's scenes stay referenced until the launch has finished.
rc_status trace_common(rc_ctx *c, int mode, const rc_job *jobs, int32_t n_jobs, float *out_range,
                       int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris, void *stream,
                       const rc_tuning *forced, StageBuf *own, std::vector<int> *skipped)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (c->mock) return fail(RC_E_STATE, "a mock context has no device to cast on");
    rc_tuning tuning;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        tuning = forced ? *forced : c->tuning;
    }
    const size_t cap = n_jobs > 0 ? (size_t)n_jobs : 0;
    std::vector<DevJob> dj(cap);
    std::vector<Scene *> held(cap);
    int n_run = 0;
    int64_t total = 0;
    int fmt = FMT_BINARY;
    rc_status st = prepare_jobs(c, tuning, jobs, n_jobs, dj.data(), held.data(), &n_run, total,
                                fmt, skipped);
    dj.resize(n_run);
    held.resize(n_run);
    // until the launch is enqueued, a failure drops the references here
    struct Guard {
        rc_ctx *c;
        std::vector<Scene *> &h;
        ~Guard() { if (!h.empty()) drop_holds(c, h.data(), h.size()); }
    } guard{c, held};
    if (st != RC_OK) return st;
    if (total == 0) return RC_OK;
    if (!out_range || !out_hit) return fail(RC_E_INVAL, "null output");
    if (mode == TRACE_STATS && (!out_nodes || !out_tris)) return fail(RC_E_INVAL, "null stats output");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevJob *djd = nullptr;
    WorkQueues *dq = nullptr;
    hipError_t e = hipSuccess;
    if (own) {
        st = stage_own(c, *own, dj, total, s, &djd, &dq);
        if (st != RC_OK) return st;
        e = trace_launch(mode, fmt, config_of(tuning, dj.data(), n_run), djd, n_run, dq, total,
                         out_range, out_hit, out_nodes, out_tris, s);
    } else {
        std::lock_guard<std::mutex> lk(c->job_mu);
        JobSlot *slot = nullptr;
        st = stage_jobs(c, dj, total, s, &djd, &dq, &slot);
        if (st != RC_OK) return st;
        e = trace_launch(mode, fmt, config_of(tuning, dj.data(), n_run), djd, n_run, dq, total,
                         out_range, out_hit, out_nodes, out_tris, s);
        if (e == hipSuccess) e = hipEventRecord(slot->done, s);
        if (e == hipSuccess) slot->used = true;
    }
    if (e != hipSuccess) {
        // part of the batch may be on the device: let it finish first
        (void)hipStreamSynchronize(s);
        return fail(RC_E_DEVICE, "traversal launch failed: %s", hipGetErrorString(e));
    }
    return drop_after(c, s, held);
}

rc_status ensure_build_ws(rc_ctx *c, size_t need, hipStream_t s)
{
    if (need > c->ws_bytes) {
        if (c->ws) {
            HIP_TRY(hipDeviceSynchronize());
            dev_free(c, c->ws, c->ws_bytes);
            c->ws = nullptr;
            c->ws_bytes = 0;
        }
        rc_status st = dev_alloc(c, &c->ws, need);
        if (st != RC_OK) return st;
        c->ws_bytes = need;
        c->ws_event_recorded = false;
    }
    if (c->ws_event_recorded) HIP_TRY(hipStreamWaitEvent(s, c->ws_event, 0));
    return RC_OK;
}

// ---------------------------------------------------------------------------
// Launch scratch of rc_raycast_batch_noalloc: the work queues and job table
// of one launch in a fixed device array.  Each GPU holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress gives for that device (the array's name is a host
// stand-in, not a device address).  Calls that overlap on one GPU share it.
constexpr size_t kScratchBytes = sizeof(WorkQueues) + sizeof(DevJob) * kNoAllocJobs;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};

// Address of this device's scratch; the device must be current.  Looked up
// once per device.
rc_status scratch_of_device(int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return fail(RC_E_INVAL, "device %d: at most %d devices", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RC_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s",
                        device, hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[device];
    return RC_OK;
}

// The job table reaches the scratch as kernel arguments (16 records per
// launch), so no host staging buffer is needed.
constexpr int kFillJobs = 16;
struct ScratchFill {
    uint4 words[kFillJobs * sizeof(DevJob) / 16];
    WorkQueues queues;
    int32_t first, count, with_queues, pad;
};
static_assert(sizeof(DevJob) % 16 == 0, "job records are whole uint4s");
static_assert(sizeof(ScratchFill) <= 4096, "kernel arguments stay within 4 KiB");

__global__ void k_fill_scratch(char *scr, ScratchFill a)
{
    constexpr int per = (int)(sizeof(DevJob) / 16);
    uint4 *jobs = reinterpret_cast<uint4 *>(scr + sizeof(WorkQueues)) + a.first * per;
    for (int i = threadIdx.x; i < a.count * per; i += blockDim.x) jobs[i] = a.words[i];
    if (a.with_queues && threadIdx.x < kQueues) {
        WorkQueues *q = reinterpret_cast<WorkQueues *>(scr);
        q->head[threadIdx.x] = a.queues.head[threadIdx.x];
        q->end[threadIdx.x] = a.queues.end[threadIdx.x];
    }
}

}  // namespace rc

using namespace rc;

extern "C" {

const char *rc_last_error(void) { return g_err.c_str(); }

int32_t rc_version(void) { return 1; }

rc_status rc_create(int device, uint64_t hbm_budget_bytes, rc_ctx **out)
{
    if (!out) return fail(RC_E_INVAL, "out is NULL");
    *out = nullptr;
    if (device == RC_DEVICE_MOCK) {
        rc_ctx *c = new rc_ctx();
        c->device = RC_DEVICE_MOCK;
        c->mock = true;
        c->budget = hbm_budget_bytes;
        c->tuning = default_tuning();
        *out = c;
        return RC_OK;
    }
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(RC_E_INVAL, "device %d not in [0, %d)", device, n);
    HIP_TRY(hipSetDevice(device));
    rc_ctx *c = new rc_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->tuning = default_tuning();
    hipError_t e = hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < kSlots; ++i)
        e = hipEventCreateWithFlags(&c->slots[i].done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void **)&c->flags_dev, 256);
    if (e != hipSuccess) {
        rc_destroy(c);
        return fail(RC_E_DEVICE, "context setup failed: %s", hipGetErrorString(e));
    }
    rc_status st = scratch_of_device(device, &c->scratch);
    if (st != RC_OK) {
        rc_destroy(c);
        return st;
    }
    // drop records of rc_raycast_batch_noalloc, allocated here once
    c->drop_pool.resize(kDropPool);
    c->drop_free.reserve(kDropPool);
    for (int i = 0; i < kDropPool; ++i) {
        c->drop_pool[i].c = c;
        c->drop_pool[i].slot = i;
        c->drop_pool[i].held.reserve(kNoAllocJobs);
        c->drop_free.push_back(kDropPool - 1 - i);
    }
    *out = c;
    return RC_OK;
}

void rc_destroy(rc_ctx *c)
{
    if (!c) return;
    serve_shutdown(c);
    if (c->mock) {
        for (auto &s : c->scenes)
            if (s.alive) free_scene(c, s);
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    {
        // every drop host function has run before the scenes go
        std::unique_lock<std::mutex> lk(c->ref_mu);
        c->ref_cv.wait(lk, [&] { return c->pending_drops == 0; });
    }
    for (auto &s : c->scenes)
        if (s.alive) free_scene(c, s);
    for (auto &p : c->patterns)
        if (p.alive) dev_free(c, p.dirs, p.bytes);
    for (auto &g : c->gsets)
        if (g.alive) free_gauss_set(c, g);
    if (c->mc_table) dev_free(c, c->mc_table, 256 + 256 * 15);
    if (c->mesh_ws) dev_free(c, c->mesh_ws, c->mesh_ws_bytes);
    for (auto &sl : c->slots) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) dev_free(c, sl.dev, slot_bytes(sl.cap));
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (c->ws) dev_free(c, c->ws, c->ws_bytes);
    if (c->ws_event) (void)hipEventDestroy(c->ws_event);
    if (c->flags_dev) (void)hipFree(c->flags_dev);
    delete c;
}

rc_status rc_scene_upload(rc_ctx *c, const float *verts, int64_t nv, const int32_t *tris,
                          int64_t nt, int src_is_device, void *stream, int32_t *out_scene)
{
    if (!c || !out_scene) return fail(RC_E_INVAL, "null context or out_scene");
    if (nv < 0 || nt < 0) return fail(RC_E_INVAL, "negative sizes");
    if (nt > 0x7ffffffeLL) return fail(RC_E_INVAL, "too many triangles (%lld)", (long long)nt);
    if ((nv > 0 && !verts) || (nt > 0 && !tris)) return fail(RC_E_INVAL, "null mesh array");
    if (nt > 0 && nv == 0) return fail(RC_E_INVAL, "triangles without vertices");
    if (c->mock) {
        if (src_is_device) return fail(RC_E_INVAL, "a mock context takes host arrays only");
        for (int64_t i = 0; i < 3 * nt; ++i)
            if (tris[i] < 0 || tris[i] >= nv) return fail(RC_E_INVAL, "invalid mesh: index out of range");
        for (int64_t i = 0; i < 3 * nv; ++i)
            if (!isfinite(verts[i])) return fail(RC_E_INVAL, "invalid mesh: non-finite vertex");
        std::lock_guard<std::mutex> lk(c->mu);
        reap_locked(c);
        Scene sc;
        sc.nv = nv;
        sc.nt = nt;
        // the host copy of the vertices is the mock scene's "device" memory
        sc.bytes = sizeof(float) * 3 * (uint64_t)(nv > 0 ? nv : 1);
        if (c->budget && c->used + sc.bytes > c->budget)
            return fail(RC_E_NOMEM, "device budget exceeded: %llu + %llu > %llu bytes",
                        (unsigned long long)c->used, (unsigned long long)sc.bytes,
                        (unsigned long long)c->budget);
        sc.host_verts = static_cast<float *>(malloc(sc.bytes));
        if (!sc.host_verts) return fail(RC_E_NOMEM, "host copy of the mock scene");
        if (nv > 0) memcpy(sc.host_verts, verts, sizeof(float) * 3 * nv);
        for (int64_t i = 0; i < 3 * nv; ++i) sc.host_sum += sc.host_verts[i];
        c->used += sc.bytes;
        sc.alive = true;
        int32_t id = -1;
        for (size_t i = 0; i < c->scenes.size(); ++i)
            if (!c->scenes[i].alive) { id = (int32_t)i; break; }
        if (id < 0) {
            id = (int32_t)c->scenes.size();
            c->scenes.push_back(sc);
        } else {
            c->scenes[id] = sc;
        }
        *out_scene = id;
        return RC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    Scene sc;
    sc.nv = nv;
    sc.nt = nt;
    rc_status st = dev_alloc(c, (void **)&sc.verts, sizeof(float) * 3 * nv);
    if (st == RC_OK) st = dev_alloc(c, (void **)&sc.tris, sizeof(int32_t) * 3 * nt);
    if (st == RC_OK) st = dev_alloc(c, (void **)&sc.box_dev, sizeof(float) * 8);
    if (st != RC_OK) {
        free_scene(c, sc);
        return st;
    }
    hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipSuccess;
    if (nv) e = hipMemcpyAsync(sc.verts, verts, sizeof(float) * 3 * nv, kind, s);
    if (e == hipSuccess && nt) e = hipMemcpyAsync(sc.tris, tris, sizeof(int32_t) * 3 * nt, kind, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->flags_dev, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = validate_mesh_launch(sc.verts, nv, sc.tris, nt, c->flags_dev, s);
    int32_t flags = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, c->flags_dev, sizeof(int32_t),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_scene(c, sc);
        return fail(RC_E_DEVICE, "scene upload failed: %s", hipGetErrorString(e));
    }
    if (flags) {
        free_scene(c, sc);
        return fail(RC_E_INVAL, "invalid mesh:%s%s", (flags & 1) ? " index out of range" : "",
                    (flags & 2) ? " non-finite vertex" : "");
    }
    sc.alive = true;
    sc.bytes = sizeof(float) * 3 * nv + sizeof(int32_t) * 3 * nt;
    int32_t id = -1;
    for (size_t i = 0; i < c->scenes.size(); ++i)
        if (!c->scenes[i].alive) { id = (int32_t)i; break; }
    if (id < 0) {
        id = (int32_t)c->scenes.size();
        c->scenes.push_back(sc);
    } else {
        c->scenes[id] = sc;
    }
    *out_scene = id;
    return RC_OK;
}

rc_status rc_lbvh_build(rc_ctx *c, int32_t scene, const rc_build_opts *opts, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    int bits = 10, fmt = RC_NODE_FP32;
    if (opts) {
        if (opts->morton_bits) bits = opts->morton_bits;
        fmt = opts->node_format;
    }
    if (bits < 1 || bits > 10) return fail(RC_E_INVAL, "morton_bits must be in 1..10");
    if (fmt != RC_NODE_FP32 && fmt != RC_NODE_Q8)
        return fail(RC_E_INVAL, "node format %d not supported", fmt);
    if (c->mock) {
        std::lock_guard<std::mutex> lk(c->mu);
        Scene *sc = get_scene(c, scene);
        if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
        sc->has_bvh = true;
        sc->morton_bits = bits;
        sc->node_format = fmt;
        return RC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    Scene *sc = get_scene(c, scene);
    if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
    const int64_t nt = sc->nt, ni = nt > 1 ? nt - 1 : 1;
    if (nt > 0 && !sc->nodes) {
        rc_status st = dev_alloc(c, (void **)&sc->morton, sizeof(uint32_t) * nt);
        if (st == RC_OK) st = dev_alloc(c, (void **)&sc->sorted, sizeof(uint32_t) * nt);
        if (st == RC_OK) st = dev_alloc(c, (void **)&sc->topo, sizeof(int32_t) * 3 * ni);
        if (st == RC_OK) st = dev_alloc(c, (void **)&sc->nodes, sizeof(NodeRec) * ni);
        if (st == RC_OK) st = dev_alloc(c, (void **)&sc->trirecs, sizeof(TriRec) * nt);
        if (st != RC_OK) {
            free_bvh(c, *sc);
            return st;
        }
        sc->bytes += scene_bvh_bytes(nt);
    }
    if (nt > 0 && fmt == RC_NODE_Q8 && !sc->q8nodes) {
        rc_status st = dev_alloc(c, (void **)&sc->q8nodes, sizeof(NodeRec) * ni);
        if (st != RC_OK) return st;
        sc->bytes += sizeof(NodeRec) * ni;
    }
    if (nt > 0) {
        rc_status st = ensure_build_ws(c, lbvh_workspace_bytes(nt), s);
        if (st != RC_OK) return st;
        BuildBuffers b;
        b.verts = sc->verts;
        b.tris = sc->tris;
        b.nv = sc->nv;
        b.nt = nt;
        b.morton_bits = bits;
        b.ws = c->ws;
        b.ws_bytes = c->ws_bytes;
        b.morton = sc->morton;
        b.sorted = sc->sorted;
        b.topo = sc->topo;
        b.nodes = sc->nodes;
        b.trirecs = sc->trirecs;
        b.scene_box = sc->box_dev;
        b.depth_out = reinterpret_cast<int32_t *>(sc->box_dev + 6);
        b.q8nodes = fmt == RC_NODE_Q8 ? sc->q8nodes : nullptr;
        b.q8_count = reinterpret_cast<uint32_t *>(sc->box_dev + 7);
        // the build's kernels read and write the scene: it stays referenced
        // until they have finished
        hold_scene(c, sc);
        std::vector<Scene *> held(1, sc);
        hipError_t e = lbvh_build_launch(b, s);
        if (e == hipSuccess) e = hipEventRecord(c->ws_event, s);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s);
            drop_holds(c, held.data(), 1);
            return fail(RC_E_DEVICE, "LBVH build failed: %s", hipGetErrorString(e));
        }
        c->ws_event_recorded = true;
        rc_status st2 = drop_after(c, s, held);
        if (st2 != RC_OK) return st2;
    }
    sc->has_bvh = true;
    sc->morton_bits = bits;
    sc->node_format = fmt;
    return RC_OK;
}

rc_status rc_scene_release(rc_ctx *c, int32_t scene)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (!c->mock) HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    Scene *sc = get_scene(c, scene);
    if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
    bool now = false;
    {
        std::lock_guard<std::mutex> rl(c->ref_mu);
        sc->dead = true;
        now = sc->refs == 0;
    }
    // in use: the last reference to go puts it on the reap list instead
    if (now) free_scene(c, *sc);
    return RC_OK;
}

rc_status rc_pattern_upload(rc_ctx *c, const float *dirs, int32_t n_beams, int32_t n_az_hint,
                            int32_t *out_pattern)
{
    if (!c || !out_pattern) return fail(RC_E_INVAL, "null context or out_pattern");
    if (n_beams < 1 || !dirs) return fail(RC_E_INVAL, "need n_beams >= 1 and a direction array");
    for (int32_t j = 0; j < n_beams; ++j) {
        const float *d = dirs + 3 * (int64_t)j;
        if (!isfinite(d[0]) || !isfinite(d[1]) || !isfinite(d[2]))
            return fail(RC_E_INVAL, "beam %d is not finite", j);
        if (d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f)
            return fail(RC_E_INVAL, "beam %d is the zero vector", j);
    }
    if (c->mock) {
        std::lock_guard<std::mutex> lk(c->mu);
        Pattern p;
        p.alive = true;
        p.n_beams = n_beams;
        p.n_az = n_az_hint > 0 ? n_az_hint : n_beams;
        c->patterns.push_back(p);
        *out_pattern = (int32_t)c->patterns.size() - 1;
        return RC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    Pattern p;
    p.n_beams = n_beams;
    p.n_az = n_az_hint > 0 ? n_az_hint : n_beams;
    p.bytes = sizeof(float) * 3 * (size_t)n_beams;
    rc_status st = dev_alloc(c, (void **)&p.dirs, p.bytes);
    if (st != RC_OK) return st;
    hipError_t e = hipMemcpy(p.dirs, dirs, p.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(c, p.dirs, p.bytes);
        return fail(RC_E_DEVICE, "pattern copy failed: %s", hipGetErrorString(e));
    }
    p.alive = true;
    int32_t id = -1;
    for (size_t i = 0; i < c->patterns.size(); ++i)
        if (!c->patterns[i].alive) { id = (int32_t)i; break; }
    if (id < 0) {
        id = (int32_t)c->patterns.size();
        c->patterns.push_back(p);
    } else {
        c->patterns[id] = p;
    }
    *out_pattern = id;
    return RC_OK;
}

rc_status rc_raycast_batch(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, float *out_range,
                           int32_t *out_hit, void *stream)
{
    return trace_common(c, TRACE_BVH, jobs, n_jobs, out_range, out_hit, nullptr, nullptr, stream);
}

rc_status rc_raycast_batch_noalloc(rc_ctx *c, const rc_job *jobs, int32_t n_jobs,
                                   float *out_range, int32_t *out_hit, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (c->mock) return fail(RC_E_STATE, "a mock context has no device to cast on");
    if (n_jobs < 0 || n_jobs > kNoAllocJobs)
        return fail(RC_E_INVAL,
                    "rc_raycast_batch_noalloc takes 0..%d jobs (%d given): its job table lives "
                    "in a fixed %zu-byte device array", kNoAllocJobs, (int)n_jobs, kScratchBytes);
    if (!c->scratch) return fail(RC_E_STATE, "no launch scratch on device %d", c->device);
    rc_tuning tuning;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        tuning = c->tuning;
    }
    DevJob dj[kNoAllocJobs];
    Scene *held[kNoAllocJobs];
    int n_run = 0;
    int64_t total = 0;
    int fmt = FMT_BINARY;
    rc_status st = prepare_jobs(c, tuning, jobs, n_jobs, dj, held, &n_run, total, fmt, nullptr);
    if (st == RC_OK && total > 0 && (!out_range || !out_hit)) st = fail(RC_E_INVAL, "null output");
    if (st == RC_OK && total > 0 && hipSetDevice(c->device) != hipSuccess)
        st = fail(RC_E_DEVICE, "hipSetDevice(%d) failed", c->device);
    DropRec *d = nullptr;
    if (st == RC_OK && total > 0) {
        std::lock_guard<std::mutex> lk(c->ref_mu);
        if (!c->drop_free.empty()) {
            d = &c->drop_pool[c->drop_free.back()];
            c->drop_free.pop_back();
        }
    }
    if (st == RC_OK && total > 0 && !d)
        st = fail(RC_E_BUSY, "%d launches of rc_raycast_batch_noalloc are still in flight",
                  kDropPool);
    if (st != RC_OK || total == 0) {
        drop_holds(c, held, (size_t)n_run);
        return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    WorkQueues q;
    init_queues(q, total);
    hipError_t e = hipSuccess;
    for (int first = 0; e == hipSuccess && first < n_run; first += kFillJobs) {
        ScratchFill a;
        a.first = first;
        a.count = n_run - first < kFillJobs ? n_run - first : kFillJobs;
        a.with_queues = first == 0;
        a.pad = 0;
        a.queues = q;
        memcpy(a.words, dj + first, sizeof(DevJob) * (size_t)a.count);
        hipLaunchKernelGGL(k_fill_scratch, dim3(1), dim3(64), 0, s, c->scratch, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = trace_launch(TRACE_BVH, fmt, config_of(tuning, dj, n_run),
                         reinterpret_cast<DevJob *>(c->scratch + sizeof(WorkQueues)), n_run,
                         reinterpret_cast<WorkQueues *>(c->scratch), total, out_range, out_hit,
                         nullptr, nullptr, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        drop_holds(c, held, (size_t)n_run);
        std::lock_guard<std::mutex> lk(c->ref_mu);
        c->drop_free.push_back(d->slot);
        return fail(RC_E_DEVICE, "traversal launch failed: %s", hipGetErrorString(e));
    }
    d->held.assign(held, held + n_run);   // within the reserved capacity
    return enqueue_drop(c, s, d);
}

rc_status rc_raycast_bruteforce(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, float *out_range,
                                int32_t *out_hit, void *stream)
{
    return trace_common(c, TRACE_BRUTE, jobs, n_jobs, out_range, out_hit, nullptr, nullptr,
                        stream);
}

rc_status rc_raycast_stats(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, float *out_range,
                           int32_t *out_hit, int32_t *out_nodes, int32_t *out_tris, void *stream)
{
    return trace_common(c, TRACE_STATS, jobs, n_jobs, out_range, out_hit, out_nodes, out_tris,
                        stream);
}

rc_status rc_scene_get_info(rc_ctx *c, int32_t scene, rc_scene_info *out)
{
    if (!c || !out) return fail(RC_E_INVAL, "null argument");
    if (c->mock) {
        std::lock_guard<std::mutex> lk(c->mu);
        Scene *sc = get_scene(c, scene);
        if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
        memset(out, 0, sizeof *out);
        out->n_verts = sc->nv;
        out->n_tris = sc->nt;
        out->has_bvh = sc->has_bvh ? 1 : 0;
        out->node_format = sc->node_format;
        out->morton_bits = sc->morton_bits;
        return RC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    Scene *sc = get_scene(c, scene);
    if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
    memset(out, 0, sizeof *out);
    out->n_verts = sc->nv;
    out->n_tris = sc->nt;
    out->n_nodes = sc->nt > 1 ? sc->nt - 1 : 0;
    out->node_format = sc->node_format;
    out->morton_bits = sc->morton_bits;
    out->has_bvh = sc->has_bvh ? 1 : 0;
    out->device_bytes = sc->bytes;
    if (sc->has_bvh && sc->nt > 0) {
        float hb[8];
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(hb, sc->box_dev, sizeof hb, hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a) {
            out->scene_lo[a] = hb[a];
            out->scene_hi[a] = hb[3 + a];
        }
        int32_t depth;
        memcpy(&depth, &hb[6], sizeof depth);
        out->depth = depth;
        uint32_t nq;
        memcpy(&nq, &hb[7], sizeof nq);
        out->n_q8_nodes = sc->node_format == RC_NODE_Q8 ? (sc->nt > 1 ? nq : 0) : 0;
    }
    return RC_OK;
}

rc_status rc_scene_debug_copy(rc_ctx *c, int32_t scene, int32_t what, void *dst, uint64_t bytes)
{
    if (!c || !dst) return fail(RC_E_INVAL, "null argument");
    if (c->mock) return fail(RC_E_STATE, "a mock context holds no device arrays");
    HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    Scene *sc = get_scene(c, scene);
    if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", scene);
    if (!sc->has_bvh) return fail(RC_E_STATE, "scene %d has no BVH", scene);
    const int64_t nt = sc->nt, ni = nt > 1 ? nt - 1 : 0;
    const void *src = nullptr;
    uint64_t size = 0;
    switch (what) {
    case RC_DBG_MORTON: src = sc->morton; size = 4ull * nt; break;
    case RC_DBG_SORTED: src = sc->sorted; size = 4ull * nt; break;
    case RC_DBG_TOPOLOGY: src = sc->topo; size = 12ull * ni; break;
    case RC_DBG_NODES: src = sc->nodes; size = sizeof(NodeRec) * (uint64_t)ni; break;
    case RC_DBG_TRIS: src = sc->trirecs; size = sizeof(TriRec) * (uint64_t)nt; break;
    case RC_DBG_Q8NODES:
        if (sc->node_format != RC_NODE_Q8) return fail(RC_E_STATE, "scene %d has no Q8 nodes", scene);
        src = sc->q8nodes;
        size = sizeof(NodeRec) * (uint64_t)ni;
        break;
    default: return fail(RC_E_INVAL, "unknown debug array %d", what);
    }
    if (bytes != size)
        return fail(RC_E_INVAL, "array %d holds %llu bytes, %llu requested", what,
                    (unsigned long long)size, (unsigned long long)bytes);
    if (size == 0) return RC_OK;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(dst, src, size, hipMemcpyDeviceToHost));
    return RC_OK;
}

uint64_t rc_device_bytes(rc_ctx *c)
{
    if (!c) return 0;
    if (!c->mock) (void)hipSetDevice(c->device);
    std::lock_guard<std::mutex> lk(c->mu);
    reap_locked(c);
    return c->used;
}

rc_status rc_set_tuning(rc_ctx *c, const rc_tuning *t)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (!t) {
        std::lock_guard<std::mutex> lk(c->job_mu);
        c->tuning = default_tuning();
        return RC_OK;
    }
    rc_status st = check_tuning(t);
    if (st != RC_OK) return st;
    std::lock_guard<std::mutex> lk(c->job_mu);
    c->tuning = *t;
    return RC_OK;
}

}  // extern "C"

namespace rc {

rc_status check_tuning(const rc_tuning *t)
{
    if (t->persistent != 0 && t->persistent != 1) return fail(RC_E_INVAL, "persistent must be 0 or 1");
    if (t->persistent && t->stack_lds != 8 && t->stack_lds != 16 && t->stack_lds != 24)
        return fail(RC_E_INVAL, "persistent traversal needs stack_lds in {8, 16, 24}");
    if (!t->persistent && t->stack_lds != 0 && t->stack_lds != 8 && t->stack_lds != 16)
        return fail(RC_E_INVAL, "one-ray-per-thread traversal needs stack_lds in {0, 8, 16}");
    if (t->chunk_max != 0 && (t->chunk_max < 64 || t->chunk_max > (1 << 20)))
        return fail(RC_E_INVAL, "chunk_max must be 0 or 64..2^20");
    if (t->waves_cap != 0 && t->waves_cap != 1) return fail(RC_E_INVAL, "waves_cap must be 0 or 1");
    if (t->group_waves != 1 && t->group_waves != 4) return fail(RC_E_INVAL, "group_waves must be 1 or 4");
    if (t->leaf_batch < 0 || t->leaf_batch > 64) return fail(RC_E_INVAL, "leaf_batch must be 0..64");
    if (t->refill_min < 1 || t->refill_min > 64) return fail(RC_E_INVAL, "refill_min must be 1..64");
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return fail(RC_E_INVAL, "blocks_per_cu must be 0..64");
    if (t->tile_az < 0 || t->tile_el < 0 || (int64_t)t->tile_az * t->tile_el > (1 << 20))
        return fail(RC_E_INVAL, "bad tile shape");
    return RC_OK;
}

// Candidate launch shapes for the autotuner (all give identical results).
std::vector<rc_tuning> tuning_candidates()
{
    std::vector<rc_tuning> v;
    const int tiles[4][2] = {{16, 4}, {8, 8}, {32, 2}, {0, 0}};
    for (int gw : {1, 4})
        for (int ss : {0, 8})
            for (int cap : {1, 0})
                for (auto &tl : tiles) {
                    if (gw == 4 && tl[0] != 16 && tl[0] != 0) continue;
                    rc_tuning t = default_tuning();
                    t.persistent = 0;
                    t.stack_lds = ss;
                    t.waves_cap = cap;
                    t.tile_az = tl[0];
                    t.tile_el = tl[1];
                    t.group_waves = gw;
                    v.push_back(t);
                }
    // queued leaf tests (Q8 trees; ignored on plain trees, where these
    // candidates repeat the first ones)
    for (int lb : {16, 32, 64})
        for (int gw : {1, 4}) {
            rc_tuning t = default_tuning();
            t.leaf_batch = lb;
            t.group_waves = gw;
            v.push_back(t);
        }
    for (int ss : {8, 16})
        for (int rm : {48, 64})
            for (int b : {2, 4}) {
                rc_tuning t = default_tuning();
                t.persistent = 1;
                t.stack_lds = ss;
                t.refill_min = rm;
                t.blocks_per_cu = b;
                t.waves_cap = 0;
                t.chunk_max = 1024;
                v.push_back(t);
            }
    return v;
}

}  // namespace rc

namespace rc {

int log2_class(int64_t n)
{
    int k = 0;
    while (n > 1) { n >>= 1; ++k; }
    return k;
}

// Cache key of a batch (see rc_tuning_cache_load): device, node format,
// size class of the largest scene, pattern shape, ray and job-count classes.
rc_status tune_key(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, std::string *key)
{
    if (n_jobs < 1 || !jobs) return fail(RC_E_INVAL, "bad job list");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, c->device));
    int64_t max_tris = 0, rays = 0;
    int fmt = -1;
    int32_t n_beams = -1, n_az = -1;
    bool mixed = false;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (int32_t i = 0; i < n_jobs; ++i) {
            Scene *sc = get_scene(c, jobs[i].scene);
            Pattern *pt = get_pattern(c, jobs[i].pattern);
            if (!sc || !pt) return fail(RC_E_NOTFOUND, "job %d: unknown scene or pattern", i);
            if (sc->nt > max_tris) max_tris = sc->nt;
            const int f = sc->node_format;
            fmt = fmt < 0 ? f : (fmt == f ? fmt : 2);
            const int32_t na = pt->n_az > 0 ? pt->n_az : pt->n_beams;
            if (n_beams < 0) { n_beams = pt->n_beams; n_az = na; }
            else if (n_beams != pt->n_beams || n_az != na) mixed = true;
            rays += (int64_t)jobs[i].n_envs * pt->n_beams;
        }
    }
    char buf[256];
    char pat[64];
    if (mixed) snprintf(pat, sizeof pat, "mixed");
    else snprintf(pat, sizeof pat, "%dx%d", n_beams / (n_az > 0 ? n_az : 1), n_az);
    snprintf(buf, sizeof buf, "%s:%dcu|fmt%d|tris2^%d|pat%s|rays2^%d|jobs2^%d",
             prop.gcnArchName, prop.multiProcessorCount, fmt, log2_class(max_tris), pat,
             log2_class(rays), log2_class(n_jobs));
    for (char *p = buf; *p; ++p)
        if (*p == ' ' || *p == '\t' || *p == '\n') *p = '_';
    *key = buf;
    return RC_OK;
}

constexpr const char *kTuneCacheHeader = "rcast-tuning-cache v2";
constexpr const char *kTuneCacheHeaderV1 = "rcast-tuning-cache v1";  // no leaf_batch column

}  // namespace rc

extern "C" {

rc_status rc_tuning_cache_load(rc_ctx *c, const char *path)
{
    if (!c || !path) return fail(RC_E_INVAL, "null argument");
    std::map<std::string, rc_tuning> entries;
    FILE *f = fopen(path, "r");
    if (f) {
        char line[1024];
        int ln = 0, fields = 11;
        rc_status st = RC_OK;
        while (st == RC_OK && fgets(line, sizeof line, f)) {
            ++ln;
            if (ln == 1) {
                if (strncmp(line, kTuneCacheHeader, strlen(kTuneCacheHeader)) == 0)
                    fields = 11;
                else if (strncmp(line, kTuneCacheHeaderV1, strlen(kTuneCacheHeaderV1)) == 0)
                    fields = 10;
                else
                    st = fail(RC_E_INVAL, "%s: not a tuning cache (first line)", path);
                continue;
            }
            if (line[0] == '\n' || line[0] == '#') continue;
            char key[512];
            rc_tuning t;
            memset(&t, 0, sizeof t);
            const int n = sscanf(line, "%511s %d %d %d %d %d %d %d %d %d %d", key, &t.persistent,
                                 &t.stack_lds, &t.refill_min, &t.blocks_per_cu, &t.tile_az,
                                 &t.tile_el, &t.chunk_max, &t.waves_cap, &t.group_waves,
                                 &t.leaf_batch);
            if (n != fields) {
                st = fail(RC_E_INVAL, "%s:%d: malformed entry", path, ln);
                break;
            }
            if (check_tuning(&t) != RC_OK) {
                st = fail(RC_E_INVAL, "%s:%d: tuning out of range", path, ln);
                break;
            }
            entries[key] = t;
        }
        if (st == RC_OK && ferror(f)) st = fail(RC_E_DEVICE, "%s: read error", path);
        fclose(f);
        if (st != RC_OK) return st;
    } else if (errno != ENOENT) {
        return fail(RC_E_DEVICE, "%s: cannot open (%s)", path, strerror(errno));
    }
    std::lock_guard<std::mutex> lk(c->job_mu);
    for (auto &kv : entries) c->tune_cache[kv.first] = kv.second;
    c->tune_cache_on = true;
    return RC_OK;
}

rc_status rc_tuning_cache_save(rc_ctx *c, const char *path)
{
    if (!c || !path) return fail(RC_E_INVAL, "null argument");
    std::map<std::string, rc_tuning> entries;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        entries = c->tune_cache;
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(RC_E_DEVICE, "%s: cannot create (%s)", tmp.c_str(), strerror(errno));
    bool ok = fprintf(f, "%s\n", kTuneCacheHeader) > 0;
    for (auto &kv : entries) {
        const rc_tuning &t = kv.second;
        ok = ok && fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d\n", kv.first.c_str(),
                           t.persistent, t.stack_lds, t.refill_min, t.blocks_per_cu, t.tile_az,
                           t.tile_el, t.chunk_max, t.waves_cap, t.group_waves,
                           t.leaf_batch) > 0;
    }
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(RC_E_DEVICE, "%s: write failed", path);
    }
    return RC_OK;
}

rc_status rc_autotune(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, float *out_range,
                      int32_t *out_hit, void *stream, int32_t reps, rc_tuning *out_best,
                      float *out_ms)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (c->mock) return fail(RC_E_STATE, "a mock context has no device to tune");
    if (reps < 1) reps = 1;
    HIP_TRY(hipSetDevice(c->device));
    bool use_cache;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        use_cache = c->tune_cache_on;
    }
    std::string key;
    if (use_cache) {
        rc_status st = tune_key(c, jobs, n_jobs, &key);
        if (st != RC_OK) return st;
        std::lock_guard<std::mutex> lk(c->job_mu);
        auto it = c->tune_cache.find(key);
        if (it != c->tune_cache.end()) {
            c->tuning = it->second;
            if (out_best) *out_best = it->second;
            if (out_ms) *out_ms = -1.0f;
            return RC_OK;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    rc_tuning best = default_tuning();
    float best_ms = INFINITY;
    rc_status result = RC_OK;
    for (const rc_tuning &cand : tuning_candidates()) {
        // warm-up, then the fastest of `reps` timed launches
        rc_status st = trace_common(c, TRACE_BVH, jobs, n_jobs, out_range, out_hit, nullptr,
                                    nullptr, stream, &cand);
        if (st != RC_OK) { result = st; break; }
        float ms = INFINITY;
        for (int r = 0; r < reps && st == RC_OK; ++r) {
            hipError_t e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                st = trace_common(c, TRACE_BVH, jobs, n_jobs, out_range, out_hit, nullptr,
                                  nullptr, stream, &cand);
            if (e == hipSuccess && st == RC_OK) e = hipEventRecord(e1, s);
            if (e == hipSuccess && st == RC_OK) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess && st == RC_OK) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) st = fail(RC_E_DEVICE, "autotune timing failed: %s", hipGetErrorString(e));
            if (st == RC_OK && t < ms) ms = t;
        }
        if (st != RC_OK) { result = st; break; }
        if (ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != RC_OK) return result;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        c->tuning = best;
        if (use_cache) c->tune_cache[key] = best;
    }
    if (out_best) *out_best = best;
    if (out_ms) *out_ms = best_ms;
    return RC_OK;
}

rc_status rc_get_tuning(rc_ctx *c, rc_tuning *t)
{
    if (!c || !t) return fail(RC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(c->job_mu);
    *t = c->tuning;
    return RC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Captured launches.

struct rc_graph {
    rc_ctx *ctx = nullptr;
    std::vector<Scene *> held;   // the graph's scenes, referenced until it is destroyed
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    char *dev = nullptr;
    size_t bytes = 0;
    int64_t rays = 0;
};

extern "C" {

rc_status rc_graph_create(rc_ctx *c, const rc_job *jobs, int32_t n_jobs, float *out_range,
                          int32_t *out_hit, rc_graph **out)
{
    if (!c || !out) return fail(RC_E_INVAL, "null argument");
    *out = nullptr;
    if (c->mock) return fail(RC_E_STATE, "a mock context cannot capture launches");
    rc_tuning tuning;
    {
        std::lock_guard<std::mutex> lk(c->job_mu);
        tuning = c->tuning;
    }
    const size_t cap = n_jobs > 0 ? (size_t)n_jobs : 0;
    std::vector<DevJob> dj(cap);
    std::vector<Scene *> held(cap);
    int n_run = 0;
    int64_t total = 0;
    int fmt = FMT_BINARY;
    rc_status st = prepare_jobs(c, tuning, jobs, n_jobs, dj.data(), held.data(), &n_run, total,
                                fmt, nullptr);
    held.resize(n_run);
    dj.resize(n_run);
    if (st == RC_OK && total > 0 && (!out_range || !out_hit))
        st = fail(RC_E_INVAL, "null output");
    if (st == RC_OK && hipSetDevice(c->device) != hipSuccess)
        st = fail(RC_E_DEVICE, "hipSetDevice(%d) failed", c->device);
    if (st != RC_OK) {
        drop_holds(c, held.data(), held.size());
        return st;
    }
    rc_graph *g = new rc_graph();
    g->ctx = c;
    g->held.swap(held);
    g->rays = total;
    const size_t nj = dj.empty() ? 1 : dj.size();
    g->bytes = sizeof(DevJob) * nj + 2 * sizeof(WorkQueues);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        st = dev_alloc(c, (void **)&g->dev, g->bytes);
    }
    if (st != RC_OK) {
        drop_holds(c, g->held.data(), g->held.size());
        delete g;
        return st;
    }
    std::vector<char> host(g->bytes, 0);
    memcpy(host.data(), dj.data(), sizeof(DevJob) * dj.size());
    WorkQueues init;
    init_queues(init, total);
    memcpy(host.data() + sizeof(DevJob) * nj + sizeof(WorkQueues), &init, sizeof init);
    DevJob *djd = reinterpret_cast<DevJob *>(g->dev);
    WorkQueues *live = reinterpret_cast<WorkQueues *>(g->dev + sizeof(DevJob) * nj);
    WorkQueues *tmpl = live + 1;
    hipError_t e = hipMemcpy(g->dev, host.data(), g->bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && total > 0) {
        e = queue_reset_launch(live, tmpl, g->cap);
        if (e == hipSuccess)
            e = trace_launch(TRACE_BVH, fmt, config_of(tuning, dj.data(), n_run), djd, n_run, live,
                             total,
                             out_range, out_hit, nullptr, nullptr, g->cap);
        if (e != hipSuccess) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(g->cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
        }
    }
    if (e == hipSuccess) e = hipStreamEndCapture(g->cap, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        rc_graph_destroy(g);
        return fail(RC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return RC_OK;
}

rc_status rc_graph_launch(rc_graph *g, void *stream)
{
    if (!g) return fail(RC_E_INVAL, "null graph");
    HIP_TRY(hipSetDevice(g->ctx->device));
    HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return RC_OK;
}

void rc_graph_destroy(rc_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    drop_holds(g->ctx, g->held.data(), g->held.size());
    {
        std::lock_guard<std::mutex> lk(g->ctx->mu);
        if (g->dev) dev_free(g->ctx, g->dev, g->bytes);
        reap_locked(g->ctx);
    }
    delete g;
}

}  // extern "C"
