// serve.hip -- continuous-batching request server of librcast.
//
// Requests (one scene, one beam pattern, n_envs host poses, a range
// interval) arrive through rc_serve_submit from any thread.  A scheduler
// thread admits them in arrival order while their memory footprint fits in
// the server's arenas -- outputs (8 bytes per ray: range + hit) and poses --
// and folds every request admitted at that moment into ONE batched launch
// (a job table over several scenes and patterns).  Up to `max_inflight`
// launches run at once on separate streams, so requests arriving while
// others are on the GPU start as soon as a launch slot and memory are free
// (continuous batching, not a queue in front of one launch).  Completion is
// signalled by a host function enqueued behind each launch; results stay in
// the arena until the caller releases the ticket.  A request's results are
// independent of what it was batched with: every ray is a pure function of
// its own inputs.
//
// A mock context (device RC_DEVICE_MOCK) runs the same scheduler against a
// host-thread "device" that sleeps in proportion to the rays and writes a
// recognisable pattern, so admission, batching, ticket life cycle and
// failure isolation are testable without a GPU.
#include "ctx.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

namespace rc {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) in abstract units; coalesces on free.
class Arena {
public:
    void init(uint64_t size)
    {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        in_use_ = 0;
    }
    bool alloc(uint64_t n, uint64_t *off)
    {
        if (n == 0) n = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const uint64_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            in_use_ += n;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        if (n == 0) n = 1;
        in_use_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    uint64_t size() const { return size_; }
    uint64_t in_use() const { return in_use_; }

private:
    uint64_t size_ = 0, in_use_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

enum ReqState { REQ_PENDING = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_FAILED = 3 };

struct Batch;

struct Request {
    uint64_t ticket = 0;
    rc_request req{};
    int64_t n_rays = 0;
    std::vector<float> poses;
    int state = REQ_PENDING;
    rc_status status = RC_OK;
    std::string error;
    Clock::time_point t_submit, t_done;
    uint64_t out_off = 0;     // in rays
    uint64_t pose_off = 0;    // in floats
    bool has_mem = false;
};

struct Batch {
    ServeState *S = nullptr;
    std::vector<Request *> reqs;
    int stream = 0;
    // mock device: each request's referenced scene and, like the pointers of
    // a device job table, its memory as resolved when the batch was formed
    struct MockJob {
        Scene *sc = nullptr;
        const float *verts = nullptr;
        int64_t nv = 0;
        double sum = 0.0;
    };
    std::vector<MockJob> mock;
};

struct ServeState {
    rc_ctx *ctx = nullptr;
    rc_serve_opts opts{};
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> tickets;
    uint64_t next_ticket = 1;
    uint64_t generation = 0;   // bumps whenever arena memory is returned
    Arena out_arena, pose_arena;
    float *range_buf = nullptr;
    int32_t *hit_buf = nullptr;
    float *pose_buf = nullptr;
    uint64_t range_bytes = 0, pose_bytes = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_busy;
    std::vector<StageBuf> stage;   // job table per stream
    int inflight = 0;
    rc_serve_stats stats{};
    // mock device: one simulated execution queue per stream, so launches on
    // different streams overlap as kernels on a GPU do
    std::vector<std::thread> mock_threads;
    std::vector<std::deque<Batch *>> mock_queue;
    std::condition_variable mock_cv;
    bool mock_stop = false;   // set only after the scheduler thread has exited
};

namespace {

void update_peaks(ServeState &S)
{
    const uint64_t bytes = S.out_arena.in_use() * 8 + S.pose_arena.in_use() * 4;
    S.stats.bytes_in_use = bytes;
    if (bytes > S.stats.peak_bytes) S.stats.peak_bytes = bytes;
    if ((uint64_t)S.inflight > S.stats.peak_inflight) S.stats.peak_inflight = S.inflight;
}

void free_request_memory(ServeState &S, Request *r)
{
    if (!r->has_mem) return;
    S.out_arena.release(r->out_off, (uint64_t)r->n_rays);
    S.pose_arena.release(r->pose_off, (uint64_t)r->req.n_envs * 12);
    r->has_mem = false;
    ++S.generation;
    update_peaks(S);
}

// Called (under S.mu) when a batch has finished on the device.
void complete_batch_locked(ServeState &S, Batch *b)
{
    const auto now = Clock::now();
    for (Request *r : b->reqs) {
        if (r->state == REQ_RUNNING) {
            r->state = REQ_DONE;
            r->t_done = now;
            ++S.stats.completed;
        }
    }
    S.stream_busy[b->stream] = 0;
    --S.inflight;
    delete b;
    S.cv.notify_all();
}

void on_device_done(void *arg)
{
    Batch *b = static_cast<Batch *>(arg);
    ServeState &S = *b->S;
    std::lock_guard<std::mutex> lk(S.mu);
    complete_batch_locked(S, b);
}

void fail_request_locked(ServeState &S, Request *r, rc_status st, const std::string &msg)
{
    r->state = REQ_FAILED;
    r->status = st;
    r->error = msg;
    r->t_done = Clock::now();
    ++S.stats.failed;
}

// Simulated device queue of one stream: launches in order, each taking
// mock_ns_per_ray per ray.
void mock_loop(ServeState *Sp, int q)
{
    ServeState &S = *Sp;
    std::unique_lock<std::mutex> lk(S.mu);
    while (true) {
        S.mock_cv.wait(lk, [&] { return S.mock_stop || !S.mock_queue[q].empty(); });
        if (S.mock_queue[q].empty()) {
            if (S.mock_stop) return;
            continue;
        }
        Batch *b = S.mock_queue[q].front();
        S.mock_queue[q].pop_front();
        int64_t rays = 0;
        for (Request *r : b->reqs) rays += r->n_rays;
        const int64_t ns = rays * (int64_t)S.opts.mock_ns_per_ray;
        lk.unlock();
        if (ns > 0) std::this_thread::sleep_for(std::chrono::nanoseconds(ns));
        // "kernel": read each request's scene memory, which must still be the
        // uploaded vertices (a scene released meanwhile is only freed after
        // this batch has dropped its references)
        std::vector<char> intact(b->reqs.size(), 1);
        for (size_t i = 0; i < b->reqs.size(); ++i) {
            const Batch::MockJob &m = b->mock[i];
            double sum = 0.0;
            for (int64_t k = 0; k < 3 * m.nv; ++k) sum += m.verts[k];
            intact[i] = sum == m.sum;
        }
        // the "kernel" has finished: drop the batch's scene references
        // before its requests complete, as the device path's stream order
        // does (c->mu is taken without S.mu)
        {
            std::vector<Scene *> held;
            for (const Batch::MockJob &m : b->mock) held.push_back(m.sc);
            rc_ctx *c = S.ctx;
            drop_holds(c, held.data(), held.size());
            std::lock_guard<std::mutex> clk(c->mu);
            reap_locked(c);
        }
        lk.lock();
        for (size_t i = 0; i < b->reqs.size(); ++i) {
            Request *r = b->reqs[i];
            if (r->state != REQ_RUNNING) continue;
            if (!intact[i]) {
                fail_request_locked(S, r, RC_E_DEVICE, "scene memory changed during the launch");
                continue;
            }
            if (r->req.scene + 1 == S.opts.mock_fail_scene) {
                fail_request_locked(S, r, RC_E_DEVICE, "simulated device error");
                continue;
            }
            for (int64_t k = 0; k < r->n_rays; ++k) {
                S.range_buf[r->out_off + k] = (float)k;
                S.hit_buf[r->out_off + k] = r->req.scene;
            }
        }
        complete_batch_locked(S, b);
    }
}

// Launch one admitted batch (S.mu NOT held).  Returns false on failure,
// with every request of the batch marked failed by the caller.
rc_status launch_batch(ServeState &S, Batch *b, std::string &err)
{
    rc_ctx *c = S.ctx;
    // a request whose scene or pattern has gone since it was submitted fails
    // on its own; the rest of the batch proceeds.  The scenes of the others
    // are referenced in the same step (under c->mu), so a release from now on
    // defers its free until the launch has finished.
    if (c->mock) {
        std::vector<Request *> gone, kept;
        {
            std::lock_guard<std::mutex> clk(c->mu);
            for (Request *r : b->reqs) {
                Scene *sc = get_scene(c, r->req.scene);
                Pattern *pt = get_pattern(c, r->req.pattern);
                if (!sc || !pt || (sc->nt > 0 && !sc->has_bvh)) {
                    gone.push_back(r);
                    continue;
                }
                hold_scene(c, sc);
                Batch::MockJob m;
                m.sc = sc;
                m.verts = sc->host_verts;
                m.nv = sc->nv;
                m.sum = sc->host_sum;
                b->mock.push_back(m);
                kept.push_back(r);
                memcpy(S.pose_buf + r->pose_off, r->poses.data(), r->poses.size() * sizeof(float));
            }
        }
        if (S.opts.mock_launch_delay_us > 0)   // the window between resolution and launch
            std::this_thread::sleep_for(std::chrono::microseconds(S.opts.mock_launch_delay_us));
        std::lock_guard<std::mutex> lk(S.mu);
        // a failed request leaves the batch: its caller may release it at once
        b->reqs.swap(kept);
        for (Request *r : gone)
            fail_request_locked(S, r, RC_E_NOTFOUND, "scene or pattern no longer usable");
        S.mock_queue[b->stream].push_back(b);
        S.mock_cv.notify_all();
        return RC_OK;
    }
    hipStream_t s = S.streams[b->stream];
    const std::vector<Request *> ok = b->reqs;
    std::vector<rc_job> jobs(ok.size());
    for (size_t i = 0; i < ok.size(); ++i) {
        Request *r = ok[i];
        hipError_t e = hipMemcpyAsync(S.pose_buf + r->pose_off, r->poses.data(),
                                      r->poses.size() * sizeof(float), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return RC_E_DEVICE;
        }
        rc_job &j = jobs[i];
        j.scene = r->req.scene;
        j.pattern = r->req.pattern;
        j.n_envs = r->req.n_envs;
        j.reserved0 = 0;
        j.poses_3x4 = S.pose_buf + r->pose_off;
        j.t_min = r->req.t_min;
        j.t_max = r->req.t_max;
        j.out_offset = (int64_t)r->out_off;
    }
    rc_status st = RC_OK;
    std::vector<int> skipped;
    if (!jobs.empty())
        st = trace_common(c, TRACE_BVH, jobs.data(), (int32_t)jobs.size(), S.range_buf, S.hit_buf,
                          nullptr, nullptr, s, nullptr, &S.stage[b->stream], &skipped);
    if (st != RC_OK) {
        err = rc_last_error();
        return st;
    }
    if (!skipped.empty()) {
        // failed requests leave the batch before its completion function is
        // enqueued: their callers may release them at once
        std::lock_guard<std::mutex> lk(S.mu);
        std::vector<char> drop(b->reqs.size(), 0);
        for (int i : skipped) {
            fail_request_locked(S, b->reqs[i], RC_E_NOTFOUND, "scene or pattern no longer usable");
            drop[i] = 1;
        }
        size_t k = 0;
        for (size_t i = 0; i < b->reqs.size(); ++i)
            if (!drop[i]) b->reqs[k++] = b->reqs[i];
        b->reqs.resize(k);
    }
    hipError_t e = hipLaunchHostFunc(s, on_device_done, b);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return RC_E_DEVICE;
    }
    return RC_OK;
}

void worker_loop(ServeState *Sp)
{
    ServeState &S = *Sp;
    if (!S.ctx->mock) (void)hipSetDevice(S.ctx->device);
    std::unique_lock<std::mutex> lk(S.mu);
    while (!S.stop) {
        S.cv.wait(lk, [&] {
            return S.stop || (!S.pending.empty() && S.inflight < S.opts.max_inflight);
        });
        if (S.stop) break;
        if (!S.ctx->mock) {
            // free scenes released while their batches ran (not under S.mu)
            lk.unlock();
            {
                std::lock_guard<std::mutex> clk(S.ctx->mu);
                reap_locked(S.ctx);
            }
            lk.lock();
            if (S.stop) break;
            if (S.pending.empty() || S.inflight >= S.opts.max_inflight) continue;
        }
        Batch *b = new Batch();
        b->S = &S;
        int64_t rays = 0;
        const int64_t cap = (int64_t)S.opts.max_batch_rays_m * 1000000;
        // admission order: arrival order (policy 0), or requests queued
        // longer than max_wait_ms in arrival order followed by the younger
        // ones by ray count (policy 1)
        std::vector<Request *> order(S.pending.begin(), S.pending.end());
        size_t n_old = order.size();
        if (S.opts.policy == 1) {
            const auto now = Clock::now();
            const auto limit = std::chrono::milliseconds(S.opts.max_wait_ms);
            auto young = std::stable_partition(order.begin(), order.end(), [&](Request *r) {
                return now - r->t_submit >= limit;
            });
            n_old = (size_t)(young - order.begin());
            std::stable_sort(young, order.end(),
                             [](Request *a, Request *c2) { return a->n_rays < c2->n_rays; });
        }
        bool any = false;
        for (size_t k = 0; k < order.size(); ++k) {
            Request *r = order[k];
            const bool in_order = k < n_old;   // may not be overtaken
            bool fits = !(cap > 0 && !b->reqs.empty() && rays + r->n_rays > cap);
            uint64_t oo = 0, po = 0;
            if (fits && !S.out_arena.alloc((uint64_t)r->n_rays, &oo)) fits = false;
            if (fits && !S.pose_arena.alloc((uint64_t)r->req.n_envs * 12, &po)) {
                S.out_arena.release(oo, (uint64_t)r->n_rays);
                fits = false;
            }
            if (!fits) {
                if (in_order) break;   // nothing behind it may go first
                continue;              // a smaller young request may still fit
            }
            r->out_off = oo;
            r->pose_off = po;
            r->has_mem = true;
            r->state = REQ_RUNNING;
            b->reqs.push_back(r);
            any = true;
            rays += r->n_rays;
        }
        if (any) {
            // drop the admitted (now running) requests from the queue,
            // keeping the order of the rest
            std::deque<Request *> rest;
            for (Request *r : S.pending)
                if (r->state == REQ_PENDING) rest.push_back(r);
            S.pending.swap(rest);
        }
        if (b->reqs.empty()) {
            delete b;
            // nothing fits yet: wait until memory is returned or (for the
            // small-first order) a new request arrives
            const uint64_t gen = S.generation, sub = S.stats.submitted;
            S.cv.wait(lk, [&] {
                return S.stop || S.generation != gen || S.pending.empty() ||
                       (S.opts.policy == 1 && S.stats.submitted != sub);
            });
            continue;
        }
        int si = 0;
        while (S.stream_busy[si]) ++si;   // inflight < max_inflight: one is free
        S.stream_busy[si] = 1;
        b->stream = si;
        ++S.inflight;
        ++S.stats.launches;
        if (b->reqs.size() > S.stats.max_batch_requests) S.stats.max_batch_requests = b->reqs.size();
        update_peaks(S);
        lk.unlock();
        std::string err;
        rc_status st = launch_batch(S, b, err);
        // a failed launch may have left copies from this stream's staging
        // in flight: let them drain before the stream is handed out again
        if (st != RC_OK && !S.ctx->mock) (void)hipStreamSynchronize(S.streams[si]);
        lk.lock();
        if (st != RC_OK) {
            for (Request *r : b->reqs)
                if (r->state == REQ_RUNNING) fail_request_locked(S, r, st, err);
            S.stream_busy[si] = 0;
            --S.inflight;
            delete b;
            S.cv.notify_all();
        }
    }
}

}  // namespace

void serve_shutdown(rc_ctx *c)
{
    ServeState *S = c->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    // no launch can be issued any more; drain: the simulated device empties
    // its queues before returning, real launches finish (and their
    // completion callbacks run) on their streams
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->mock_stop = true;
        S->mock_cv.notify_all();
    }
    for (std::thread &t : S->mock_threads)
        if (t.joinable()) t.join();
    for (hipStream_t s : S->streams) (void)hipStreamSynchronize(s);
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->inflight == 0; });
    }
    for (auto &kv : S->tickets) delete kv.second;
    if (c->mock) {
        free(S->range_buf);
        free(S->hit_buf);
        free(S->pose_buf);
    } else {
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
        for (StageBuf &b : S->stage) stage_free(c, b);
        std::lock_guard<std::mutex> lk(c->mu);
        dev_free(c, S->range_buf, S->range_bytes);
        dev_free(c, S->hit_buf, S->range_bytes);
        dev_free(c, S->pose_buf, S->pose_bytes);
    }
    delete S;
    c->serve = nullptr;
}

}  // namespace rc

using namespace rc;

extern "C" {

rc_status rc_serve_start(rc_ctx *c, const rc_serve_opts *opts)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (c->serve) return fail(RC_E_STATE, "server already running");
    rc_serve_opts o{};
    if (opts) o = *opts;
    if (o.arena_bytes == 0) o.arena_bytes = 4ull << 30;
    if (o.max_inflight == 0) o.max_inflight = 2;
    if (o.max_inflight < 1 || o.max_inflight > 8) return fail(RC_E_INVAL, "max_inflight must be 1..8");
    if (o.max_batch_rays_m < 0) return fail(RC_E_INVAL, "max_batch_rays_m < 0");
    if (o.mock_ns_per_ray < 0) return fail(RC_E_INVAL, "mock_ns_per_ray < 0");
    if (o.arena_bytes < (1u << 20)) return fail(RC_E_INVAL, "arena_bytes must be >= 1 MiB");
    if (o.policy != 0 && o.policy != 1) return fail(RC_E_INVAL, "policy must be 0 or 1");
    if (o.max_wait_ms < 0) return fail(RC_E_INVAL, "max_wait_ms < 0");
    if (o.mock_launch_delay_us < 0) return fail(RC_E_INVAL, "mock_launch_delay_us < 0");
    if (o.max_wait_ms == 0) o.max_wait_ms = 200;
    ServeState *S = new ServeState();
    S->ctx = c;
    S->opts = o;
    // poses take 1/64 of the arena (>= 256 KiB), outputs the rest
    S->pose_bytes = o.arena_bytes / 64 < (256u << 10) ? (256u << 10) : o.arena_bytes / 64;
    const uint64_t out_rays = (o.arena_bytes - S->pose_bytes) / 8;
    S->range_bytes = out_rays * 4;
    S->out_arena.init(out_rays);
    S->pose_arena.init(S->pose_bytes / 4);
    rc_status st = RC_OK;
    if (c->mock) {
        S->range_buf = static_cast<float *>(malloc(S->range_bytes));
        S->hit_buf = static_cast<int32_t *>(malloc(S->range_bytes));
        S->pose_buf = static_cast<float *>(malloc(S->pose_bytes));
        if (!S->range_buf || !S->hit_buf || !S->pose_buf) st = fail(RC_E_NOMEM, "host arena");
    } else {
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) st = fail(RC_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(c->mu);
        if (st == RC_OK) st = dev_alloc(c, (void **)&S->range_buf, S->range_bytes);
        if (st == RC_OK) st = dev_alloc(c, (void **)&S->hit_buf, S->range_bytes);
        if (st == RC_OK) st = dev_alloc(c, (void **)&S->pose_buf, S->pose_bytes);
        for (int i = 0; st == RC_OK && i < o.max_inflight; ++i) {
            hipStream_t s = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e != hipSuccess) st = fail(RC_E_DEVICE, "stream: %s", hipGetErrorString(e));
            else S->streams.push_back(s);
        }
    }
    if (st != RC_OK) {
        if (c->mock) {
            free(S->range_buf);
            free(S->hit_buf);
            free(S->pose_buf);
        } else {
            for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
            std::lock_guard<std::mutex> lk(c->mu);
            dev_free(c, S->range_buf, S->range_bytes);
            dev_free(c, S->hit_buf, S->range_bytes);
            dev_free(c, S->pose_buf, S->pose_bytes);
        }
        delete S;
        return st;
    }
    S->stream_busy.assign(o.max_inflight, 0);
    S->stage.resize(o.max_inflight);
    S->stats.out_capacity_bytes = out_rays * 8;
    c->serve = S;
    S->worker = std::thread(worker_loop, S);
    if (c->mock) {
        S->mock_queue.resize(o.max_inflight);
        for (int q = 0; q < o.max_inflight; ++q) S->mock_threads.emplace_back(mock_loop, S, q);
    }
    return RC_OK;
}

rc_status rc_serve_stop(rc_ctx *c)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (!c->serve) return fail(RC_E_STATE, "server not running");
    serve_shutdown(c);
    return RC_OK;
}

rc_status rc_serve_submit(rc_ctx *c, const rc_request *rq, uint64_t *out_ticket)
{
    if (!c || !rq || !out_ticket) return fail(RC_E_INVAL, "null argument");
    ServeState *S = c->serve;
    if (!S) return fail(RC_E_STATE, "server not running (rc_serve_start)");
    if (rq->n_envs < 1 || !rq->poses_3x4) return fail(RC_E_INVAL, "need n_envs >= 1 and poses");
    if (!(rq->t_min >= 0.0f) || !(rq->t_max >= rq->t_min))
        return fail(RC_E_INVAL, "need 0 <= t_min <= t_max");
    int32_t n_beams = 0;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        Scene *sc = get_scene(c, rq->scene);
        if (!sc) return fail(RC_E_NOTFOUND, "unknown scene %d", rq->scene);
        if (sc->nt > 0 && !sc->has_bvh) return fail(RC_E_STATE, "scene %d has no BVH", rq->scene);
        Pattern *pt = get_pattern(c, rq->pattern);
        if (!pt) return fail(RC_E_NOTFOUND, "unknown pattern %d", rq->pattern);
        n_beams = pt->n_beams;
    }
    const int64_t rays = (int64_t)rq->n_envs * n_beams;
    if (rays > (int64_t)0x7fffffff) return fail(RC_E_INVAL, "more than 2^31-1 rays");
    for (int64_t i = 0; i < (int64_t)rq->n_envs * 12; ++i)
        if (!isfinite(rq->poses_3x4[i])) return fail(RC_E_INVAL, "non-finite pose value");
    Request *r = new Request();
    r->req = *rq;
    r->n_rays = rays;
    r->poses.assign(rq->poses_3x4, rq->poses_3x4 + (size_t)rq->n_envs * 12);
    std::lock_guard<std::mutex> lk(S->mu);
    if ((uint64_t)rays > S->out_arena.size() ||
        (uint64_t)rq->n_envs * 12 > S->pose_arena.size()) {
        ++S->stats.rejected;
        delete r;
        return fail(RC_E_NOMEM, "request needs %lld rays of output; the server holds %llu",
                    (long long)rays, (unsigned long long)S->out_arena.size());
    }
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    S->tickets[r->ticket] = r;
    S->pending.push_back(r);
    ++S->stats.submitted;
    S->cv.notify_all();
    *out_ticket = r->ticket;
    return RC_OK;
}

rc_status rc_serve_poll(rc_ctx *c, uint64_t ticket, int64_t timeout_us, const float **out_range,
                        const int32_t **out_hit, double *latency_ms)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    ServeState *S = c->serve;
    if (!S) return fail(RC_E_STATE, "server not running");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(RC_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    auto finished = [&] { return r->state == REQ_DONE || r->state == REQ_FAILED; };
    if (!finished() && timeout_us > 0)
        S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), finished);
    else if (!finished() && timeout_us < 0)
        S->cv.wait(lk, finished);
    if (!finished()) return RC_PENDING;
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (r->state == REQ_FAILED) return fail(r->status, "request failed: %s", r->error.c_str());
    if (out_range) *out_range = S->range_buf + r->out_off;
    if (out_hit) *out_hit = S->hit_buf + r->out_off;
    return RC_OK;
}

rc_status rc_serve_release(rc_ctx *c, uint64_t ticket)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    ServeState *S = c->serve;
    if (!S) return fail(RC_E_STATE, "server not running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(RC_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->state == REQ_RUNNING) return fail(RC_E_BUSY, "ticket %llu is on the device", (unsigned long long)ticket);
    if (r->state == REQ_PENDING) {
        for (auto q = S->pending.begin(); q != S->pending.end(); ++q)
            if (*q == r) {
                S->pending.erase(q);
                break;
            }
        ++S->stats.cancelled;
    }
    free_request_memory(*S, r);
    S->tickets.erase(it);
    delete r;
    S->cv.notify_all();
    return RC_OK;
}

rc_status rc_serve_copy(rc_ctx *c, uint64_t ticket, float *range_dst, int32_t *hit_dst,
                        int dst_is_host)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    ServeState *S = c->serve;
    if (!S) return fail(RC_E_STATE, "server not running");
    const float *src_r = nullptr;
    const int32_t *src_h = nullptr;
    int64_t n = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->tickets.find(ticket);
        if (it == S->tickets.end())
            return fail(RC_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
        Request *r = it->second;
        if (r->state == REQ_FAILED) return fail(r->status, "request failed: %s", r->error.c_str());
        if (r->state != REQ_DONE) return RC_PENDING;
        src_r = S->range_buf + r->out_off;
        src_h = S->hit_buf + r->out_off;
        n = r->n_rays;
    }
    // the ticket cannot be released concurrently by a well-behaved caller
    if (c->mock) {
        if (!dst_is_host) return fail(RC_E_INVAL, "a mock context copies to host memory only");
        if (range_dst) memcpy(range_dst, src_r, sizeof(float) * n);
        if (hit_dst) memcpy(hit_dst, src_h, sizeof(int32_t) * n);
        return RC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    const hipMemcpyKind k = dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (range_dst) HIP_TRY(hipMemcpy(range_dst, src_r, sizeof(float) * n, k));
    if (hit_dst) HIP_TRY(hipMemcpy(hit_dst, src_h, sizeof(int32_t) * n, k));
    return RC_OK;
}

rc_status rc_serve_get_stats(rc_ctx *c, rc_serve_stats *out)
{
    if (!c || !out) return fail(RC_E_INVAL, "null argument");
    ServeState *S = c->serve;
    if (!S) return fail(RC_E_STATE, "server not running");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->pending = S->pending.size();
    out->inflight = (uint64_t)S->inflight;
    return RC_OK;
}

}  // extern "C"
