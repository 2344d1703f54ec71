// serve_stress.cpp -- multi-threaded stress of the request server on the
// mock device (host only), for sanitizer builds of librcast.
//
// Four submitter threads each push requests over two scenes and three beam
// patterns, poll them to completion, check the simulated results
// (range = ray index within the request, hit = scene id), copy them out and
// release the ticket; a fifth thread polls statistics.  One scene's
// requests fail on purpose.  A sixth thread keeps uploading a scene,
// submitting requests on it and releasing it while they are queued or
// running: each of those requests either completes with intact results or
// fails with RC_E_NOTFOUND (never with the simulated device's "scene memory
// changed"), and under AddressSanitizer any early free of the scene's memory
// would be a use after free.  Runs once with arrival-order admission and
// once with small-first admission under a per-launch ray cap.  Exit status 0
// when every check passes.
#include "rcast.h"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

static std::atomic<int> g_bad{0};

#define CHECK(cond)                                                             \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            g_bad.fetch_add(1);                                                 \
        }                                                                       \
    } while (0)

int main()
{
    rc_ctx *c = nullptr;
    if (rc_create(RC_DEVICE_MOCK, 0, &c) != RC_OK) return 2;
    const float v[9] = {0, 0, 0, 1, 0, 0, 0, 1, 0};
    const int32_t t[3] = {0, 1, 2};
    int32_t scene[3];
    for (int k = 0; k < 3; ++k) {
        CHECK(rc_scene_upload(c, v, 3, t, 1, 0, nullptr, &scene[k]) == RC_OK);
        CHECK(rc_lbvh_build(c, scene[k], nullptr, nullptr) == RC_OK);
    }
    const int nb[3] = {64, 500, 2000};
    int32_t pat[3];
    for (int p = 0; p < 3; ++p) {
        std::vector<float> d(3 * nb[p], 0.0f);
        for (int j = 0; j < nb[p]; ++j) d[3 * j] = 1.0f;
        CHECK(rc_pattern_upload(c, d.data(), nb[p], 0, &pat[p]) == RC_OK);
    }
    // first in arrival order, then small-first with aging and a ray cap
    for (int policy = 0; policy < 2; ++policy) {
    rc_serve_opts o{};
    o.arena_bytes = 4u << 20;
    o.max_inflight = 3;
    o.mock_ns_per_ray = 20;
    o.mock_fail_scene = scene[2] + 1;
    o.policy = policy;
    o.max_wait_ms = 5;
    o.max_batch_rays_m = policy;
    CHECK(rc_serve_start(c, &o) == RC_OK);

    std::atomic<bool> done{false};
    std::thread watcher([&] {
        rc_serve_stats s;
        while (!done.load()) {
            CHECK(rc_serve_get_stats(c, &s) == RC_OK);
            CHECK(s.bytes_in_use <= (4u << 20));
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    std::vector<std::thread> th;
    th.emplace_back([&] {
        std::vector<float> poses(12 * 4, 0.0f);
        for (int e = 0; e < 4; ++e) poses[12 * e + 0] = poses[12 * e + 5] = poses[12 * e + 10] = 1.0f;
        std::vector<float> vv(3 * 600);
        std::vector<int32_t> tt(3 * 200);
        for (int round = 0; round < 40; ++round) {
            for (size_t k = 0; k < vv.size(); ++k) vv[k] = (float)((k * 7 + round) % 13);
            for (size_t k = 0; k < tt.size(); ++k) tt[k] = (int32_t)k;
            int32_t sc = -1;
            CHECK(rc_scene_upload(c, vv.data(), 600, tt.data(), 200, 0, nullptr, &sc) == RC_OK);
            CHECK(rc_lbvh_build(c, sc, nullptr, nullptr) == RC_OK);
            uint64_t tk[6];
            int n_sub = 0;
            bool released = false;
            for (int i = 0; i < 6; ++i) {
                rc_request rq{};
                rq.scene = sc;
                rq.pattern = pat[i % 3];
                rq.n_envs = 1 + i % 4;
                rq.poses_3x4 = poses.data();
                rq.t_max = 1.0f;
                const rc_status st = rc_serve_submit(c, &rq, &tk[n_sub]);
                if (released) CHECK(st == RC_E_NOTFOUND);   // the handle died with the release
                else if (st == RC_OK) ++n_sub;
                else CHECK(false);
                if (i == 2 + round % 3) {
                    CHECK(rc_scene_release(c, sc) == RC_OK);
                    released = true;
                }
            }
            for (int i = 0; i < n_sub; ++i) {
                const float *rr = nullptr;
                const int32_t *hh = nullptr;
                double lat = 0.0;
                rc_status st = rc_serve_poll(c, tk[i], -1, &rr, &hh, &lat);
                CHECK(st == RC_OK || st == RC_E_NOTFOUND);
                if (st == RC_OK) {
                    const int n = (1 + i % 4) * nb[i % 3];
                    for (int k = 0; k < n; ++k) {
                        if (rr[k] != (float)k || hh[k] != sc) {
                            CHECK(false);
                            break;
                        }
                    }
                }
                CHECK(rc_serve_release(c, tk[i]) == RC_OK);
            }
        }
    });
    for (int w = 0; w < 4; ++w) {
        th.emplace_back([&, w] {
            std::vector<float> poses(12 * 8, 0.0f);
            for (int e = 0; e < 8; ++e) {
                poses[12 * e + 0] = poses[12 * e + 5] = poses[12 * e + 10] = 1.0f;
            }
            for (int i = 0; i < 60; ++i) {
                const int s = (w + i) % 3, p = i % 3, envs = 1 + (i * 7 + w) % 8;
                rc_request rq{};
                rq.scene = scene[s];
                rq.pattern = pat[p];
                rq.n_envs = envs;
                rq.poses_3x4 = poses.data();
                rq.t_min = 0.0f;
                rq.t_max = 10.0f;
                uint64_t tk = 0;
                if (rc_serve_submit(c, &rq, &tk) != RC_OK) {
                    CHECK(false);
                    continue;
                }
                const float *rr = nullptr;
                const int32_t *hh = nullptr;
                double lat = 0.0;
                rc_status st = rc_serve_poll(c, tk, -1, &rr, &hh, &lat);
                if (s == 2) {
                    CHECK(st == RC_E_DEVICE);
                } else {
                    CHECK(st == RC_OK);
                    const int n = envs * nb[p];
                    std::vector<float> r(n);
                    std::vector<int32_t> h(n);
                    CHECK(rc_serve_copy(c, tk, r.data(), h.data(), 1) == RC_OK);
                    for (int k = 0; k < n; ++k) {
                        if (r[k] != (float)k || h[k] != scene[s]) {
                            CHECK(false);
                            break;
                        }
                    }
                }
                CHECK(rc_serve_release(c, tk) == RC_OK);
            }
        });
    }
    for (auto &x : th) x.join();
    done.store(true);
    watcher.join();
    rc_serve_stats s;
    CHECK(rc_serve_get_stats(c, &s) == RC_OK);
    CHECK(s.completed + s.failed == s.submitted && s.bytes_in_use == 0);
    CHECK(s.submitted >= 240 + 40 * 3);
    CHECK(rc_serve_stop(c) == RC_OK);
    }
    // every released scene has been freed: only the three fixed ones remain
    CHECK(rc_device_bytes(c) == 3 * sizeof(v));
    rc_destroy(c);
    std::printf("serve_stress: %s\n", g_bad.load() ? "FAILED" : "ok");
    return g_bad.load() ? 1 : 0;
}
