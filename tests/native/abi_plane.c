/* Drives librcast through its C ABI alone (no Python): a 2 km square floor
 * at z = 0 seen from a sensor 1.7 m above it.  A ray with direction d from
 * o hits the floor at t = -o_z / d_z (closed form), and rays pointing up
 * miss.  Checks both node formats, the brute-force cross-check and one
 * error path.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "rcast.h"

#define PI_D 3.14159265358979323846
#define N_EL 10
#define N_AZ 16
#define NB (N_EL * N_AZ)

static int fails = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                  \
            fprintf(stderr, "\n");                         \
            ++fails;                                       \
        }                                                  \
    } while (0)
#define RC(call) CHECK((call) == RC_OK, "%s: %s", #call, rc_last_error())

int main(void)
{
    const float verts[12] = {-1000, -1000, 0, 1000, -1000, 0, 1000, 1000, 0, -1000, 1000, 0};
    const int32_t tris[6] = {0, 1, 2, 0, 2, 3};
    /* elevations -80..-5 deg (down) and one ring at +10 deg (up) */
    float dirs[NB * 3];
    for (int e = 0; e < N_EL; ++e)
        for (int a = 0; a < N_AZ; ++a) {
            const double el = (e < N_EL - 1 ? -80.0 + e * (75.0 / (N_EL - 2)) : 10.0) * PI_D / 180.0;
            const double az = a * 2.0 * PI_D / N_AZ;
            float *d = dirs + 3 * (e * N_AZ + a);
            d[0] = (float)(cos(el) * cos(az));
            d[1] = (float)(cos(el) * sin(az));
            d[2] = (float)sin(el);
        }
    const double yaw = 0.3;
    const float pose[12] = {(float)cos(yaw), (float)-sin(yaw), 0, 1.5f,
                            (float)sin(yaw), (float)cos(yaw), 0, -2.5f,
                            0, 0, 1, 1.7f};

    rc_ctx *ctx = NULL;
    RC(rc_create(0, 0, &ctx));
    if (!ctx) return 1;
    int32_t scene = -1, pat = -1;
    RC(rc_scene_upload(ctx, verts, 4, tris, 2, 0, NULL, &scene));
    RC(rc_pattern_upload(ctx, dirs, NB, N_AZ, &pat));
    float *d_pose = NULL, *d_range = NULL;
    int32_t *d_hit = NULL;
    CHECK(hipMalloc((void **)&d_pose, sizeof pose) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&d_range, NB * sizeof(float)) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&d_hit, NB * sizeof(int32_t)) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(d_pose, pose, sizeof pose, hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy");
    rc_job job;
    memset(&job, 0, sizeof job);
    job.scene = scene;
    job.pattern = pat;
    job.n_envs = 1;
    job.poses_3x4 = d_pose;
    job.t_min = 0.0f;
    job.t_max = 1000.0f;

    float range[2][NB], brute_r[NB];
    int32_t hit[2][NB], brute_h[NB];
    for (int f = 0; f < 2; ++f) {
        rc_build_opts o;
        memset(&o, 0, sizeof o);
        o.node_format = f ? RC_NODE_Q8 : RC_NODE_FP32;
        RC(rc_lbvh_build(ctx, scene, &o, NULL));
        RC(rc_raycast_batch(ctx, &job, 1, d_range, d_hit, NULL));
        CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
        CHECK(hipMemcpy(range[f], d_range, sizeof range[f], hipMemcpyDeviceToHost) == hipSuccess, "copy");
        CHECK(hipMemcpy(hit[f], d_hit, sizeof hit[f], hipMemcpyDeviceToHost) == hipSuccess, "copy");
    }
    RC(rc_raycast_bruteforce(ctx, &job, 1, d_range, d_hit, NULL));
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    CHECK(hipMemcpy(brute_r, d_range, sizeof brute_r, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(hipMemcpy(brute_h, d_hit, sizeof brute_h, hipMemcpyDeviceToHost) == hipSuccess, "copy");

    double max_err = 0.0;
    for (int j = 0; j < NB; ++j) {
        /* the library's ray: R b normalised in FP64 */
        const float *b = dirs + 3 * j;
        double d[3], n = 0.0;
        for (int i = 0; i < 3; ++i) {
            d[i] = (double)pose[4 * i] * b[0] + (double)pose[4 * i + 1] * b[1] +
                   (double)pose[4 * i + 2] * b[2];
            n += d[i] * d[i];
        }
        n = sqrt(n);
        const double dz = d[2] / n;
        for (int f = 0; f < 2; ++f) {
            if (dz < 0.0) {
                const double t = -(double)pose[11] / dz;
                CHECK(hit[f][j] == 0 || hit[f][j] == 1, "beam %d: hit %d", j, hit[f][j]);
                const double err = fabs(range[f][j] - t);
                CHECK(err <= 1e-4 + 1e-6 * t, "beam %d: range %.7f vs %.7f", j, range[f][j], t);
                if (err > max_err) max_err = err;
            } else {
                CHECK(hit[f][j] == -1 && isinf(range[f][j]), "beam %d: expected a miss", j);
            }
        }
        CHECK(memcmp(&range[0][j], &range[1][j], 4) == 0 && hit[0][j] == hit[1][j],
              "beam %d: FP32 and Q8 nodes differ", j);
        CHECK(memcmp(&range[1][j], &brute_r[j], 4) == 0 && hit[1][j] == brute_h[j],
              "beam %d: BVH and brute force differ", j);
    }
    /* an error path: an empty interval is rejected with a message */
    job.t_min = 2.0f;
    job.t_max = 1.0f;
    CHECK(rc_raycast_batch(ctx, &job, 1, d_range, d_hit, NULL) == RC_E_INVAL, "bad interval");
    CHECK(strlen(rc_last_error()) > 0, "no error text");

    RC(rc_scene_release(ctx, scene));
    (void)hipFree(d_pose);
    (void)hipFree(d_range);
    (void)hipFree(d_hit);
    rc_destroy(ctx);
    printf("abi_plane: %d beams, max range error %.3g m, %s\n", NB, max_err,
           fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
