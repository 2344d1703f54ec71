/*
 * oracle.c -- FP64 reference for batched LiDAR ray casting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (FGGS-LiDAR, Sec. IV-C, "LiDAR measurement model" and the
 * nearest-intersection equation t*_j = min_k eta(r_j, tri_k)):
 *
 *   for every environment e and beam j
 *     origin    o = t_e                      (translation column of the pose)
 *     direction d = normalize(R_e b_j)       (d_j is a unit vector, so the
 *                                             ray parameter is the range)
 *     t*        = min over all triangles k of the ray-triangle parameter,
 *                 discarding misses and parameters outside [t_min, t_max]
 *     hit id    = the k attaining t*, the lowest k on exact ties
 *
 * This is the naive O(N_rays * N_tris) baseline the paper contrasts its BVH
 * traversal with (Sec. IV-C, "naive baseline" cost): every ray is tested
 * against every triangle.  No acceleration structure, no blocking.
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes):
 *   - the ray-triangle test eta is the watertight test of Woop, Benthin and
 *     Wald (JCGT 2013), evaluated in FP64, two-sided (no face culling);
 *     an edge function that comes out exactly zero is recomputed exactly
 *     (binary128 products of doubles are exact, so its sign is exact);
 *   - [t_min, t_max] is closed;
 *   - a miss is reported as t = +inf, id = -1;
 *   - zero-area triangles are never hit (determinant zero).
 *
 * Inputs are FP32 (as the user holds them) and are promoted exactly to FP64.
 * Pose layout: f32[12] row-major [R | t] (3 rows of 4).
 *
 * Parity pins for this file are in tests/test_oracle_*.py: closed forms
 * (plane, box room, analytic sphere within tessellation error), exact
 * rational arithmetic on random triangle soups, watertightness of closed
 * meshes, hand-made special cases and the edge-nearness construction.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

/* ------------------------------------------------------------------------ */
/* Ray generation: Sec. IV-C, r_j(t) = x_s + t d_j with x_s = t_s and d_j a
 * unit direction given by the scan pattern, rotated into the world by R_s. */
static void make_ray(const float *pose, const float *beam, double o[3],
                     double d[3])
{
    for (int i = 0; i < 3; ++i) {
        o[i] = (double)pose[4 * i + 3];
        d[i] = (double)pose[4 * i + 0] * (double)beam[0] +
               (double)pose[4 * i + 1] * (double)beam[1] +
               (double)pose[4 * i + 2] * (double)beam[2];
    }
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= n;
    d[1] /= n;
    d[2] /= n;
}

void oracle_make_rays(const float *poses, int64_t n_envs, const float *dirs,
                      int64_t n_beams, double *out_o, double *out_d)
{
    for (int64_t e = 0; e < n_envs; ++e)
        for (int64_t j = 0; j < n_beams; ++j) {
            int64_t r = e * n_beams + j;
            make_ray(poses + 12 * e, dirs + 3 * j, out_o + 3 * r,
                     out_d + 3 * r);
        }
}

/* ------------------------------------------------------------------------ */
/* Watertight ray-triangle test (Woop, Benthin, Wald 2013) in FP64.
 * Returns 1 and stores the ray parameter in *t_out on a hit. */
typedef struct {
    double o[3];
    int kx, ky, kz;
    double Sx, Sy, Sz;
} ray_frame;

static void ray_frame_init(ray_frame *f, const double o[3], const double d[3])
{
    /* kz: dimension where |d| is largest, lowest index on ties */
    int kz = 0;
    if (fabs(d[1]) > fabs(d[kz])) kz = 1;
    if (fabs(d[2]) > fabs(d[kz])) kz = 2;
    int kx = (kz + 1) % 3;
    int ky = (kx + 1) % 3;
    if (d[kz] < 0.0) { int s = kx; kx = ky; ky = s; }  /* keep winding */
    f->kx = kx; f->ky = ky; f->kz = kz;
    f->Sx = d[kx] / d[kz];
    f->Sy = d[ky] / d[kz];
    f->Sz = 1.0 / d[kz];
    f->o[0] = o[0]; f->o[1] = o[1]; f->o[2] = o[2];
}

static int woop_test(const ray_frame *f, const float *v0, const float *v1,
                     const float *v2, double *t_out)
{
    const int kx = f->kx, ky = f->ky, kz = f->kz;
    /* vertices relative to the ray origin */
    double A[3], B[3], C[3];
    for (int i = 0; i < 3; ++i) {
        A[i] = (double)v0[i] - f->o[i];
        B[i] = (double)v1[i] - f->o[i];
        C[i] = (double)v2[i] - f->o[i];
    }
    /* shear and scale so that the ray becomes the +z axis */
    double Ax = A[kx] - f->Sx * A[kz], Ay = A[ky] - f->Sy * A[kz];
    double Bx = B[kx] - f->Sx * B[kz], By = B[ky] - f->Sy * B[kz];
    double Cx = C[kx] - f->Sx * C[kz], Cy = C[ky] - f->Sy * C[kz];
    /* scaled barycentric coordinates (2-D edge functions) */
    double U = Cx * By - Cy * Bx;
    double V = Ax * Cy - Ay * Cx;
    double W = Bx * Ay - By * Ax;
    double Az = f->Sz * A[kz], Bz = f->Sz * B[kz], Cz = f->Sz * C[kz];

    if (U == 0.0 || V == 0.0 || W == 0.0) {
        /* exact fallback: a product of two doubles is exact in binary128
         * and the correctly rounded difference keeps the exact sign */
        quad Uq = (quad)Cx * (quad)By - (quad)Cy * (quad)Bx;
        quad Vq = (quad)Ax * (quad)Cy - (quad)Ay * (quad)Cx;
        quad Wq = (quad)Bx * (quad)Ay - (quad)By * (quad)Ax;
        if ((Uq < 0 || Vq < 0 || Wq < 0) && (Uq > 0 || Vq > 0 || Wq > 0))
            return 0;
        quad detq = Uq + Vq + Wq;
        if (detq == 0) return 0;
        quad Tq = Uq * (quad)Az + Vq * (quad)Bz + Wq * (quad)Cz;
        *t_out = (double)(Tq / detq);
        return 1;
    }
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0))
        return 0;
    double det = U + V + W;
    if (det == 0.0) return 0;
    double T = U * Az + V * Bz + W * Cz;
    *t_out = T / det;
    return 1;
}

/* Single-ray, single-triangle entry point (used by the pin tests). */
int oracle_tri_test(const double *o, const double *d, const float *v0,
                    const float *v1, const float *v2, double *t_out)
{
    ray_frame f;
    ray_frame_init(&f, o, d);
    return woop_test(&f, v0, v1, v2, t_out);
}

/* ------------------------------------------------------------------------ */
/* Closest hit over all triangles: the nearest-intersection equation. */
static void closest_hit(const double o[3], const double d[3],
                        const float *verts, const int32_t *tris, int64_t nt,
                        double t_min, double t_max, double *best_t,
                        int32_t *best_id)
{
    ray_frame f;
    ray_frame_init(&f, o, d);
    double bt = INFINITY;
    int32_t bid = -1;
    for (int64_t k = 0; k < nt; ++k) {
        const int32_t *tri = tris + 3 * k;
        double t;
        if (!woop_test(&f, verts + 3 * (int64_t)tri[0],
                       verts + 3 * (int64_t)tri[1],
                       verts + 3 * (int64_t)tri[2], &t))
            continue;
        if (t < t_min || t > t_max) continue;
        if (t < bt || (t == bt && k < bid)) { bt = t; bid = (int32_t)k; }
    }
    *best_t = bt;
    *best_id = bid;
}

/* ------------------------------------------------------------------------ */
/* Edge nearness and ambiguity (the checker).
 *
 * A ray is "edge-near" when some triangle edge, seen from the ray origin,
 * lies within `eps_rad` radians of the ray direction and is no farther from
 * the origin than the ray's result (t* + tol, or t_max + tol on a miss).
 * The angular distance from d to the great-circle arc spanned by the edge
 * endpoints a, b (relative to o) is the angle to the plane (o, a, b) when
 * d's projection onto that plane falls inside the wedge between a and b,
 * and the smaller angle to a or b otherwise.
 *
 * A ray is "ambiguous" when a second triangle is hit within tol(t*) of t*,
 * or when any hit lies within tol of t_min or of a finite t_max;
 * tol(t) = 1e-4 + 1e-6 t.
 * Several results are correct for such rays. */
static double tol_of(double t) { return 1e-4 + 1e-6 * fabs(t); }

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double angle_between(const double u[3], const double v[3])
{
    double c[3];
    cross3(u, v, c);
    return atan2(sqrt(dot3(c, c)), dot3(u, v));
}

/* angular distance from unit d to the arc of edge (a, b) seen from o */
double oracle_edge_angle(const double *o, const double *d, const float *a,
                         const float *b)
{
    double ap[3], bp[3], n[3];
    for (int i = 0; i < 3; ++i) {
        ap[i] = (double)a[i] - o[i];
        bp[i] = (double)b[i] - o[i];
    }
    cross3(ap, bp, n);
    double nn = dot3(n, n);
    double ea = angle_between(d, ap), eb = angle_between(d, bp);
    double best = ea < eb ? ea : eb;
    if (nn > 0.0) {
        double dn = dot3(d, n);
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = d[i] - dn / nn * n[i];
        double c1[3], c2[3];
        cross3(ap, p, c1);
        cross3(p, bp, c2);
        if (dot3(c1, n) >= 0.0 && dot3(c2, n) >= 0.0 && dot3(p, p) > 0.0) {
            double s = fabs(dn) / sqrt(nn);
            if (s > 1.0) s = 1.0;
            double w = asin(s);
            if (w < best) best = w;
        }
    }
    return best;
}

static double seg_dist(const double o[3], const float *a, const float *b)
{
    double ap[3], ab[3];
    for (int i = 0; i < 3; ++i) {
        ap[i] = (double)a[i] - o[i];
        ab[i] = (double)b[i] - (double)a[i];
    }
    double l2 = dot3(ab, ab), u = 0.0;
    if (l2 > 0.0) {
        u = -dot3(ap, ab) / l2;
        if (u < 0.0) u = 0.0;
        if (u > 1.0) u = 1.0;
    }
    double x[3] = {ap[0] + u * ab[0], ap[1] + u * ab[1], ap[2] + u * ab[2]};
    return sqrt(dot3(x, x));
}

enum { FLAG_EDGE_NEAR = 1, FLAG_AMBIGUOUS = 2 };

static void check_ray(const double o[3], const double d[3], const float *verts,
                      const int32_t *tris, int64_t nt, double t_min,
                      double t_max, double best_t, int32_t best_id,
                      double eps_rad, int32_t *flags, double *second_t,
                      double *min_edge_angle)
{
    ray_frame f;
    ray_frame_init(&f, o, d);
    double depth_lim = (best_id >= 0 ? best_t : t_max);
    depth_lim += tol_of(depth_lim);
    double s_eps = sin(eps_rad);
    int32_t fl = 0;
    double st = INFINITY, mina = INFINITY;
    for (int64_t k = 0; k < nt; ++k) {
        const float *v[3] = {verts + 3 * (int64_t)tris[3 * k + 0],
                             verts + 3 * (int64_t)tris[3 * k + 1],
                             verts + 3 * (int64_t)tris[3 * k + 2]};
        double t;
        if (woop_test(&f, v[0], v[1], v[2], &t)) {
            /* an infinite t_max has no neighbourhood: nothing is near it */
            if (fabs(t - t_min) <= tol_of(t_min) ||
                (isfinite(t_max) && fabs(t - t_max) <= tol_of(t_max)))
                fl |= FLAG_AMBIGUOUS;
            if (k != best_id && t >= t_min - tol_of(t_min) &&
                t <= t_max + tol_of(t_max)) {
                if (t < st) st = t;
                if (best_id >= 0 && fabs(t - best_t) <= tol_of(best_t))
                    fl |= FLAG_AMBIGUOUS;
            }
        }
        for (int e = 0; e < 3; ++e) {
            const float *a = v[e], *b = v[(e + 1) % 3];
            /* cheap reject: angle to the plane (o, a, b) exceeds eps */
            double ap[3], bp[3], n[3];
            for (int i = 0; i < 3; ++i) {
                ap[i] = (double)a[i] - o[i];
                bp[i] = (double)b[i] - o[i];
            }
            cross3(ap, bp, n);
            double nn = dot3(n, n), dn = dot3(d, n);
            if (nn > 0.0 && dn * dn > 4.0 * s_eps * s_eps * nn) continue;
            if (seg_dist(o, a, b) > depth_lim) continue;
            double w = oracle_edge_angle(o, d, a, b);
            if (w < mina) mina = w;
            if (w <= eps_rad) fl |= FLAG_EDGE_NEAR;
        }
    }
    *flags = fl;
    *second_t = st;
    *min_edge_angle = mina;
}

/* ------------------------------------------------------------------------ */
/* Batched driver: rays are (env, beam) pairs or an explicit index sample,
 * striped across threads. */
typedef struct {
    const float *verts;
    const int32_t *tris;
    int64_t nt;
    const float *poses;
    const float *dirs;
    int64_t n_beams;
    const int64_t *ray_idx; /* NULL: ray r is index r */
    int64_t n_rays;
    double t_min, t_max;
    double *out_t;
    int32_t *out_id;
    /* checker outputs (NULL to skip) */
    int32_t *out_flags;
    double *out_second_t;
    double *out_min_angle;
    double eps_rad;
    int tid, nthreads;
} job_t;

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    for (int64_t r = j->tid; r < j->n_rays; r += j->nthreads) {
        int64_t g = j->ray_idx ? j->ray_idx[r] : r;
        int64_t e = g / j->n_beams, b = g % j->n_beams;
        double o[3], d[3];
        make_ray(j->poses + 12 * e, j->dirs + 3 * b, o, d);
        double bt;
        int32_t bid;
        closest_hit(o, d, j->verts, j->tris, j->nt, j->t_min, j->t_max, &bt,
                    &bid);
        j->out_t[r] = bt;
        j->out_id[r] = bid;
        if (j->out_flags)
            check_ray(o, d, j->verts, j->tris, j->nt, j->t_min, j->t_max, bt,
                      bid, j->eps_rad, j->out_flags + r, j->out_second_t + r,
                      j->out_min_angle + r);
    }
    return NULL;
}

static int run_jobs(job_t *proto, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int i = 0; i < nthreads; ++i) {
        jobs[i] = *proto;
        jobs[i].tid = i;
        jobs[i].nthreads = nthreads;
    }
    int started = 0;
    for (int i = 1; i < nthreads; ++i) {
        if (pthread_create(&th[i], NULL, worker, &jobs[i]) != 0) break;
        started = i;
    }
    /* any thread that failed to start is covered by running its stripe here */
    worker(&jobs[0]);
    for (int i = started + 1; i < nthreads; ++i) worker(&jobs[i]);
    for (int i = 1; i <= started; ++i) pthread_join(th[i], NULL);
    return nthreads;
}

/* Closest hit for rays (env, beam) given by ray_idx[n_rays] (flattened
 * index e * n_beams + b), or all n_envs * n_beams rays when ray_idx is NULL
 * (then n_rays must equal n_envs * n_beams).  Returns the thread count. */
int oracle_raycast(const float *verts, int64_t nv, const int32_t *tris,
                   int64_t nt, const float *poses, const float *dirs,
                   int64_t n_beams, const int64_t *ray_idx, int64_t n_rays,
                   double t_min, double t_max, double *out_t, int32_t *out_id,
                   int nthreads)
{
    (void)nv;
    job_t j;
    memset(&j, 0, sizeof j);
    j.verts = verts; j.tris = tris; j.nt = nt; j.poses = poses;
    j.dirs = dirs; j.n_beams = n_beams; j.ray_idx = ray_idx;
    j.n_rays = n_rays; j.t_min = t_min; j.t_max = t_max;
    j.out_t = out_t; j.out_id = out_id;
    return run_jobs(&j, nthreads);
}

/* Closest hit plus the checker outputs (edge-near / ambiguous flags, the
 * nearest hit of any other triangle, and the smallest relevant edge angle). */
int oracle_raycast_checked(const float *verts, int64_t nv, const int32_t *tris,
                           int64_t nt, const float *poses, const float *dirs,
                           int64_t n_beams, const int64_t *ray_idx,
                           int64_t n_rays, double t_min, double t_max,
                           double eps_rad, double *out_t, int32_t *out_id,
                           int32_t *out_flags, double *out_second_t,
                           double *out_min_angle, int nthreads)
{
    (void)nv;
    job_t j;
    memset(&j, 0, sizeof j);
    j.verts = verts; j.tris = tris; j.nt = nt; j.poses = poses;
    j.dirs = dirs; j.n_beams = n_beams; j.ray_idx = ray_idx;
    j.n_rays = n_rays; j.t_min = t_min; j.t_max = t_max;
    j.out_t = out_t; j.out_id = out_id; j.out_flags = out_flags;
    j.out_second_t = out_second_t; j.out_min_angle = out_min_angle;
    j.eps_rad = eps_rad;
    return run_jobs(&j, nthreads);
}
