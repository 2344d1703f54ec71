/*
 * sdfmesh.c -- seeded synthetic scene geometry (input generator).
 *
 * Builds the closed indoor test meshes: the zero set of a signed distance
 * field (free space positive) made of one room box and a union of solid
 * primitives, polygonised with a marching-cubes variant whose per-cell
 * polygons are derived from the sign changes on the cube faces.  This file
 * produces inputs only; it holds no ray-casting arithmetic.
 *
 * Marching cubes here: for each cell, every cube face whose corners change
 * sign contributes one or two segments between the crossing points on its
 * edges.  A face with four crossings (diagonal corners equal) always cuts
 * off its free (non-negative) corners, a rule that depends only on that
 * face's corners and so agrees between the two cells sharing the face.
 * Each crossing point is the endpoint of exactly two segments (one per face
 * through its cube edge), so the segments close into simple loops, which
 * are fanned into triangles.  Crossing points live on grid edges and are
 * shared between cells, hence the mesh is closed: every mesh edge belongs
 * to exactly two triangles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { PRIM_BOX = 0, PRIM_SPHERE = 1, PRIM_CYLINDER = 2 };

/* primitive parameters, 8 doubles each:
 *   box:      cx cy cz  hx hy hz  yaw  -
 *   sphere:   cx cy cz  r  -  -   -    -
 *   cylinder: cx cy cz  r  hz -   -    -    (vertical axis)            */

static double box_sdf(double px, double py, double pz, double hx, double hy,
                      double hz)
{
    double qx = fabs(px) - hx, qy = fabs(py) - hy, qz = fabs(pz) - hz;
    double ox = qx > 0 ? qx : 0, oy = qy > 0 ? qy : 0, oz = qz > 0 ? qz : 0;
    double m = qx > qy ? qx : qy;
    m = m > qz ? m : qz;
    return sqrt(ox * ox + oy * oy + oz * oz) + (m < 0 ? m : 0);
}

static double prim_sdf(int type, const double *p, double x, double y, double z)
{
    double dx = x - p[0], dy = y - p[1], dz = z - p[2];
    if (type == PRIM_BOX) {
        double c = cos(p[6]), s = sin(p[6]);
        double lx = c * dx + s * dy, ly = -s * dx + c * dy;
        return box_sdf(lx, ly, dz, p[3], p[4], p[5]);
    }
    if (type == PRIM_SPHERE) return sqrt(dx * dx + dy * dy + dz * dz) - p[3];
    /* vertical capped cylinder */
    double a = sqrt(dx * dx + dy * dy) - p[3], b = fabs(dz) - p[4];
    double oa = a > 0 ? a : 0, ob = b > 0 ? b : 0;
    double m = a > b ? a : b;
    return sqrt(oa * oa + ob * ob) + (m < 0 ? m : 0);
}

/* conservative axis-aligned half extent of a primitive */
static void prim_extent(int type, const double *p, double e[3])
{
    if (type == PRIM_BOX) {
        double c = fabs(cos(p[6])), s = fabs(sin(p[6]));
        e[0] = c * p[3] + s * p[4];
        e[1] = s * p[3] + c * p[4];
        e[2] = p[5];
    } else if (type == PRIM_SPHERE) {
        e[0] = e[1] = e[2] = p[3];
    } else {
        e[0] = e[1] = p[3];
        e[2] = p[4];
    }
}

/* free-space field: positive inside the room and outside every primitive */
static double scene_sdf(const double *room, int n, const int32_t *types,
                        const double *params, double x, double y, double z)
{
    double cx = 0.5 * (room[0] + room[3]), cy = 0.5 * (room[1] + room[4]),
           cz = 0.5 * (room[2] + room[5]);
    double f = -box_sdf(x - cx, y - cy, z - cz, 0.5 * (room[3] - room[0]),
                        0.5 * (room[4] - room[1]), 0.5 * (room[5] - room[2]));
    for (int i = 0; i < n; ++i) {
        double g = prim_sdf(types[i], params + 8 * i, x, y, z);
        if (g < f) f = g;
    }
    return f;
}

void sdf_eval(const double *room, int n, const int32_t *types,
              const double *params, const double *pts, int64_t npts,
              double *out)
{
    for (int64_t i = 0; i < npts; ++i)
        out[i] = scene_sdf(room, n, types, params, pts[3 * i], pts[3 * i + 1],
                           pts[3 * i + 2]);
}

/* ------------------------------------------------------------------------ */
/* Per-configuration polygon table, derived from face sign changes. */

/* corner c = x + 2y + 4z; cube edges as corner pairs */
static const int EDGE_C[12][2] = {
    {0, 1}, {2, 3}, {4, 5}, {6, 7},  /* along x */
    {0, 2}, {1, 3}, {4, 6}, {5, 7},  /* along y */
    {0, 4}, {1, 5}, {2, 6}, {3, 7}}; /* along z */
/* faces as cyclic corner lists */
static const int FACE_C[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                 {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};

static int edge_of(int a, int b)
{
    for (int e = 0; e < 12; ++e)
        if ((EDGE_C[e][0] == a && EDGE_C[e][1] == b) ||
            (EDGE_C[e][0] == b && EDGE_C[e][1] == a))
            return e;
    return -1;
}

/* table[cfg]: up to 4 loops, each a list of cube edges (-1 terminated) */
typedef struct {
    int n_loops;
    int len[4];
    int8_t loop[4][12];
} cell_polys;

static cell_polys TABLE[256];
static int table_ready = 0;

static void build_table(void)
{
    for (int cfg = 0; cfg < 256; ++cfg) {
        int neg[8];
        for (int c = 0; c < 8; ++c) neg[c] = (cfg >> c) & 1;
        /* segments between crossing edges on each face */
        int seg[12][2], ns = 0;
        for (int f = 0; f < 6; ++f) {
            const int *q = FACE_C[f];
            int cross[4], nc = 0;
            for (int i = 0; i < 4; ++i)
                cross[i] = neg[q[i]] != neg[q[(i + 1) % 4]];
            for (int i = 0; i < 4; ++i) nc += cross[i];
            if (nc == 2) {
                int a = -1, b = -1;
                for (int i = 0; i < 4; ++i)
                    if (cross[i]) {
                        int e = edge_of(q[i], q[(i + 1) % 4]);
                        if (a < 0) a = e; else b = e;
                    }
                seg[ns][0] = a; seg[ns][1] = b; ++ns;
            } else if (nc == 4) {
                /* cut off the free corners: corner q[i] is cut by the
                 * segment joining its two incident face edges */
                for (int i = 0; i < 4; ++i) {
                    if (neg[q[i]]) continue;
                    int ePrev = edge_of(q[(i + 3) % 4], q[i]);
                    int eNext = edge_of(q[i], q[(i + 1) % 4]);
                    seg[ns][0] = ePrev; seg[ns][1] = eNext; ++ns;
                }
            }
        }
        /* link segments into loops */
        cell_polys *cp = &TABLE[cfg];
        memset(cp, 0, sizeof *cp);
        int used[12] = {0};
        for (int s0 = 0; s0 < ns; ++s0) {
            if (used[s0]) continue;
            int L = cp->n_loops++;
            int n = 0;
            used[s0] = 1;
            cp->loop[L][n++] = (int8_t)seg[s0][0];
            int cur = seg[s0][1];
            while (cur != seg[s0][0]) {
                cp->loop[L][n++] = (int8_t)cur;
                int found = 0;
                for (int s = 0; s < ns; ++s) {
                    if (used[s]) continue;
                    if (seg[s][0] == cur) { cur = seg[s][1]; used[s] = 1; found = 1; break; }
                    if (seg[s][1] == cur) { cur = seg[s][0]; used[s] = 1; found = 1; break; }
                }
                if (!found) break; /* cannot happen: every point has degree 2 */
            }
            cp->len[L] = n;
        }
    }
    table_ready = 1;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    float *v;
    int64_t nv, cv;
    int32_t *t;
    int64_t nt, ct;
} mesh_buf;

static int push_v(mesh_buf *m, double x, double y, double z)
{
    if (m->nv == m->cv) {
        m->cv = m->cv ? 2 * m->cv : 1 << 16;
        float *nv = (float *)realloc(m->v, (size_t)m->cv * 3 * sizeof(float));
        if (!nv) return -1;
        m->v = nv;
    }
    m->v[3 * m->nv + 0] = (float)x;
    m->v[3 * m->nv + 1] = (float)y;
    m->v[3 * m->nv + 2] = (float)z;
    return (int)m->nv++;
}

static int push_t(mesh_buf *m, int32_t a, int32_t b, int32_t c)
{
    if (m->nt == m->ct) {
        m->ct = m->ct ? 2 * m->ct : 1 << 16;
        int32_t *nt = (int32_t *)realloc(m->t, (size_t)m->ct * 3 * sizeof(int32_t));
        if (!nt) return -1;
        m->t = nt;
    }
    m->t[3 * m->nt + 0] = a;
    m->t[3 * m->nt + 1] = b;
    m->t[3 * m->nt + 2] = c;
    m->nt++;
    return 0;
}

/* Polygonise the scene field on a grid with spacing h covering the room
 * plus a margin of `pad` cells.  On success returns 0 and hands out
 * malloc'd arrays (free with sdfmesh_free). */
int sdfmesh_build(const double *room, int n, const int32_t *types,
                  const double *params, double h, int pad, float **out_v,
                  int64_t *out_nv, int32_t **out_t, int64_t *out_nt)
{
    if (!table_ready) build_table();
    double ox = room[0] - pad * h, oy = room[1] - pad * h, oz = room[2] - pad * h;
    int64_t nx = (int64_t)ceil((room[3] - room[0]) / h) + 2 * pad + 1;
    int64_t ny = (int64_t)ceil((room[4] - room[1]) / h) + 2 * pad + 1;
    int64_t nz = (int64_t)ceil((room[5] - room[2]) / h) + 2 * pad + 1;
    int64_t npt = nx * ny * nz;
    double clampv = 2.0 * h;
    float *f = (float *)malloc((size_t)npt * sizeof(float));
    int32_t *emap = (int32_t *)malloc((size_t)npt * 3 * sizeof(int32_t));
    if (!f || !emap) { free(f); free(emap); return -1; }

    /* room term, clamped to [-2h, 2h] */
    double cx = 0.5 * (room[0] + room[3]), cy = 0.5 * (room[1] + room[4]),
           cz = 0.5 * (room[2] + room[5]);
    double rx = 0.5 * (room[3] - room[0]), ry = 0.5 * (room[4] - room[1]),
           rz = 0.5 * (room[5] - room[2]);
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double x = ox + i * h, y = oy + j * h, z = oz + k * h;
                double v = -box_sdf(x - cx, y - cy, z - cz, rx, ry, rz);
                if (v > clampv) v = clampv;
                if (v < -clampv) v = -clampv;
                f[(k * ny + j) * nx + i] = (float)v;
            }
    /* primitives: only points within their box grown by 2h can change the
     * clamped minimum */
    for (int p = 0; p < n; ++p) {
        const double *q = params + 8 * p;
        double e[3];
        prim_extent(types[p], q, e);
        int64_t lo[3], hi[3];
        const double o3[3] = {ox, oy, oz};
        const int64_t n3[3] = {nx, ny, nz};
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int64_t)floor((q[a] - e[a] - clampv - o3[a]) / h);
            hi[a] = (int64_t)ceil((q[a] + e[a] + clampv - o3[a]) / h);
            if (lo[a] < 0) lo[a] = 0;
            if (hi[a] > n3[a] - 1) hi[a] = n3[a] - 1;
        }
        for (int64_t k = lo[2]; k <= hi[2]; ++k)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                    double v = prim_sdf(types[p], q, ox + i * h, oy + j * h,
                                        oz + k * h);
                    float *dst = &f[(k * ny + j) * nx + i];
                    if (v < *dst) *dst = (float)(v < -clampv ? -clampv : v);
                }
    }
    for (int64_t i = 0; i < npt * 3; ++i) emap[i] = -1;

    mesh_buf m;
    memset(&m, 0, sizeof m);
    int rc = 0;
    for (int64_t k = 0; k + 1 < nz && !rc; ++k)
        for (int64_t j = 0; j + 1 < ny && !rc; ++j)
            for (int64_t i = 0; i + 1 < nx && !rc; ++i) {
                float cv[8];
                int cfg = 0;
                for (int c = 0; c < 8; ++c) {
                    int64_t ii = i + (c & 1), jj = j + ((c >> 1) & 1),
                            kk = k + ((c >> 2) & 1);
                    cv[c] = f[(kk * ny + jj) * nx + ii];
                    if (cv[c] < 0.0f) cfg |= 1 << c;
                }
                if (cfg == 0 || cfg == 255) continue;
                const cell_polys *cp = &TABLE[cfg];
                for (int L = 0; L < cp->n_loops && !rc; ++L) {
                    int32_t vid[12];
                    for (int s = 0; s < cp->len[L]; ++s) {
                        int e = cp->loop[L][s];
                        int a = EDGE_C[e][0], b = EDGE_C[e][1];
                        int axis = e / 4;
                        int64_t ii = i + (a & 1), jj = j + ((a >> 1) & 1),
                                kk = k + ((a >> 2) & 1);
                        int64_t key = ((kk * ny + jj) * nx + ii) * 3 + axis;
                        if (emap[key] < 0) {
                            double fa = cv[a], fb = cv[b];
                            double u = fa / (fa - fb);
                            double x = ox + ii * h, y = oy + jj * h, z = oz + kk * h;
                            if (axis == 0) x += u * h;
                            else if (axis == 1) y += u * h;
                            else z += u * h;
                            int id = push_v(&m, x, y, z);
                            if (id < 0) { rc = -1; break; }
                            emap[key] = id;
                        }
                        vid[s] = emap[key];
                    }
                    for (int s = 1; !rc && s + 1 < cp->len[L]; ++s)
                        if (push_t(&m, vid[0], vid[s], vid[s + 1])) rc = -1;
                }
            }
    free(f);
    free(emap);
    if (rc) { free(m.v); free(m.t); return -1; }
    *out_v = m.v;
    *out_nv = m.nv;
    *out_t = m.t;
    *out_nt = m.nt;
    return 0;
}

void sdfmesh_free(void *p) { free(p); }
