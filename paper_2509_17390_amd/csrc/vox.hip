// vox.hip -- C ABI of the Gaussian-to-occupancy conversion (FGGS-LiDAR
// Sec. IV-A on the Gaussian model of Sec. III-A): Gaussian sets, their
// LBVH, and the tiled density / occupancy / surface launches.
#include "ctx.h"

#include <math.h>
#include <string.h>

#include <mutex>
#include <utility>
#include <vector>

namespace rc {

void free_gauss_set(rc_ctx *c, GaussSet &g)
{
    const int64_t n = g.n, ni = n > 1 ? n - 1 : 1;
    dev_free(c, g.params, sizeof(float4) * 3 * n);
    dev_free(c, g.boxes, sizeof(float) * 6 * n);
    dev_free(c, g.morton, sizeof(uint32_t) * n);
    dev_free(c, g.sorted, sizeof(uint32_t) * n);
    dev_free(c, g.topo, sizeof(int32_t) * 3 * ni);
    dev_free(c, g.nodes, sizeof(NodeRec) * ni);
    dev_free(c, g.recs, sizeof(GaussRec) * n);
    dev_free(c, g.box_dev, sizeof(float) * 8);
    g = GaussSet();
}

namespace {

GaussSet *get_gset(rc_ctx *c, int32_t id)
{
    if (id < 0 || id >= (int32_t)c->gsets.size() || !c->gsets[id].alive) return nullptr;
    return &c->gsets[id];
}

// Checks the grid and fills the launch description.
rc_status make_grid(const rc_grid *gr, VoxGrid &g)
{
    if (!gr) return fail(RC_E_INVAL, "null grid");
    const int tile = gr->tile ? gr->tile : kVoxTile;
    if (tile != kVoxTile) return fail(RC_E_INVAL, "tile edge %d not supported (8)", gr->tile);
    if (!(gr->spacing > 0.0f) || !isfinite(gr->spacing))
        return fail(RC_E_INVAL, "spacing must be finite and > 0");
    if (!isfinite(gr->theta)) return fail(RC_E_INVAL, "theta must be finite");
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(gr->origin[a])) return fail(RC_E_INVAL, "origin must be finite");
        if (gr->dims[a] < 1 || gr->dims[a] > (1 << 30))
            return fail(RC_E_INVAL, "dims must be in 1..2^30");
        const double far = fabs((double)gr->origin[a]) + (double)gr->dims[a] * gr->spacing;
        if (!(far < 1e38)) return fail(RC_E_INVAL, "grid extends beyond the float range");
    }
    memset(&g, 0, sizeof g);
    for (int a = 0; a < 3; ++a) g.o[a] = gr->origin[a];
    g.h = gr->spacing;
    g.nx = gr->dims[0];
    g.ny = gr->dims[1];
    g.nz = gr->dims[2];
    g.tx = (g.nx + kVoxTile - 1) / kVoxTile;
    g.ty = (g.ny + kVoxTile - 1) / kVoxTile;
    g.tz = (g.nz + kVoxTile - 1) / kVoxTile;
    g.n_tiles = (int64_t)g.tx * g.ty * g.tz;
    if (g.n_tiles > 0x7ffffff0LL) return fail(RC_E_INVAL, "too many tiles (%lld)", (long long)g.n_tiles);
    g.theta = gr->theta;
    return RC_OK;
}

// Looks up a built set for a conversion launch (caller holds c->mu).
rc_status built_set(rc_ctx *c, int32_t set, GaussSet **out)
{
    GaussSet *g = get_gset(c, set);
    if (!g) return fail(RC_E_NOTFOUND, "unknown Gaussian set %d", set);
    if (!g->has_bvh) return fail(RC_E_STATE, "Gaussian set %d is not built (call rc_gauss_build)", set);
    *out = g;
    return RC_OK;
}

}  // namespace
}  // namespace rc

using namespace rc;

rc_status rc_gauss_upload(rc_ctx *c, const float *means, const float *quats, const float *scales,
                          const float *opacity, int64_t n, int src_is_device, void *stream,
                          int32_t *out_set)
{
    if (!c || !out_set) return fail(RC_E_INVAL, "null context or out_set");
    if (n < 0) return fail(RC_E_INVAL, "negative size");
    if (n > 0x7ffffffeLL) return fail(RC_E_INVAL, "too many Gaussians (%lld)", (long long)n);
    if (n > 0 && (!means || !quats || !scales || !opacity))
        return fail(RC_E_INVAL, "null Gaussian array");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not convert Gaussians");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mu);
    GaussSet g;
    g.n = n;
    rc_status st = dev_alloc(c, (void **)&g.params, sizeof(float4) * 3 * n);
    if (st == RC_OK) st = dev_alloc(c, (void **)&g.box_dev, sizeof(float) * 8);
    // host arrays are staged on the device first (11 floats per Gaussian)
    float *stage = nullptr;
    if (st == RC_OK && !src_is_device && n > 0) st = dev_alloc(c, (void **)&stage, sizeof(float) * 11 * n);
    if (st != RC_OK) {
        free_gauss_set(c, g);
        return st;
    }
    GaussArrays arr;
    arr.n = n;
    hipError_t e = hipSuccess;
    if (src_is_device) {
        arr.mean = means;
        arr.quat = quats;
        arr.scale = scales;
        arr.opacity = opacity;
    } else {
        arr.mean = stage;
        arr.quat = stage + 3 * n;
        arr.scale = stage + 7 * n;
        arr.opacity = stage + 10 * n;
        const hipMemcpyKind kind = hipMemcpyHostToDevice;
        if (n) e = hipMemcpyAsync((void *)arr.mean, means, sizeof(float) * 3 * n, kind, s);
        if (e == hipSuccess && n) e = hipMemcpyAsync((void *)arr.quat, quats, sizeof(float) * 4 * n, kind, s);
        if (e == hipSuccess && n) e = hipMemcpyAsync((void *)arr.scale, scales, sizeof(float) * 3 * n, kind, s);
        if (e == hipSuccess && n) e = hipMemcpyAsync((void *)arr.opacity, opacity, sizeof(float) * n, kind, s);
    }
    const GaussParams p = g.view();
    if (e == hipSuccess) e = gauss_pack_launch(arr, g.params, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->flags_dev, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = gauss_validate_launch(p, c->flags_dev, s);
    int32_t flags = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&flags, c->flags_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) (void)hipDeviceSynchronize();   // nothing may still use the buffers
    if (stage) dev_free(c, stage, sizeof(float) * 11 * n);
    if (e != hipSuccess) {
        free_gauss_set(c, g);
        return fail(RC_E_DEVICE, "Gaussian upload failed: %s", hipGetErrorString(e));
    }
    if (flags) {
        free_gauss_set(c, g);
        return fail(RC_E_INVAL, "invalid Gaussians:%s%s%s%s", (flags & 1) ? " non-finite value" : "",
                    (flags & 2) ? " scale <= 0" : "", (flags & 4) ? " zero quaternion" : "",
                    (flags & 8) ? " opacity outside [0, 1]" : "");
    }
    g.alive = true;
    g.bytes = sizeof(float4) * 3 * n;
    int32_t id = -1;
    for (size_t i = 0; i < c->gsets.size(); ++i)
        if (!c->gsets[i].alive) { id = (int32_t)i; break; }
    if (id < 0) {
        id = (int32_t)c->gsets.size();
        c->gsets.push_back(g);
    } else {
        c->gsets[id] = g;
    }
    *out_set = id;
    return RC_OK;
}

rc_status rc_gauss_build(rc_ctx *c, int32_t set, const rc_gauss_opts *opts, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    float k = 3.0f;
    int bits = 10;
    if (opts) {
        if (opts->cutoff_sigma != 0.0f) k = opts->cutoff_sigma;
        if (opts->morton_bits) bits = opts->morton_bits;
    }
    if (!(k > 0.0f) || !isfinite(k)) return fail(RC_E_INVAL, "cutoff_sigma must be finite and > 0");
    if (bits < 1 || bits > 10) return fail(RC_E_INVAL, "morton_bits must be in 1..10");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not convert Gaussians");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mu);
    GaussSet *g = get_gset(c, set);
    if (!g) return fail(RC_E_NOTFOUND, "unknown Gaussian set %d", set);
    const int64_t n = g->n, ni = n > 1 ? n - 1 : 1;
    if (n > 0 && !g->nodes) {
        rc_status st = dev_alloc(c, (void **)&g->boxes, sizeof(float) * 6 * n);
        if (st == RC_OK) st = dev_alloc(c, (void **)&g->morton, sizeof(uint32_t) * n);
        if (st == RC_OK) st = dev_alloc(c, (void **)&g->sorted, sizeof(uint32_t) * n);
        if (st == RC_OK) st = dev_alloc(c, (void **)&g->topo, sizeof(int32_t) * 3 * ni);
        if (st == RC_OK) st = dev_alloc(c, (void **)&g->nodes, sizeof(NodeRec) * ni);
        if (st == RC_OK) st = dev_alloc(c, (void **)&g->recs, sizeof(GaussRec) * n);
        if (st != RC_OK) {
            dev_free(c, g->boxes, sizeof(float) * 6 * n);
            dev_free(c, g->morton, sizeof(uint32_t) * n);
            dev_free(c, g->sorted, sizeof(uint32_t) * n);
            dev_free(c, g->topo, sizeof(int32_t) * 3 * ni);
            dev_free(c, g->nodes, sizeof(NodeRec) * ni);
            dev_free(c, g->recs, sizeof(GaussRec) * n);
            g->boxes = nullptr;
            g->morton = g->sorted = nullptr;
            g->topo = nullptr;
            g->nodes = nullptr;
            g->recs = nullptr;
            return st;
        }
        g->bytes += sizeof(float) * 6 * n + sizeof(uint32_t) * 2 * n + sizeof(int32_t) * 3 * ni +
                    sizeof(NodeRec) * ni + sizeof(GaussRec) * n;
    }
    if (n > 0) {
        rc_status st = ensure_build_ws(c, lbvh_workspace_bytes(n), s);
        if (st != RC_OK) return st;
        const GaussParams p = g->view();
        HIP_TRY(gauss_boxes_launch(p, k, g->boxes, s));
        BuildBuffers b;
        b.verts = nullptr;
        b.tris = nullptr;
        b.nv = 0;
        b.nt = n;
        b.morton_bits = bits;
        b.ws = c->ws;
        b.ws_bytes = c->ws_bytes;
        b.morton = g->morton;
        b.sorted = g->sorted;
        b.topo = g->topo;
        b.nodes = g->nodes;
        b.trirecs = nullptr;
        b.scene_box = g->box_dev;
        b.depth_out = reinterpret_cast<int32_t *>(g->box_dev + 6);
        b.q8nodes = nullptr;
        b.q8_count = nullptr;
        HIP_TRY(lbvh_build_boxes_launch(b, g->boxes, s));
        HIP_TRY(gauss_records_launch(p, g->sorted, g->recs, s));
        HIP_TRY(hipEventRecord(c->ws_event, s));
        c->ws_event_recorded = true;
    }
    g->has_bvh = true;
    g->cutoff = k;
    g->morton_bits = bits;
    return RC_OK;
}

rc_status rc_gauss_release(rc_ctx *c, int32_t set)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not convert Gaussians");
    HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    GaussSet *g = get_gset(c, set);
    if (!g) return fail(RC_E_NOTFOUND, "unknown Gaussian set %d", set);
    HIP_TRY(hipDeviceSynchronize());
    free_gauss_set(c, *g);
    return RC_OK;
}

rc_status rc_voxelize(rc_ctx *c, int32_t set, const rc_grid *grid, float *out_density,
                      uint8_t *out_occ, uint8_t *out_surf, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (!out_density && !out_occ && !out_surf) return fail(RC_E_INVAL, "no output given");
    if (out_surf && !out_occ) return fail(RC_E_INVAL, "the surface mask needs out_occ");
    VoxGrid vg;
    rc_status st = make_grid(grid, vg);
    if (st != RC_OK) return st;
    if (c->mock) return fail(RC_E_STATE, "a mock context does not convert Gaussians");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NodeRec *nodes;
    const GaussRec *recs;
    const float *boxes;
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        GaussSet *g;
        st = built_set(c, set, &g);
        if (st != RC_OK) return st;
        nodes = g->nodes;
        recs = g->recs;
        boxes = g->boxes;
        n = g->n;
    }
    HIP_TRY(voxelize_launch(0, nodes, recs, boxes, n, vg, out_density, out_occ, nullptr, s));
    if (out_surf) HIP_TRY(surface_launch(out_occ, out_surf, vg, s));
    return RC_OK;
}

rc_status rc_voxelize_counts(rc_ctx *c, int32_t set, const rc_grid *grid, int32_t *out_counts,
                             void *stream)
{
    if (!c || !out_counts) return fail(RC_E_INVAL, "null argument");
    VoxGrid vg;
    rc_status st = make_grid(grid, vg);
    if (st != RC_OK) return st;
    if (c->mock) return fail(RC_E_STATE, "a mock context does not convert Gaussians");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NodeRec *nodes;
    const GaussRec *recs;
    const float *boxes;
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        GaussSet *g;
        st = built_set(c, set, &g);
        if (st != RC_OK) return st;
        nodes = g->nodes;
        recs = g->recs;
        boxes = g->boxes;
        n = g->n;
    }
    HIP_TRY(voxelize_launch(1, nodes, recs, boxes, n, vg, nullptr, nullptr, out_counts, s));
    return RC_OK;
}

rc_status rc_gauss_debug_copy(rc_ctx *c, int32_t set, int32_t what, void *dst, uint64_t bytes)
{
    if (!c || !dst) return fail(RC_E_INVAL, "null argument");
    if (c->mock) return fail(RC_E_STATE, "a mock context holds no device arrays");
    HIP_TRY(hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->mu);
    GaussSet *g;
    rc_status st = built_set(c, set, &g);
    if (st != RC_OK) return st;
    const int64_t n = g->n, ni = n > 1 ? n - 1 : 0;
    const void *src = nullptr;
    uint64_t size = 0;
    switch (what) {
    case RC_GDBG_BOXES: src = g->boxes; size = 24ull * n; break;
    case RC_GDBG_SORTED: src = g->sorted; size = 4ull * n; break;
    case RC_GDBG_TOPOLOGY: src = g->topo; size = 12ull * ni; break;
    case RC_GDBG_RECORDS: src = g->recs; size = sizeof(GaussRec) * (uint64_t)n; break;
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

// ---------------------------------------------------------------------------
// Narrow-band TSDF and marching cubes (Sec. IV-B).

namespace {

rc_status make_tsdf_grid(const rc_grid *gr, TsdfGrid &g)
{
    if (!gr) return fail(RC_E_INVAL, "null grid");
    if (!(gr->spacing > 0.0f) || !isfinite(gr->spacing))
        return fail(RC_E_INVAL, "spacing must be finite and > 0");
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(gr->origin[a])) return fail(RC_E_INVAL, "origin must be finite");
        if (gr->dims[a] < 1 || gr->dims[a] > (1 << 30))
            return fail(RC_E_INVAL, "dims must be in 1..2^30");
        const double far = fabs((double)gr->origin[a]) + (double)gr->dims[a] * gr->spacing;
        if (!(far < 1e38)) return fail(RC_E_INVAL, "grid extends beyond the float range");
    }
    memset(&g, 0, sizeof g);
    for (int a = 0; a < 3; ++a) g.o[a] = gr->origin[a];
    g.h = gr->spacing;
    g.hf = gr->spacing;
    g.nx = gr->dims[0];
    g.ny = gr->dims[1];
    g.nz = gr->dims[2];
    g.n = (int64_t)g.nx * g.ny * g.nz;
    if (g.n > ((int64_t)1 << 34)) return fail(RC_E_INVAL, "grid too large");
    g.cx = fastdiv_constant((uint32_t)g.nx);
    g.cy = fastdiv_constant((uint32_t)g.ny);
    return RC_OK;
}

// Sub-buffers carved from the context's grow-only TSDF / marching-cubes
// scratch (the caller holds c->mesh_mu for the whole call; the calls are
// synchronous, so nothing still uses the scratch when it is regrown).
struct Scratch {
    rc_ctx *c;
    size_t used = 0;
    std::vector<std::pair<void **, size_t>> want;
    explicit Scratch(rc_ctx *ctx) : c(ctx) {}
    template <class T>
    void take(T **p, size_t bytes)
    {
        want.push_back({(void **)p, (bytes + 255) & ~(size_t)255});
    }
    rc_status commit()
    {
        size_t need = 0;
        for (auto &w : want) need += w.second;
        if (need > c->mesh_ws_bytes) {
            if (c->mesh_ws) dev_free(c, c->mesh_ws, c->mesh_ws_bytes);
            c->mesh_ws = nullptr;
            c->mesh_ws_bytes = 0;
            rc_status st = dev_alloc(c, &c->mesh_ws, need);
            if (st != RC_OK) return st;
            c->mesh_ws_bytes = need;
        }
        char *base = static_cast<char *>(c->mesh_ws);
        for (auto &w : want) {
            *w.first = base;
            base += w.second;
        }
        return RC_OK;
    }
};

}  // namespace

// Outside-labelling rounds enqueued per flag read: 6 first (the usual
// masks settle in 5 to 10 rounds), then 2, 4 and 8 at a time, so that few
// rounds run after the fixed point and a slow mask still costs few reads.
constexpr int kFloodBatchMax = 8;
inline int flood_batch(int k) { return k == 0 ? 6 : (k == 1 ? 2 : (k == 2 ? 4 : 8)); }

rc_status rc_tsdf(rc_ctx *c, const rc_grid *grid, const uint8_t *surf, const rc_tsdf_opts *opts,
                  float *out_phi, uint8_t *out_vtilde, void *stream)
{
    if (!c || !surf || !out_phi || !opts) return fail(RC_E_INVAL, "null argument");
    TsdfGrid g;
    rc_status st = make_tsdf_grid(grid, g);
    if (st != RC_OK) return st;
    const float sigma = opts->sigma_smooth, tau = opts->tau, r = opts->band;
    if (!(sigma > 0.0f) || !isfinite(sigma)) return fail(RC_E_INVAL, "sigma_smooth must be finite and > 0");
    const int quant = opts->threshold_mode;
    if (quant != 0 && quant != 1) return fail(RC_E_INVAL, "threshold_mode must be 0 or 1");
    if (quant == 0 && !isfinite(tau)) return fail(RC_E_INVAL, "tau must be finite");
    if (quant == 1 && !(opts->quantile >= 0.0f && opts->quantile <= 1.0f))
        return fail(RC_E_INVAL, "quantile must be in [0, 1]");
    if (!(r > 0.0f) || !isfinite(r)) return fail(RC_E_INVAL, "band must be finite and > 0");
    const double sv = (double)sigma / (double)g.hf;
    const double nn = floor(2.0 * sv * sv + 0.5);
    Binomial w;
    memset(&w, 0, sizeof w);
    w.n = nn < 1.0 ? 1 : (nn > kMaxBinomial ? kMaxBinomial + 1 : (int)nn);
    if (w.n > kMaxBinomial) return fail(RC_E_INVAL, "sigma_smooth too large for the spacing (n > 10)");
    for (int k = 0; k <= 2 * w.n; ++k) {   // C(2n, k)
        uint64_t b = 1;
        for (int q = 1; q <= k; ++q) b = b * (uint64_t)(2 * w.n - q + 1) / (uint64_t)q;
        w.w[k] = (uint32_t)b;
    }
    const double thr_d = quant ? 0.0 : ceil((double)tau * ldexp(1.0, 6 * w.n));
    const uint64_t thr = thr_d <= 0.0 ? 0ull : (uint64_t)thr_d;
    // quantile re-threshold: V' >= Quantile_q(V') with the quantile
    // interpolated linearly between the order statistics x_k and x_(k+1),
    // k = floor(q (N - 1)); no sum lies strictly between them, so the test
    // is sum >= x_k when q (N - 1) is an integer, else sum >= x_(k+1)
    uint64_t q_rank = 0;
    if (quant) {
        const double pos = (double)opts->quantile * (double)(g.n - 1);
        const double k = floor(pos);
        q_rank = (uint64_t)k + (pos > k ? 2 : 1);
        if (q_rank > (uint64_t)g.n) q_rank = (uint64_t)g.n;
    }
    const double shells_d = ceil((double)r / (double)g.hf);
    if (shells_d > 250.0) return fail(RC_E_INVAL, "band / spacing above 250 shells");
    const int shells = (int)shells_d;
    if (c->mock) return fail(RC_E_STATE, "a mock context does not build TSDFs");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    uint32_t *a;
    uint64_t *b;
    uint8_t *vt = out_vtilde, *pbuf;
    uint64_t *fw, *ow, *seg;
    int32_t *flag;
    // the shell kernel reads whole words up to one z-layer beyond the grid
    const int64_t pad = tsdf_shell_pad(g);
    const int64_t nwords = (int64_t)tsdf_words_per_row(g) * g.ny * g.nz;
    ws.take(&a, tsdf_smooth_a_bytes(g));
    ws.take(&b, tsdf_smooth_b_bytes(g));
    if (!vt) ws.take(&vt, g.n);
    ws.take(&pbuf, g.n + 2 * pad + 4);
    ws.take(&fw, sizeof(uint64_t) * nwords);
    ws.take(&ow, sizeof(uint64_t) * nwords);
    ws.take(&seg, sizeof(uint64_t) * 5 * tsdf_seg_words(g));
    ws.take(&flag, sizeof(int32_t) * kFloodBatchMax);
    uint64_t *sums = nullptr;
    char *sel = nullptr;
    if (quant) {
        ws.take(&sums, sizeof(uint64_t) * (size_t)g.n);
        ws.take(&sel, radix_select_state_bytes());
    }
    st = ws.commit();
    if (st != RC_OK) return st;
    uint8_t *p = pbuf + pad;
    if (quant) {
        HIP_TRY(tsdf_smooth_sums_launch(surf, a, b, sums, g, w, s));
        HIP_TRY(radix_select_u64_launch(sums, g.n, q_rank, sel, s));
        HIP_TRY(tsdf_threshold_launch(sums, radix_select_value(sel), vt, g.n, s));
        HIP_TRY(tsdf_pack_launch(vt, fw, ow, g, s));
    } else if (tsdf_smooth_pack_fused(w)) {
        HIP_TRY(tsdf_smooth_pack_launch(surf, vt, fw, ow, g, w, thr, s));
    } else {
        HIP_TRY(tsdf_smooth_launch(surf, a, b, vt, g, w, thr, s));
        HIP_TRY(tsdf_pack_launch(vt, fw, ow, g, s));
    }
    // rounds until one changes nothing, enqueued in batches with one flag
    // read per batch: a round after a round that changed nothing returns at
    // once, and repeating a settled round changes nothing
    for (int64_t it = 0, k = 0;; ++k) {
        const int nb = flood_batch((int)(k < 3 ? k : 3));
        int32_t changed[kFloodBatchMax];
        HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t) * nb, s));
        for (int r = 0; r < nb; ++r)
            HIP_TRY(tsdf_flood_round_launch(fw, ow, seg, g, r ? flag + r - 1 : nullptr, flag + r,
                                            s));
        HIP_TRY(hipMemcpyAsync(changed, flag, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!changed[nb - 1]) break;
        it += nb;
        if (it > g.n) return fail(RC_E_DEVICE, "outside labelling did not settle");
    }
    HIP_TRY(tsdf_shells_phi_launch(vt, ow, p, out_phi, g, shells, g.hf, r, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RC_OK;
}

rc_status rc_marching_cubes(rc_ctx *c, const rc_grid *grid, const float *phi, float iso,
                            float *out_verts, int32_t *out_tris, float *out_normals,
                            int64_t cap_verts, int64_t cap_tris, int64_t *n_verts,
                            int64_t *n_tris, void *stream)
{
    if (!c || !phi || !n_verts || !n_tris) return fail(RC_E_INVAL, "null argument");
    if (!isfinite(iso)) return fail(RC_E_INVAL, "iso must be finite");
    if ((out_verts == nullptr) != (out_tris == nullptr))
        return fail(RC_E_INVAL, "give both output arrays or neither");
    if (out_normals && !out_verts) return fail(RC_E_INVAL, "normals need the vertex array");
    TsdfGrid g;
    rc_status st = make_tsdf_grid(grid, g);
    if (st != RC_OK) return st;
    // at most 3 vertices per lattice point and 5 triangles per cell: 32-bit
    // counts and int32 vertex ids hold grids up to 2^29 voxels
    if (g.n > ((int64_t)1 << 29)) return fail(RC_E_INVAL, "grid too large for 32-bit counts");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not extract meshes");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (!c->mc_table) {
            uint8_t host[256 + 256 * 15];
            mc_table_copy(host, reinterpret_cast<int8_t *>(host + 256));
            st = dev_alloc(c, (void **)&c->mc_table, sizeof host);
            if (st != RC_OK) return st;
            HIP_TRY(hipMemcpy(c->mc_table, host, sizeof host, hipMemcpyHostToDevice));
        }
    }
    const uint8_t *ntri = c->mc_table;
    const int8_t *tris_of = reinterpret_cast<const int8_t *>(c->mc_table + 256);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    uint8_t *mask, *cases;
    uint16_t *voff;
    uint32_t *vs, *ts;
    const int64_t ns = mc_scan_sums_len(g.n);
    ws.take(&mask, g.n);
    ws.take(&cases, g.n);
    ws.take(&voff, sizeof(uint16_t) * g.n);
    ws.take(&vs, sizeof(uint32_t) * ns);
    ws.take(&ts, sizeof(uint32_t) * ns);
    st = ws.commit();
    if (st != RC_OK) return st;
    HIP_TRY(mc_count_launch(phi, g, iso, ntri, mask, cases, voff, vs, ts, s));
    uint32_t tot[2];
    HIP_TRY(hipMemcpyAsync(&tot[0], vs + ns - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&tot[1], ts + ns - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_verts = tot[0];
    *n_tris = tot[1];
    if (!out_verts) return RC_OK;
    if (cap_verts < (int64_t)tot[0] || cap_tris < (int64_t)tot[1])
        return fail(RC_E_NOMEM, "mesh needs %u vertices and %u triangles", tot[0], tot[1]);
    HIP_TRY(mc_emit_launch(phi, g, iso, ntri, tris_of, mask, cases, voff, vs, ts, out_verts,
                           out_tris, out_normals, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RC_OK;
}

rc_status rc_marching_cubes_step(rc_ctx *c, const rc_grid *grid, const float *phi, float iso,
                                 int32_t step, float *out_verts, int32_t *out_tris,
                                 float *out_normals, int64_t cap_verts, int64_t cap_tris,
                                 int64_t *n_verts, int64_t *n_tris, void *stream)
{
    if (step < 1) return fail(RC_E_INVAL, "mc_step must be >= 1");
    if (step == 1)
        return rc_marching_cubes(c, grid, phi, iso, out_verts, out_tris, out_normals, cap_verts,
                                 cap_tris, n_verts, n_tris, stream);
    if (!c || !phi || !n_verts || !n_tris) return fail(RC_E_INVAL, "null argument");
    TsdfGrid g;
    rc_status st = make_tsdf_grid(grid, g);
    if (st != RC_OK) return st;
    if (c->mock) return fail(RC_E_STATE, "a mock context does not extract meshes");
    // the lattice of every step-th voxel centre: a grid of spacing
    // fl32(step h) and origin fl32(o - (step - 1) h / 2), whose voxel
    // centres fall on the fine centres (i step + 1/2) h
    rc_grid sub = *grid;
    sub.spacing = (float)((double)grid->spacing * (double)step);
    for (int a = 0; a < 3; ++a) {
        sub.dims[a] = (grid->dims[a] - 1) / step + 1;
        sub.origin[a] =
            (float)((double)grid->origin[a] - (double)(step - 1) * (double)grid->spacing / 2.0);
    }
    const int64_t m = (int64_t)sub.dims[0] * sub.dims[1] * sub.dims[2];
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *fine = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        st = dev_alloc(c, (void **)&fine, sizeof(float) * (size_t)m);
    }
    if (st != RC_OK) return st;
    hipError_t e = mc_stride_gather_launch(phi, g, step, sub.dims[0], sub.dims[1], sub.dims[2],
                                           fine, s);
    if (e != hipSuccess) st = fail(RC_E_DEVICE, "stride gather: %s", hipGetErrorString(e));
    if (st == RC_OK)
        st = rc_marching_cubes(c, &sub, fine, iso, out_verts, out_tris, out_normals, cap_verts,
                               cap_tris, n_verts, n_tris, stream);
    // rc_marching_cubes is synchronous, so the gathered field is no longer read
    if (st != RC_OK) (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> lk(c->mu);
    dev_free(c, fine, sizeof(float) * (size_t)m);
    return st;
}

rc_status rc_marching_cubes_table(uint8_t *count, int8_t *tris)
{
    if (!count || !tris) return fail(RC_E_INVAL, "null argument");
    mc_table_copy(count, tris);
    return RC_OK;
}

// ---------------------------------------------------------------------------
// Nearest neighbours and fidelity metrics (Sec. V).

namespace {

rc_status check_cloud(const float *p, int64_t n, const char *what)
{
    if (n < 0) return fail(RC_E_INVAL, "%s: negative size", what);
    if (n > 0x7ffffffeLL) return fail(RC_E_INVAL, "%s: too many points", what);
    if (n > 0 && !p) return fail(RC_E_INVAL, "%s: null array", what);
    return RC_OK;
}

}  // namespace

rc_status rc_nearest(rc_ctx *c, const float *ref, int64_t n_ref, const float *query,
                     int64_t n_query, double *out_dist, int32_t *out_idx, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    rc_status st = check_cloud(ref, n_ref, "reference");
    if (st == RC_OK) st = check_cloud(query, n_query, "query");
    if (st != RC_OK) return st;
    if (n_query > 0 && (!out_dist || !out_idx)) return fail(RC_E_INVAL, "null output");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not search point clouds");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    char *scr;
    ws.take(&scr, nn_scratch_bytes(n_ref));
    st = ws.commit();
    if (st != RC_OK) return st;
    {
        std::lock_guard<std::mutex> lk2(c->mu);
        st = ensure_build_ws(c, nn_workspace_bytes(n_ref), s);
        if (st != RC_OK) return st;
        HIP_TRY(nearest_launch(ref, n_ref, query, n_query, out_dist, out_idx, scr, c->ws,
                               c->ws_bytes, s));
        HIP_TRY(hipEventRecord(c->ws_event, s));
        c->ws_event_recorded = true;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return RC_OK;
}

rc_status rc_chamfer_fscore(rc_ctx *c, const float *p, int64_t n_p, const float *g, int64_t n_g,
                            float tau, rc_fidelity *out, void *stream)
{
    if (!c || !out) return fail(RC_E_INVAL, "null argument");
    rc_status st = check_cloud(p, n_p, "P");
    if (st == RC_OK) st = check_cloud(g, n_g, "G");
    if (st != RC_OK) return st;
    if (n_p == 0 || n_g == 0) return fail(RC_E_INVAL, "both clouds must hold points");
    if (!(tau >= 0.0f) || !isfinite(tau)) return fail(RC_E_INVAL, "tau must be finite and >= 0");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not search point clouds");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    const size_t nn = nn_scratch_bytes(n_p) > nn_scratch_bytes(n_g) ? nn_scratch_bytes(n_p)
                                                                      : nn_scratch_bytes(n_g);
    Scratch ws(c);
    char *scr;
    double *dpg, *dgp, *sums;
    int32_t *ipg, *igp;
    unsigned long long *cnts;
    ws.take(&scr, nn);
    ws.take(&dpg, sizeof(double) * n_p);
    ws.take(&ipg, sizeof(int32_t) * n_p);
    ws.take(&dgp, sizeof(double) * n_g);
    ws.take(&igp, sizeof(int32_t) * n_g);
    ws.take(&sums, sizeof(double) * 2);
    ws.take(&cnts, sizeof(unsigned long long) * 2);
    st = ws.commit();
    if (st != RC_OK) return st;
    {
        std::lock_guard<std::mutex> lk2(c->mu);
        const int64_t nmax = n_p > n_g ? n_p : n_g;
        st = ensure_build_ws(c, nn_workspace_bytes(nmax), s);
        if (st != RC_OK) return st;
        HIP_TRY(nearest_launch(g, n_g, p, n_p, dpg, ipg, scr, c->ws, c->ws_bytes, s));
        HIP_TRY(metric_sums_launch(dpg, n_p, (double)tau, scr, nn_metric_offset(n_g), &sums[0],
                                   &cnts[0], s));
        HIP_TRY(nearest_launch(p, n_p, g, n_g, dgp, igp, scr, c->ws, c->ws_bytes, s));
        HIP_TRY(metric_sums_launch(dgp, n_g, (double)tau, scr, nn_metric_offset(n_p), &sums[1],
                                   &cnts[1], s));
        HIP_TRY(hipEventRecord(c->ws_event, s));
        c->ws_event_recorded = true;
    }
    double hs[2];
    unsigned long long hc[2];
    HIP_TRY(hipMemcpyAsync(hs, sums, sizeof hs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hc, cnts, sizeof hc, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    memset(out, 0, sizeof *out);
    out->n_p = n_p;
    out->n_g = n_g;
    out->mean_pg = hs[0] / (double)n_p;
    out->mean_gp = hs[1] / (double)n_g;
    out->chamfer = 0.5 * (out->mean_pg + out->mean_gp);
    out->precision = (double)hc[0] / (double)n_p;
    out->recall = (double)hc[1] / (double)n_g;
    const double pr = out->precision + out->recall;
    out->fscore = pr > 0.0 ? 2.0 * out->precision * out->recall / pr : 0.0;
    return RC_OK;
}

// ---------------------------------------------------------------------------
// Mesh optimisation (Sec. IV-B).

rc_status rc_taubin_smooth(rc_ctx *c, float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                           float lambda, float mu, int32_t iterations, void *stream)
{
    if (!c) return fail(RC_E_INVAL, "null context");
    if (nv < 0 || nt < 0) return fail(RC_E_INVAL, "negative sizes");
    if (nv > 0x7ffffffeLL || nt > 0x7ffffffeLL) return fail(RC_E_INVAL, "mesh too large");
    if ((nv > 0 && !verts) || (nt > 0 && !tris)) return fail(RC_E_INVAL, "null mesh array");
    if (nt > 0 && nv == 0) return fail(RC_E_INVAL, "triangles without vertices");
    if (!isfinite(lambda) || !isfinite(mu)) return fail(RC_E_INVAL, "lambda and mu must be finite");
    if (iterations < 0 || iterations > 100000) return fail(RC_E_INVAL, "iterations out of range");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not smooth meshes");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    int32_t *slots, *deg, *flags;
    uint32_t *cnt;
    uint8_t *fixed;
    float *tmp;
    ws.take(&slots, sizeof(int32_t) * kNbrCap * (size_t)nv);
    ws.take(&cnt, sizeof(uint32_t) * (size_t)nv);
    ws.take(&deg, sizeof(int32_t) * (size_t)nv);
    ws.take(&fixed, (size_t)nv);
    ws.take(&tmp, sizeof(float) * 3 * (size_t)nv);
    ws.take(&flags, sizeof(int32_t));
    rc_status st = ws.commit();
    if (st != RC_OK) return st;
    int32_t hf = 0;
    HIP_TRY(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    HIP_TRY(validate_mesh_launch(verts, nv, tris, nt, flags, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf) return fail(RC_E_INVAL, "invalid mesh:%s%s", (hf & 1) ? " index out of range" : "",
                        (hf & 2) ? " non-finite vertex" : "");
    HIP_TRY(nbr_build_launch(tris, nt, nv, slots, cnt, deg, fixed, flags, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf) return fail(RC_E_INVAL, "a vertex has more than %d incident triangle corners", kNbrCap / 2);
    HIP_TRY(taubin_launch(verts, tmp, slots, deg, fixed, nv, lambda, mu, iterations, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RC_OK;
}

rc_status rc_remove_small_components(rc_ctx *c, const float *verts, int64_t nv,
                                     const int32_t *tris, int64_t nt, int64_t min_faces,
                                     float *out_verts, int32_t *out_tris, int64_t *n_verts_out,
                                     int64_t *n_tris_out, void *stream)
{
    if (!c || !n_verts_out || !n_tris_out) return fail(RC_E_INVAL, "null argument");
    if (nv < 0 || nt < 0) return fail(RC_E_INVAL, "negative sizes");
    if (nv > 0x7ffffffeLL || nt > 0x7ffffffeLL) return fail(RC_E_INVAL, "mesh too large");
    if ((nv > 0 && (!verts || !out_verts)) || (nt > 0 && (!tris || !out_tris)))
        return fail(RC_E_INVAL, "null mesh array");
    if (nt > 0 && nv == 0) return fail(RC_E_INVAL, "triangles without vertices");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not edit meshes");
    *n_verts_out = 0;
    *n_tris_out = 0;
    if (nt == 0) return RC_OK;
    // components of fewer than 1 triangle do not exist: clamp, and counts
    // never exceed nt
    const uint32_t mf = (uint32_t)(min_faces < 0 ? 0 : (min_faces > nt ? nt + 1 : min_faces));
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    uint32_t *parent, *label, *faces, *used, *newid, *keep, *tpos, *sums;
    int32_t *flags;
    const size_t nss = (size_t)mc_scan_sums_len(nv > nt ? nv : nt);
    ws.take(&parent, sizeof(uint32_t) * (size_t)nv);
    ws.take(&label, sizeof(uint32_t) * (size_t)nv);
    ws.take(&faces, sizeof(uint32_t) * (size_t)nv);
    ws.take(&used, sizeof(uint32_t) * (size_t)nv);
    ws.take(&newid, sizeof(uint32_t) * (size_t)nv);
    ws.take(&keep, sizeof(uint32_t) * (size_t)nt);
    ws.take(&tpos, sizeof(uint32_t) * (size_t)nt);
    ws.take(&sums, sizeof(uint32_t) * nss);
    ws.take(&flags, sizeof(int32_t));
    rc_status st = ws.commit();
    if (st != RC_OK) return st;
    int32_t hf = 0;
    HIP_TRY(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    HIP_TRY(validate_mesh_launch(verts, nv, tris, nt, flags, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf & 1) return fail(RC_E_INVAL, "invalid mesh: index out of range");
    HIP_TRY(components_launch(tris, nt, nv, parent, label, faces, s));
    HIP_TRY(hipMemsetAsync(used, 0, sizeof(uint32_t) * (size_t)nv, s));
    HIP_TRY(components_keep_launch(tris, nt, label, faces, mf, keep, used, s));
    HIP_TRY(scan_u32_launch(keep, tpos, nt, sums, s));
    uint32_t tot[2];
    HIP_TRY(hipMemcpyAsync(&tot[1], sums + mc_scan_sums_len(nt) - 1, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(scan_u32_launch(used, newid, nv, sums, s));
    HIP_TRY(hipMemcpyAsync(&tot[0], sums + mc_scan_sums_len(nv) - 1, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(components_emit_launch(verts, nv, used, newid, tris, nt, keep, tpos, out_verts, out_tris,
                                   s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_verts_out = tot[0];
    *n_tris_out = tot[1];
    return RC_OK;
}

rc_status rc_decimate(rc_ctx *c, const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                      float ratio, float *out_verts, int32_t *out_tris, int64_t *n_verts_out,
                      int64_t *n_tris_out, float *cell_out, void *stream)
{
    if (!c || !n_verts_out || !n_tris_out) return fail(RC_E_INVAL, "null argument");
    if (nv < 1 || nt < 1) return fail(RC_E_INVAL, "the mesh needs vertices and triangles");
    if (nv > 0x7ffffffeLL || nt > 0x7ffffffeLL) return fail(RC_E_INVAL, "mesh too large");
    if (!verts || !tris || !out_verts || !out_tris) return fail(RC_E_INVAL, "null mesh array");
    if (!(ratio > 0.0f) || !isfinite(ratio)) return fail(RC_E_INVAL, "ratio must be finite and > 0");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not decimate meshes");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    int32_t *slots, *tdeg, *flags;
    uint32_t *cnt, *keys, *vals, *keys2, *vals2, *flag, *gpos, *gid, *gstart, *keep, *tpos, *used,
        *newid, *sums, *cpart;
    uint8_t *bnd;
    double *Q, *lo;
    float *partial, *box;
    char *sortws;
    const size_t nss = (size_t)mc_scan_sums_len(nv > nt ? nv : nt);
    ws.take(&slots, sizeof(int32_t) * kNbrCap * (size_t)nv);
    ws.take(&cnt, sizeof(uint32_t) * (size_t)nv);
    ws.take(&tdeg, sizeof(int32_t) * (size_t)nv);
    ws.take(&bnd, (size_t)nv);
    ws.take(&Q, sizeof(double) * 10 * (size_t)nv);
    ws.take(&keys, sizeof(uint32_t) * (size_t)nv);
    ws.take(&vals, sizeof(uint32_t) * (size_t)nv);
    ws.take(&keys2, sizeof(uint32_t) * (size_t)nv);
    ws.take(&vals2, sizeof(uint32_t) * (size_t)nv);
    ws.take(&flag, sizeof(uint32_t) * (size_t)nv);
    ws.take(&gpos, sizeof(uint32_t) * (size_t)nv);
    ws.take(&gid, sizeof(uint32_t) * (size_t)nv);
    ws.take(&gstart, sizeof(uint32_t) * ((size_t)nv + 1));
    ws.take(&used, sizeof(uint32_t) * (size_t)nv);
    ws.take(&newid, sizeof(uint32_t) * (size_t)nv);
    ws.take(&keep, sizeof(uint32_t) * (size_t)nt);
    ws.take(&tpos, sizeof(uint32_t) * (size_t)nt);
    ws.take(&sums, sizeof(uint32_t) * nss);
    ws.take(&partial, sizeof(float) * 6 * kMinmaxBlocks);
    ws.take(&box, sizeof(float) * 8);
    ws.take(&lo, sizeof(double) * 4);
    ws.take(&sortws, radix_sort_ws_bytes(nv));
    ws.take(&cpart, count_kept_ws_bytes());
    ws.take(&flags, sizeof(int32_t));
    rc_status st = ws.commit();
    if (st != RC_OK) return st;
    int32_t hf = 0;
    HIP_TRY(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    HIP_TRY(validate_mesh_launch(verts, nv, tris, nt, flags, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf) return fail(RC_E_INVAL, "invalid mesh:%s%s", (hf & 1) ? " index out of range" : "",
                        (hf & 2) ? " non-finite vertex" : "");
    // incident-triangle lists, boundary vertices, per-vertex quadrics, box
    HIP_TRY(tri_lists_launch(tris, nt, nv, slots, cnt, tdeg, flags, s));
    HIP_TRY(vertex_quadrics_launch(verts, tris, slots, tdeg, nv, Q, bnd, flags, s));
    HIP_TRY(points_box_launch(verts, nv, partial, box, s));
    float hb[6];
    HIP_TRY(hipMemcpyAsync(hb, box, sizeof hb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf) return fail(RC_E_INVAL, "a vertex has more than %d incident triangles", kNbrCap / 2);
    const double hlo[3] = {hb[0], hb[1], hb[2]};
    HIP_TRY(hipMemcpyAsync(lo, hlo, sizeof hlo, hipMemcpyHostToDevice, s));
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double e = (double)hb[3 + a] - (double)hb[a];
        if (e > ext) ext = e;
    }
    // one grouping at cell size cs: keys, stable sort, groups, kept triangles
    int64_t ngroups = 0;
    uint32_t *sk = keys, *sv = vals;
    auto group = [&](double cs, int64_t *kept) -> rc_status {
        int64_t n[3];
        for (int a = 0; a < 3; ++a) n[a] = (int64_t)floor(((double)hb[3 + a] - (double)hb[a]) / cs) + 1;
        if (n[0] * n[1] * n[2] > (int64_t)kBoundaryKey) return fail(RC_E_DEVICE, "cell grid too fine");
        HIP_TRY(cell_keys_launch(verts, nv, bnd, lo, cs, n[0], n[1], keys, vals, s));
        int in_tmp = 0;
        HIP_TRY(radix_sort_launch(keys, vals, keys2, vals2, nv, 32, sortws, s, &in_tmp));
        sk = in_tmp ? keys2 : keys;
        sv = in_tmp ? vals2 : vals;
        HIP_TRY(group_flags_launch(sk, nv, flag, s));
        HIP_TRY(scan_u32_launch(flag, gpos, nv, sums, s));
        HIP_TRY(group_ids_launch(sv, flag, gpos, nv, gid, gstart, s));
        HIP_TRY(hipMemsetAsync(used, 0, sizeof(uint32_t) * nv, s));
        HIP_TRY(keep_launch(tris, nt, gid, keep, used, s));
        HIP_TRY(scan_u32_launch(keep, tpos, nt, sums, s));
        uint32_t tot = 0;
        HIP_TRY(hipMemcpyAsync(&tot, sums + mc_scan_sums_len(nt) - 1, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        uint32_t last_pos = 0, last_flag = 0;
        HIP_TRY(hipMemcpyAsync(&last_pos, gpos + nv - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&last_flag, flag + nv - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ngroups = (int64_t)last_pos + last_flag;
        *kept = tot;
        return RC_OK;
    };
    // the bisection only needs kept-face counts: keys and one triangle pass
    auto count = [&](double cs, int64_t *kept) -> rc_status {
        int64_t n[3];
        for (int a = 0; a < 3; ++a) n[a] = (int64_t)floor(((double)hb[3 + a] - (double)hb[a]) / cs) + 1;
        if (n[0] * n[1] * n[2] > (int64_t)kBoundaryKey) return fail(RC_E_DEVICE, "cell grid too fine");
        HIP_TRY(cell_keys_launch(verts, nv, bnd, lo, cs, n[0], n[1], keys, vals, s));
        HIP_TRY(count_kept_launch(tris, nt, keys, cpart, flag, s));
        uint32_t tot = 0;
        HIP_TRY(hipMemcpyAsync(&tot, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *kept = tot;
        return RC_OK;
    };
    const int64_t target = (int64_t)floor((double)ratio * (double)nt);
    double c_lo = ext / 1023.0, c_hi = ext, cs;
    int64_t kept = 0;
    st = count(c_lo, &kept);
    if (st != RC_OK) return st;
    if (kept <= target) {
        cs = c_lo;
    } else {
        for (int it = 0; it < 12; ++it) {
            const double mid = sqrt(c_lo * c_hi);
            st = count(mid, &kept);
            if (st != RC_OK) return st;
            if (kept <= target) c_hi = mid;
            else c_lo = mid;
        }
        cs = c_hi;
    }
    st = group(cs, &kept);
    if (st != RC_OK) return st;
    HIP_TRY(scan_u32_launch(used, newid, nv, sums, s));
    uint32_t nused = 0;
    HIP_TRY(hipMemcpyAsync(&nused, sums + mc_scan_sums_len(nv) - 1, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(decimate_emit_launch(verts, Q, bnd, sv, gstart, ngroups, nv, used, newid, lo, cs, tris,
                                 nt, gid, keep, tpos, out_verts, out_tris, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_verts_out = nused;
    *n_tris_out = kept;
    if (cell_out) *cell_out = (float)cs;
    return RC_OK;
}

rc_status rc_decimate_qem(rc_ctx *c, const float *verts, int64_t nv, const int32_t *tris,
                          int64_t nt, float ratio, int32_t rounds, float *out_verts,
                          int32_t *out_tris, int64_t *n_verts_out, int64_t *n_tris_out,
                          int32_t *n_steps_out, void *stream)
{
    if (!c || !n_verts_out || !n_tris_out) return fail(RC_E_INVAL, "null argument");
    if (nv < 1 || nt < 1) return fail(RC_E_INVAL, "the mesh needs vertices and triangles");
    if (nv > 0x7ffffffeLL || nt > 0x3fffffffLL) return fail(RC_E_INVAL, "mesh too large");
    if (!verts || !tris || !out_verts || !out_tris) return fail(RC_E_INVAL, "null mesh array");
    if (!(ratio > 0.0f) || !(ratio <= 1.0f)) return fail(RC_E_INVAL, "ratio must be in (0, 1]");
    if (rounds < 1 || rounds > 64) return fail(RC_E_INVAL, "rounds must be 1..64");
    if (c->mock) return fail(RC_E_STATE, "a mock context does not decimate meshes");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(c->mesh_mu);
    Scratch ws(c);
    QemBuffers b;
    uint32_t *used, *newid, *keep, *tpos, *sums;
    int32_t *flags;
    const int64_t ne_cap = 3 * nt;
    const size_t nss = (size_t)mc_scan_sums_len(nv > nt ? nv : nt);
    ws.take(&b.P, sizeof(double) * 3 * (size_t)nv);
    ws.take(&b.F, sizeof(int32_t) * 3 * (size_t)nt);
    ws.take(&b.Q, sizeof(double) * 10 * (size_t)nv);
    ws.take(&b.prot, (size_t)nv);
    ws.take(&b.fcnt, sizeof(uint32_t) * (size_t)nv);
    ws.take(&b.fl, sizeof(int32_t) * kQemFaces * (size_t)nv);
    ws.take(&b.fdeg, sizeof(int32_t) * (size_t)nv);
    ws.take(&b.nb, sizeof(int32_t) * kQemNbrs * (size_t)nv);
    ws.take(&b.ndeg, sizeof(int32_t) * (size_t)nv);
    ws.take(&b.nlarge, sizeof(uint32_t) * (size_t)nv);
    ws.take(&b.eoff, sizeof(uint32_t) * (size_t)nv);
    ws.take(&b.key, sizeof(uint64_t) * (size_t)ne_cap);
    ws.take(&b.cand, (size_t)ne_cap);
    ws.take(&b.X, sizeof(double) * 3 * (size_t)ne_cap);
    ws.take(&b.eoff_old, sizeof(uint32_t) * (size_t)nv);
    ws.take(&b.key_old, sizeof(uint64_t) * (size_t)ne_cap);
    ws.take(&b.cand_old, (size_t)ne_cap);
    ws.take(&b.X_old, sizeof(double) * 3 * (size_t)ne_cap);
    ws.take(&b.dirty, (size_t)nv);
    ws.take(&b.absorbed, sizeof(int32_t) * (size_t)nv);
    ws.take(&b.eu, sizeof(int32_t) * (size_t)ne_cap);
    ws.take(&b.ev, sizeof(int32_t) * (size_t)ne_cap);
    ws.take(&b.eu_old, sizeof(int32_t) * (size_t)ne_cap);
    ws.take(&b.ev_old, sizeof(int32_t) * (size_t)ne_cap);
    ws.take(&b.best, sizeof(unsigned long long) * (size_t)nv);
    ws.take(&b.remap, sizeof(int32_t) * (size_t)nv);
    ws.take(&b.counters, sizeof(uint32_t) * 4);
    ws.take(&b.sel, qem_sel_bytes());
    ws.take(&used, sizeof(uint32_t) * (size_t)nv);
    ws.take(&newid, sizeof(uint32_t) * (size_t)nv);
    ws.take(&keep, sizeof(uint32_t) * (size_t)nt);
    ws.take(&tpos, sizeof(uint32_t) * (size_t)nt);
    ws.take(&sums, sizeof(uint32_t) * nss);
    ws.take(&flags, sizeof(int32_t));
    rc_status st = ws.commit();
    if (st != RC_OK) return st;
    int32_t hf = 0;
    HIP_TRY(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    HIP_TRY(validate_mesh_launch(verts, nv, tris, nt, flags, s));
    HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf) return fail(RC_E_INVAL, "invalid mesh:%s%s", (hf & 1) ? " index out of range" : "",
                        (hf & 2) ? " non-finite vertex" : "");
    HIP_TRY(qem_init_launch(verts, nv, tris, nt, b.P, b.F, s));
    uint32_t hc[4] = {0, 0, 0, 0};
    // live faces after dropping repeated-corner faces
    HIP_TRY(hipMemsetAsync(b.counters, 0, sizeof(uint32_t) * 4, s));
    HIP_TRY(qem_live_launch(b, nt, s));
    HIP_TRY(hipMemcpyAsync(hc, b.counters, sizeof hc, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t f0 = hc[2];
    int64_t nf = f0;
    int64_t n_old = 0;
    int32_t steps = 0;
    const double r = (double)ratio;
    for (int k = 1; k <= rounds; ++k) {
        const int64_t target = (int64_t)ceil((double)f0 * pow(r, (double)k / (double)rounds));
        for (int first = 1;; first = 0) {
            if (nf <= target) break;
            // the previous step's edge results become the old ones
            std::swap(b.eoff, b.eoff_old);
            std::swap(b.key, b.key_old);
            std::swap(b.cand, b.cand_old);
            std::swap(b.X, b.X_old);
            std::swap(b.eu, b.eu_old);
            std::swap(b.ev, b.ev_old);
            // incidence of the live faces (a round's start also sums the
            // quadrics and protects boundary vertices), edge numbering
            HIP_TRY(hipMemsetAsync(b.counters, 0, sizeof(uint32_t) * 4, s));
            HIP_TRY(qem_incidence_launch(b, nv, nt, first, s));
            HIP_TRY(scan_u32_launch(b.nlarge, b.eoff, nv, sums, s));
            uint32_t n_edges = 0;
            HIP_TRY(hipMemcpyAsync(&n_edges, sums + mc_scan_sums_len(nv) - 1, sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(hc, b.counters, sizeof hc, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hc[3] & 1) return fail(RC_E_INVAL, "a vertex has more than %d incident triangles",
                                       kQemFaces);
            if (hc[3] & 2) return fail(RC_E_INVAL, "a vertex has more than %d neighbours",
                                       kQemNbrs);
            // every edge lies on a live face: at most three per face
            if ((int64_t)n_edges > ne_cap) return fail(RC_E_DEVICE, "edge count overflow");
            HIP_TRY(qem_edges_launch(b, nv, n_edges, n_old, first, s));
            n_old = n_edges;
            // candidates, eligibility and contraction without a host read in
            // between: the select decides on the device whether every
            // candidate is eligible, and no candidate contracts nothing
            const uint64_t need = (uint64_t)((nf - target + 1) / 2);
            HIP_TRY(qem_select_launch(b, n_edges, need, s));
            HIP_TRY(qem_contract_launch(b, nv, n_edges, s));
            HIP_TRY(hipMemcpyAsync(hc, b.counters, sizeof hc, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hc[0] == 0) break;
            ++steps;
            if (hc[1] == 0) return fail(RC_E_DEVICE, "decimation step contracted nothing");
            // a contraction drops exactly the two faces on its edge
            if (hc[2] != 2 * hc[1]) return fail(RC_E_DEVICE, "decimation face count mismatch");
            nf -= hc[2];
        }
    }
    HIP_TRY(hipMemsetAsync(used, 0, sizeof(uint32_t) * (size_t)nv, s));
    HIP_TRY(qem_used_launch(b.F, nt, used, keep, s));
    uint32_t tot[2] = {0, 0};
    HIP_TRY(scan_u32_launch(keep, tpos, nt, sums, s));
    HIP_TRY(hipMemcpyAsync(&tot[1], sums + mc_scan_sums_len(nt) - 1, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(scan_u32_launch(used, newid, nv, sums, s));
    HIP_TRY(hipMemcpyAsync(&tot[0], sums + mc_scan_sums_len(nv) - 1, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(qem_emit_launch(b.P, nv, used, newid, b.F, nt, keep, tpos, out_verts, out_tris, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_verts_out = tot[0];
    *n_tris_out = tot[1];
    if (n_steps_out) *n_steps_out = steps;
    return RC_OK;
}
