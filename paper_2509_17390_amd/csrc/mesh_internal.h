// mesh_internal.h -- device-side interfaces of the mesh stages shared
// between the .hip files of librcast: narrow-band TSDF and marching cubes
// (tsdf.hip), nearest neighbours and fidelity metrics (nn.hip), and mesh
// optimisation (meshopt.hip), driven by vox.hip.
#pragma once

#include "gauss_internal.h"

// ---------------------------------------------------------------------------
// Narrow-band TSDF and marching cubes (tsdf.hip).

struct TsdfGrid {
    double o[3];          // origin (float32 input, exact)
    double h;             // spacing (float32 input, exact)
    float hf;             // the same spacing as float32
    int32_t nx, ny, nz;
    int64_t n;            // voxels
    // division by nx and ny for indices below 2^32: floor(i / d) is the
    // high half of c * i with c = floor((2^64 - 1) / d) + 1 (exact for all
    // 32-bit i and d >= 2); c = 0 marks d = 1
    uint64_t cx, cy;
};

// the constant of the division above
inline uint64_t fastdiv_constant(uint32_t d) { return d > 1 ? ~(uint64_t)0 / d + 1 : 0; }

// Binomial smoothing kernel: n steps, weights C(2n, n + k) for k = -n..n.
constexpr int kMaxBinomial = 10;
struct Binomial {
    int32_t n;
    uint32_t w[2 * kMaxBinomial + 1];
};

// V~ = [sum >= thr] of the separable binomial smoothing of `surf`; abuf and
// bbuf (tsdf_smooth_a_bytes / _b_bytes, 8-byte aligned) hold the x and xy
// passes (narrow and padded for kernels of at most 3 steps when surf and
// vt are 4-byte aligned, else u32 and u64).
size_t tsdf_smooth_a_bytes(const TsdfGrid &g);
size_t tsdf_smooth_b_bytes(const TsdfGrid &g);
hipError_t tsdf_smooth_launch(const uint8_t *surf, void *abuf, void *bbuf, uint8_t *vt,
                              const TsdfGrid &g, const Binomial &w, uint64_t thr, hipStream_t s);
// The integer sums of the same smoothing ([nz][ny][nx] uint64, u32 x and
// u64 xy passes in abuf / bbuf), and V~ = [sums >= *thr] with thr on the
// device (the quantile re-threshold).
hipError_t tsdf_smooth_sums_launch(const uint8_t *surf, void *abuf, void *bbuf, uint64_t *sums,
                                   const TsdfGrid &g, const Binomial &w, hipStream_t s);
hipError_t tsdf_threshold_launch(const uint64_t *sums, const uint64_t *thr, uint8_t *vt,
                                 int64_t n, hipStream_t s);
// phi at every step-th lattice point of each axis ([mz][my][mx], m = (n - 1)
// / step + 1 per axis) into out.
hipError_t mc_stride_gather_launch(const float *phi, const TsdfGrid &g, int step, int mx, int my,
                                   int mz, float *out, hipStream_t s);
// Outside labelling, bit-packed along x (tsdf_words_per_row words per
// row, [nz][ny][W] uint64 each for F and O; seg holds 5 *
// tsdf_seg_words(g) words): pack the free mask, then sweep rounds
// (*changed set when O grew).
int tsdf_words_per_row(const TsdfGrid &g);
int64_t tsdf_seg_words(const TsdfGrid &g);
// Smoothing, threshold and packing in one tiled pass (V~ into vt, the free
// and cleared outside words into F and O), for kernels of 1 to 3 steps.
bool tsdf_smooth_pack_fused(const Binomial &w);
hipError_t tsdf_smooth_pack_launch(const uint8_t *surf, uint8_t *vt, uint64_t *F, uint64_t *O,
                                   const TsdfGrid &g, const Binomial &w, uint64_t thr,
                                   hipStream_t s);
hipError_t tsdf_pack_launch(const uint8_t *vt, uint64_t *F, uint64_t *O, const TsdfGrid &g,
                            hipStream_t s);
// A round whose `prev` flag (the previous round's *changed; null: always
// run) reads 0 does nothing, so rounds can be enqueued ahead in batches.
hipError_t tsdf_flood_round_launch(const uint64_t *F, uint64_t *O, uint64_t *seg,
                                   const TsdfGrid &g, const int32_t *prev, int32_t *changed,
                                   hipStream_t s);
// Shells and phi.  p (one byte per voxel) must be 4-byte aligned with
// tsdf_shell_pad(g) readable bytes before and after it.
int64_t tsdf_shell_pad(const TsdfGrid &g);
hipError_t tsdf_shells_phi_launch(const uint8_t *vt, const uint64_t *O, uint8_t *p, float *phi,
                                  const TsdfGrid &g, int shells, float h, float r, hipStream_t s);

// Marching cubes: the case table (count[256], tri[256][15] edge ids, -1
// padded), the count pass (edge masks and cell cases, one byte each per
// point; voff: each point's vertex offset within its scan tile (u16); vsums /
// tsums: exclusive scans of the tiles' vertex and triangle totals, with
// mc_scan_sums_len(n) entries, the grand total last), and the emit pass
// (normals: float32 [nv][3] or null).
void mc_table_copy(uint8_t *count, int8_t *tri);
int64_t mc_scan_sums_len(int64_t n);
hipError_t mc_count_launch(const float *phi, const TsdfGrid &g, float iso, const uint8_t *ntri,
                           uint8_t *mask, uint8_t *cases, uint16_t *voff, uint32_t *vsums,
                           uint32_t *tsums, hipStream_t s);
hipError_t mc_emit_launch(const float *phi, const TsdfGrid &g, float iso, const uint8_t *ntri,
                          const int8_t *tris_of, const uint8_t *mask, const uint8_t *cases,
                          const uint16_t *voff, const uint32_t *vsums, const uint32_t *tsums,
                          float *verts, int32_t *tris, float *normals, hipStream_t s);

// ---------------------------------------------------------------------------
// Nearest neighbours and fidelity metrics (nn.hip).

// Scratch of nearest_launch for a reference cloud of n_ref points (build
// arrays, then the partial sums of metric_sums_launch at nn_metric_offset).
size_t nn_scratch_bytes(int64_t n_ref);
size_t nn_metric_offset(int64_t n_ref);
// LBVH build workspace (BuildBuffers::ws) for n_ref points.
size_t nn_workspace_bytes(int64_t n_ref);
// d(q, ref) (FP64) and the lowest index of a nearest reference point for
// every query; ref and query are float32 [n][3] on the device.
hipError_t nearest_launch(const float *ref, int64_t n_ref, const float *query, int64_t n_q,
                          double *out_d, int32_t *out_i, void *scratch, void *ws, size_t ws_bytes,
                          hipStream_t s);
// *out_sum = sum of d, *out_cnt = number of d <= tau (fixed summation order);
// partial sums use the scratch at byte offset `off`.
hipError_t metric_sums_launch(const double *d, int64_t n, double tau, void *scratch, size_t off,
                              double *out_sum, unsigned long long *out_cnt, hipStream_t s);

// ---------------------------------------------------------------------------
// Mesh optimisation (meshopt.hip).

constexpr int kNbrCap = 128;  // neighbour slots per vertex (two per incident triangle)
// Distinct sorted neighbours (slots [nv][kNbrCap], deg [nv]) and the fixed
// flag (boundary or isolated) of every vertex; *flags |= 1 when a vertex
// has more than kNbrCap neighbour slots.  cnt: [nv] scratch.
hipError_t nbr_build_launch(const int32_t *tris, int64_t nt, int64_t nv, int32_t *slots,
                            uint32_t *cnt, int32_t *deg, uint8_t *fixed, int32_t *flags,
                            hipStream_t s);
// `iterations` Taubin iterations in place (tmp: [nv][3] scratch).
hipError_t taubin_launch(float *verts, float *tmp, const int32_t *slots, const int32_t *deg,
                         const uint8_t *fixed, int64_t nv, float lambda, float mu, int iterations,
                         hipStream_t s);

// Stable LSD radix sort of (keys, vals) by the low key_bits bits of keys
// (build.hip); *in_tmp = 1 when the result is in (keys_tmp, vals_tmp).
size_t radix_sort_ws_bytes(int64_t n);
hipError_t radix_sort_launch(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                             int64_t n, int key_bits, void *ws, hipStream_t s, int *in_tmp);
// Exclusive scan of uint32 (tsdf.hip); sums holds mc_scan_sums_len(n)
// entries, the grand total last.
hipError_t scan_u32_launch(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *sums,
                           hipStream_t s);

// Quadric-error decimation by vertex clustering (meshopt.hip).
constexpr uint32_t kBoundaryKey = 0x40000000u;   // above every cell key (cells < 2^30)
// incident triangles of every vertex, distinct and ascending (slots
// [nv][kNbrCap], tdeg [nv]); *flags |= 1 on overflow.  cnt: [nv] scratch.
hipError_t tri_lists_launch(const int32_t *tris, int64_t nt, int64_t nv, int32_t *slots,
                            uint32_t *cnt, int32_t *tdeg, int32_t *flags, hipStream_t s);
// Q [nv][10] FP64: sum of the incident triangles' area-weighted plane
// quadrics; bnd[v] = 1 when some neighbour of v is reached through exactly
// one of its triangles (the boundary); flags[0] |= 1 when a vertex has more
// than kNbrCap / 2 triangles.
hipError_t vertex_quadrics_launch(const float *verts, const int32_t *tris, const int32_t *slots,
                                  const int32_t *tdeg, int64_t nv, double *Q, uint8_t *bnd,
                                  int32_t *flags, hipStream_t s);
// Box of the vertices: out[6] = lo xyz, hi xyz (partial: kMinmaxBlocks x 6 scratch).
constexpr int kMinmaxBlocks = 256;
hipError_t points_box_launch(const float *verts, int64_t nv, float *partial, float *out,
                             hipStream_t s);
// Cell key of every vertex (kBoundaryKey for boundary vertices), vals = index.
hipError_t cell_keys_launch(const float *verts, int64_t nv, const uint8_t *boundary,
                            const double *lo, double c, int64_t n0, int64_t n1, uint32_t *keys,
                            uint32_t *vals, hipStream_t s);
// Number of triangles whose corners fall into three groups for the keys of
// one cell size (no sort needed), into *count (device); partial holds
// count_kept_ws_bytes().
size_t count_kept_ws_bytes();
hipError_t count_kept_launch(const int32_t *tris, int64_t nt, const uint32_t *keys,
                             uint32_t *partial, uint32_t *count, hipStream_t s);
// From sorted (keys, vals): group-start flags, then (after a scan into gpos)
// the group of every vertex and the first sorted position of every group.
hipError_t group_flags_launch(const uint32_t *keys, int64_t nv, uint32_t *flag, hipStream_t s);
hipError_t group_ids_launch(const uint32_t *vals, const uint32_t *flag, const uint32_t *gpos,
                            int64_t nv, uint32_t *gid, uint32_t *gstart, hipStream_t s);
// keep[t] = 1 when the three corners of t lie in three groups; used[g] = 1
// for every group a kept triangle touches (used must be zeroed first).
hipError_t keep_launch(const int32_t *tris, int64_t nt, const uint32_t *gid, uint32_t *keep,
                       uint32_t *used, hipStream_t s);
// Connected components of a mesh (triangles joined through shared
// vertices): label[v] = a vertex of v's component shared by all its
// vertices (which one depends on thread timing), faces[label] = its
// triangle count (faces is indexed by vertex; nv entries).
hipError_t components_launch(const int32_t *tris, int64_t nt, int64_t nv, uint32_t *parent,
                             uint32_t *label, uint32_t *faces, hipStream_t s);
// keep[t] = its component has >= min_faces triangles; used[v] = 1 for the
// corners of kept triangles (used must be zero before).
hipError_t components_keep_launch(const int32_t *tris, int64_t nt, const uint32_t *label,
                                  const uint32_t *faces, uint32_t min_faces, uint32_t *keep,
                                  uint32_t *used, hipStream_t s);
// Kept vertices and triangles at their scanned positions, renumbered.
hipError_t components_emit_launch(const float *verts, int64_t nv, const uint32_t *used,
                                  const uint32_t *newid, const int32_t *tris, int64_t nt,
                                  const uint32_t *keep, const uint32_t *tpos, float *out_verts,
                                  int32_t *out_tris, hipStream_t s);
// Representatives of the used groups and the kept triangles, renumbered.
hipError_t decimate_emit_launch(const float *verts, const double *Q, const uint8_t *boundary,
                                const uint32_t *vals, const uint32_t *gstart, int64_t ngroups,
                                int64_t nv, const uint32_t *used, const uint32_t *newid,
                                const double *lo, double c, const int32_t *tris, int64_t nt,
                                const uint32_t *gid, const uint32_t *keep, const uint32_t *tpos,
                                float *out_verts, int32_t *out_tris, hipStream_t s);

// ---------------------------------------------------------------------------
// Quadric-error decimation by rounds of parallel edge contraction (qem.hip).

constexpr int kQemFaces = 64;   // incident triangles per vertex
constexpr int kQemNbrs = 64;    // distinct neighbours per vertex

struct QemBuffers {
    double *P;            // [nv][3] positions
    int32_t *F;           // [nt][3] faces; F[t][0] = -1 once removed
    double *Q;            // [nv][10] quadrics (upper triangle, row by row)
    uint8_t *prot;        // [nv] protected in this round
    uint32_t *fcnt;       // [nv] incident-face fill counters
    int32_t *fl;          // [nv][kQemFaces] incident faces, ascending
    int32_t *fdeg;        // [nv]
    int32_t *nb;          // [nv][kQemNbrs] distinct neighbours, ascending
    int32_t *ndeg;        // [nv]
    uint32_t *nlarge;     // [nv] neighbours above the vertex
    uint32_t *eoff;       // [nv] first edge number of the vertex
    uint64_t *key;        // [3 nt] candidate key (cost bits << 32 | pi(edge)) or ~0
    uint8_t *cand;        // [3 nt] edge is a candidate
    double *X;            // [3 nt][3] contraction point of a candidate
    // the previous step's eoff, key, cand and X (the host swaps the pairs
    // before each step): an edge whose two ends are clean keeps its result
    uint32_t *eoff_old;
    uint64_t *key_old;
    uint8_t *cand_old;
    double *X_old;
    int32_t *eu, *ev;     // [3 nt] edge ends
    int32_t *eu_old, *ev_old;   // the previous step's
    unsigned long long *best;   // [nv]
    int32_t *remap;       // [nv] contracted into (or -1)
    // [nv] in the closed one-rings of an edge contracted in the last step:
    // the vertex's faces, neighbours and edges are evaluated anew
    uint8_t *dirty;
    int32_t *absorbed;    // [nv] the vertex contracted into this one in the last step, or -1
    uint32_t *counters;   // [4] candidates, contracted, live faces, flags
    char *sel;            // qem_sel_bytes(): radix-select state
};

size_t qem_sel_bytes();
// P from the float32 vertices; F from the triangles, faces with a repeated
// corner removed.
hipError_t qem_init_launch(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                           double *P, int32_t *F, hipStream_t s);
// Incident faces, neighbours and neighbour counts above each vertex; at a
// round's start from all live faces, with the quadrics and protected
// flags, else for the dirty vertices only, from their previous lists.
// counters[3] |= 1 (2) when a vertex has more than kQemFaces faces
// (kQemNbrs neighbours).
hipError_t qem_incidence_launch(const QemBuffers &b, int64_t nv, int64_t nt, int round_start,
                                hipStream_t s);
// Candidate keys and points of every edge (eoff must hold the exclusive
// scan of nlarge, n_edges its total); counters[0] += candidates.  At a
// round's start every edge is evaluated; later the n_old edges of the
// previous step (eu_old, ev_old, eoff_old, key_old, cand_old, X_old) whose
// lower end is clean move to their new numbers, keeping their result when
// the upper end is clean too, and only edges with a dirty end are
// evaluated.
hipError_t qem_edges_launch(const QemBuffers &b, int64_t nv, int64_t n_edges, int64_t n_old,
                            int round_start, hipStream_t s);
// Eligibility: the need smallest candidate keys; all of them when need is
// at least counters[0] (decided on the device), else a radix select of the
// need-th smallest of the n_edges keys.
hipError_t qem_select_launch(const QemBuffers &b, int64_t n_edges, uint64_t need, hipStream_t s);
// counters[2] += live faces.
hipError_t qem_live_launch(const QemBuffers &b, int64_t nt, hipStream_t s);
// Contract the chosen edges among the eligible ones (as qem_select_launch
// left them): u takes x and Q_u + Q_v, v's
// faces are renamed to u (the two on the edge dropped), the closed
// one-rings are marked dirty (after clearing the marks); counters[1] +=
// contractions, counters[2] += faces dropped.
hipError_t qem_contract_launch(const QemBuffers &b, int64_t nv, int64_t n_edges, hipStream_t s);
// keep[t] = live face, used[v] = 1 for their corners (used zeroed first).
hipError_t qem_used_launch(const int32_t *F, int64_t nt, uint32_t *used, uint32_t *keep,
                           hipStream_t s);
// Used vertices (rounded to float32) and live faces at their scanned
// positions, renumbered.
hipError_t qem_emit_launch(const double *P, int64_t nv, const uint32_t *used,
                           const uint32_t *newid, const int32_t *F, int64_t nt,
                           const uint32_t *keep, const uint32_t *tpos, float *out_verts,
                           int32_t *out_tris, hipStream_t s);

// Radix select over 64-bit keys (qem.hip): the rank-th smallest (1-based,
// rank <= n) of keys[0..n) into the state (radix_select_state_bytes()),
// readable on the device through radix_select_value(state) once the
// launches have run.
size_t radix_select_state_bytes();
hipError_t radix_select_u64_launch(const uint64_t *keys, int64_t n, uint64_t rank, char *state,
                                   hipStream_t s);
const uint64_t *radix_select_value(const char *state);
