// gauss_internal.h -- device layouts and launchers of the Gaussian-to-occupancy
// conversion (gauss.hip).  Not part of the public interface.
#pragma once

#include "rc_internal.h"

// Gaussian evaluation record, 64 bytes = 4 x float4, in leaf order:
//   r0 = (mu.x, mu.y, mu.z, A)        A = alpha^2 * 2^31
//   r1 = (M00, M01, M02, M10)
//   r2 = (M11, M12, M20, M21)
//   r3 = (M22, id, -, -)              id: index in the uploaded set (int bits)
// with M = c0 S^-1 R^T, c0 = sqrt(log2(e) / 2), so that |M (x - mu)|^2 =
// log2(e)/2 (x - mu)^T Sigma^-1 (x - mu) and w(x) = exp2(-|M (x - mu)|^2).
struct GaussRec {
    float4 r0, r1, r2, r3;
};
static_assert(sizeof(GaussRec) == 64, "Gaussian record is 64 bytes");

// Gaussian parameters on the device, 48 bytes per Gaussian (3 x float4):
//   (mu.x, mu.y, mu.z, alpha) (q.w, q.x, q.y, q.z) (s.x, s.y, s.z, 0)
struct GaussParams {
    const float4 *g;      // [n][3]
    int64_t n;
};

// The caller's arrays (device) as rc_gauss_upload receives them.
struct GaussArrays {
    const float *mean;    // [n][3]
    const float *quat;    // [n][4] (w, x, y, z)
    const float *scale;   // [n][3]
    const float *opacity; // [n]
    int64_t n;
};

// Voxel grid of one conversion launch.
struct VoxGrid {
    double o[3];          // origin (float32 input, exact)
    double h;             // spacing (float32 input, exact)
    int32_t nx, ny, nz;   // voxels
    int32_t tx, ty, tz;   // tiles (8^3 voxels each)
    int64_t n_tiles;
    float theta;
};

constexpr int kVoxTile = 8;   // tile edge in voxels

// LBVH over ready-made primitive boxes (float32 [nt][6] lo xyz, hi xyz) in
// place of triangle boxes: b.verts / b.tris are ignored and b.trirecs must
// be null (build.hip).
hipError_t lbvh_build_boxes_launch(const BuildBuffers &b, const float *boxes, hipStream_t s);

// Interleave the uploaded arrays into the 48-byte layout.
hipError_t gauss_pack_launch(const GaussArrays &a, float4 *out, hipStream_t s);
// Validation of an uploaded set: flags[0] |= 1 non-finite value, 2 scale
// <= 0, 4 zero quaternion, 8 opacity outside [0, 1].
hipError_t gauss_validate_launch(const GaussParams &p, int32_t *flags, hipStream_t s);
// Gaussian boxes (float32 [n][6]) for cutoff k.
hipError_t gauss_boxes_launch(const GaussParams &p, float k, float *boxes, hipStream_t s);
// Evaluation records in leaf order.
hipError_t gauss_records_launch(const GaussParams &p, const uint32_t *sorted, GaussRec *recs,
                                hipStream_t s);
// Density / occupancy (mode 0) or culling-set sizes per tile (mode 1).
hipError_t voxelize_launch(int mode, const NodeRec *nodes, const GaussRec *recs,
                           const float *boxes, int64_t n_gauss, const VoxGrid &g,
                           float *density, uint8_t *occ, int32_t *tile_counts, hipStream_t s);
// Surface mask from occupancy.
hipError_t surface_launch(const uint8_t *occ, uint8_t *surf, const VoxGrid &g, hipStream_t s);
