/*
 * rcast_calib.h -- calibration kernels of librcast.
 *
 * The ray-casting cost model of FGGS-LiDAR (Sec. IV-C: the cost of a ray is
 * a per-node cost times the nodes it visits plus a per-triangle cost times
 * the triangles it tests) prices a ray in records fetched and tests run.
 * Whether those records come from HBM or from the caches, and how fast the
 * vector ALUs can run the tests, is a property of the chip that has to be
 * measured.  These two calls measure it on the device they run on, so the
 * traversal can be reported as a fraction of ceilings that it could in
 * principle reach.  Neither touches a context; both are stream-ordered and
 * return once the kernel is enqueued.  Errors: RC_E_INVAL for a bad argument
 * (nothing launched), RC_E_DEVICE when the launch fails; rc_last_error()
 * gives the text.
 */
#ifndef RCAST_CALIB_H
#define RCAST_CALIB_H

#include <stdint.h>

#include "rcast.h"

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Random 64-byte record gathers.  `records` (device, 64-byte aligned, owned
 * by the caller, at least n_records * 64 bytes, contents arbitrary) is read
 * as n_records records of 64 bytes; each of n_lanes lanes (a multiple of
 * 256, at most 2^31 * 256) reads `iters` x 4 records at seeded pseudo-random
 * indices, four at a time and independent of the data read, each record as
 * four 16-byte loads, the access pattern of one node-record fetch of the
 * traversal.  Bytes read = n_lanes * iters * 256.  `sink` (device, >= 4 KiB)
 * receives at most a few words so the loads cannot be dropped.
 * n_records must be in [1, 2^32 - 1].
 */
rc_status rc_calib_gather(const void *records, uint64_t n_records, int64_t n_lanes,
                          int32_t iters, uint32_t *sink, void *stream);

/*
 * Independent FP32 vector operations: n_lanes lanes (a multiple of 256) each
 * run `iters` iterations over eight independent chains.  mix 0: 32 FMAs per
 * iteration; mix 1: per chain one byte-to-float conversion, one FMA, one
 * maximum, one minimum, one compare and a select (the classes of a node
 * test).  The instruction count is read from hardware counters of a
 * profiled run; `sink` (device, >= 4 KiB) keeps the result live.
 */
rc_status rc_calib_valu(int64_t n_lanes, int32_t iters, int32_t mix, float *sink, void *stream);

#ifdef __cplusplus
}
#endif

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#endif /* RCAST_CALIB_H */
