#!/usr/bin/env python3
"""Benchmark: batched LiDAR ray casting on one MI355X.

Workload (one step): 4096 environments sharing the closed indoor mesh of
about one million triangles (room + 200 primitives, marching cubes at 3.5 cm),
each with a seeded free-space pose (yaw uniform), 32 x 1024 beams
(-16..+15 deg elevation) -> 134,217,728 rays, range [0.1, 120] m.

A step is the whole hot path on inputs already resident in HBM: the LBVH
build over the mesh (triangle boxes, Morton codes, radix sort, hierarchy,
refit, leaf-order records, 4-wide quantised nodes) followed by one batched
ray-cast launch (autotuned launch shape, replayed from a hipGraph) writing
range and hit id for every ray.  ``value`` = rays per step / step time.  The
same is timed with plain FP32 nodes and reported under ``forms``.

Also reported:
  * roofline -- algorithmic bytes of the traversal kernel per launch
    (rays * (64 * mean node records fetched + 40 * mean triangles tested + 8),
    the per-ray cost model of FGGS-LiDAR Sec. IV-C with canonical record
    sizes; the means come from an instrumented pass over every ray) divided
    by the kernel's mean duration (HIP events on its stream), against 8 TB/s;
  * cpu_baseline -- the FP64 oracle timed on this host's cores on a seeded
    sample of the same rays, scaled to Mrays/s.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES, OUT_BYTES = 64, 40, 8
# FP32 vector issue of one MI355X: 256 CUs x 4 SIMDs x 32 lanes per cycle at
# 2.4 GHz = 78.64 T lane-instructions/s (the published 157.3 TFLOP/s FP32
# vector peak counts an FMA lane-instruction as 2 flops); a wave64 vector
# instruction occupies its SIMD for 2 cycles, so 1,228.8 G wave-instructions/s
LANE_PEAK_T = 256 * 4 * 32 * 2.4e9 / 1e12
VALU_PEAK_GWI = LANE_PEAK_T * 1e3 / 64
# calibration launches: lanes (8 waves per SIMD on 256 CUs x 4 SIMDs, four
# times over) and iterations per lane
CALIB_LANES = 256 * 4 * 8 * 64 * 4
CALIB_GATHER_ITERS = 32
CALIB_VALU_ITERS = 2048


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(files=("trace.hip", "rc_internal.h")) -> str:
    """Hash of a kernel's code (by default the traversal: trace.hip and
    rc_internal.h) with comments and whitespace removed, so profiled counters
    stay attached to the code they were measured on, not to its comments."""
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_17390_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel_hash: str, rays: int, tris: int, tuning: dict):
    """Counters of the traversal kernel measured by rocprofv3 (profiles/):
    HBM bytes per launch, L2 hit rate, VALU utilisation.  None when absent or
    taken on a different kernel code, workload or kernel variant."""
    p = os.path.join(ROOT, "profiles", "trace_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    # the kernel variant is fixed by these fields (the packet tile only
    # reorders the rays of the same kernel)
    variant = ("persistent", "stack_lds", "waves_cap", "group_waves", "leaf_batch")
    t0 = d.get("tuning") or {}
    if (d.get("kernel_hash") != kernel_hash or d.get("rays") != rays
            or d.get("tris") != tris or any(t0.get(k) != tuning.get(k) for k in variant)):
        return None
    return d


MESH_KERNEL_FILES = ("tsdf.hip", "vox.hip", "mesh_internal.h", "rc_internal.h")


def load_mesh_traffic(n_vox: int):
    """HBM bytes of one TSDF + marching-cubes call measured by rocprofv3
    (profiles/tsdf_traffic.json); None when absent or taken on other kernel
    code or another grid."""
    p = os.path.join(ROOT, "profiles", "tsdf_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_source_hash(MESH_KERNEL_FILES) or d.get("voxels") != n_vox:
        return None
    return d


def load_cost_model():
    """Vector-instruction cost of the Q8 traversal per unit of the paper's
    cost model (Sec. IV-C: cost = C_trav N_nodes + C_tri K per ray), measured
    with coherent waves (64 copies of one ray per wave, so a wave's
    instruction count is one ray's) and fitted over eight dispatches:
    lane-instructions per ray (set-up and output), per node visit and per
    triangle test (profiles/trace_cost_model.json, `bench.py --workload
    costmodel`).  None when absent."""
    p = os.path.join(ROOT, "profiles", "trace_cost_model.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    d["kernel_hash_matches"] = d.get("kernel_hash") == kernel_source_hash()
    return d


def alu_roofline(cm, rays, mean_nodes, mean_tris, kernel_ms):
    """ALU roofline of the traversal: the cost model's lane-instructions per
    ray (C_ray + C_node N + C_tri K, with N and K the kernel's own mean node
    visits and triangle tests from the instrumented pass) times the rays of one
    launch, over the launch's time, against the chip's lane-instruction peak.
    Idle lanes (divergence) and issue stalls are what separates it from 1."""
    if cm is None:
        return None
    per_ray = cm["C_ray"] + cm["C_node"] * mean_nodes + cm["C_tri"] * mean_tris
    ach = per_ray * rays / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": round(LANE_PEAK_T, 3),
            "unit": "T lane-instructions/s", "frac": round(ach / LANE_PEAK_T, 4),
            "lane_instructions_per_ray": round(per_ray, 1),
            "cost_model": {k: cm[k] for k in ("C_ray", "C_node", "C_tri", "kernel_hash",
                                              "kernel_hash_matches")}}


def load_calib_counters():
    """Vector-instruction counts of the calibration kernels (rocprofv3
    SQ_INSTS_VALU per launch, profiles/calib_counters.json), valid while the
    calibration source is unchanged; None otherwise."""
    p = os.path.join(ROOT, "profiles", "calib_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("calib_hash") != kernel_source_hash(("calib.hip",)):
        return None
    if d.get("lanes") != CALIB_LANES or d.get("valu_iters") != CALIB_VALU_ITERS:
        return None
    return d


def calibrate(torch, dev, stream, scene_record_bytes, reps=5):
    """Measured ceilings of this device (rc_calib_gather / rc_calib_valu),
    each the best of `reps` launches timed with HIP events on the launch
    stream: random 64-byte record gathers from an L2-resident working set
    (2 MiB), from one the size of the scene's node and triangle records, and
    from 4 GiB (HBM); FP32 vector-instruction issue for the FMA-only and the
    node-test mixes (instruction counts from the profiled counters)."""
    from paper_2509_17390_amd import rcast
    lib = rcast.load()
    sp = ctypes_void(stream.cuda_stream)
    sink = torch.empty(1024, dtype=torch.int32, device=dev)
    out = {}

    def timed(fn):
        best = float("inf")
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return best

    sets = (("l2_2MiB", 2 << 20), ("scene_records", int(scene_record_bytes)),
            ("hbm_4GiB", 4 << 30))
    for name, nbytes in sets:
        n_rec = max(nbytes // 64, 1)
        buf = torch.ones(n_rec * 16, dtype=torch.float32, device=dev)

        def g():
            rcast._check(lib.rc_calib_gather(buf.data_ptr(), n_rec, CALIB_LANES,
                                             CALIB_GATHER_ITERS, sink.data_ptr(), sp))
        g()
        ms = timed(g)
        gb = CALIB_LANES * CALIB_GATHER_ITERS * 256 / (ms * 1e-3) / 1e9
        out[f"gather_{name}"] = {"working_set_MB": round(n_rec * 64 / 1e6, 1),
                                 "ms": round(ms, 4), "GB_s": round(gb, 1)}
        del buf
    counters = load_calib_counters()
    for mix in (0, 1):
        def v():
            rcast._check(lib.rc_calib_valu(CALIB_LANES, CALIB_VALU_ITERS, mix, sink.data_ptr(),
                                           sp))
        v()
        ms = timed(v)
        ent = {"ms": round(ms, 4)}
        if counters is not None:
            insts = counters[f"valu_mix{mix}_insts"]
            ent["wave_insts"] = insts
            ent["G_wave_insts_s"] = round(insts / (ms * 1e-3) / 1e9, 1)
        out[f"valu_mix{mix}"] = ent
    torch.cuda.synchronize()
    return out


def ctypes_void(p):
    import ctypes
    return ctypes.c_void_p(int(p))


def cpu_baseline(verts, tris, poses, dirs, t_min, t_max, g_range, g_hit, budget_s, seed):
    import oracle
    rng = np.random.default_rng(seed)
    n_rays = len(poses) * len(dirs)
    threads = oracle.default_threads()
    calib = np.sort(rng.choice(n_rays, threads * 4, replace=False))
    t0 = time.perf_counter()
    oracle.raycast(verts, tris, poses, dirs, t_min, t_max, ray_idx=calib, threads=threads)
    per_ray = (time.perf_counter() - t0) / len(calib)
    n = int(min(max(budget_s / per_ray, threads * 8), 1 << 16))
    idx = np.sort(rng.choice(n_rays, n, replace=False))
    t0 = time.perf_counter()
    t, ids = oracle.raycast(verts, tris, poses, dirs, t_min, t_max, ray_idx=idx, threads=threads)
    dt = time.perf_counter() - t0
    # agreement of the GPU result on the same rays (unflagged parity needs the
    # checker; here: exact ids and range within tolerance, as a sanity count)
    gh, gr = g_hit[idx], g_range[idx]
    same_id = int((gh == ids).sum())
    ok = (gh == ids) & (ids >= 0)
    err = np.abs(gr[ok].astype(np.float64) - t[ok])
    rng_ok = int((err <= 1e-4 + 1e-6 * t[ok]).sum())
    return {
        "value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
        "sample": f"{n} seeded rays of the same workload (all envs/beams), FP64 brute force "
                  f"over all {len(tris)} triangles, {dt:.1f} s",
        "gpu_agreement": {"rays": n, "same_id": same_id, "range_ok_of_same_id_hits": rng_ok,
                          "hits": int((ids >= 0).sum()),
                          "max_range_err_m": float(err.max()) if err.size else 0.0,
                          "max_rel_range_err": float((err / t[ok]).max()) if err.size else 0.0},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--envs", type=int, default=0, help="environments (0: the stored workload's)")
    ap.add_argument("--h", type=float, default=None,
                    help="marching-cubes spacing in m (default: the stored workload's)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape (profiling runs)")
    ap.add_argument("--workload", choices=("batched", "uneven", "serve", "frame", "voxelize",
                                           "mesh", "costmodel"),
                    default="batched",
                    help="batched: 4096 envs on the 1M-triangle mesh (default); uneven: 64 "
                         "resident terrains, 1024 envs, mixed patterns in one launch; serve: "
                         "Poisson requests against 16 resident scenes, served vs per-request; "
                         "frame: one sensor, 128x2048 beams, 6.4M-triangle mesh, frames/s")
    ap.add_argument("--scenes", type=int, default=0, help="uneven/serve: scene count override")
    ap.add_argument("--requests", type=int, default=1000, help="serve: requests per rate")
    ap.add_argument("--rates", type=str, default="0.1,0.3,0.5,0.7,0.9,1.1",
                    help="serve: arrival rates as fractions of the measured capacity")
    ap.add_argument("--batch-cap-m", type=int, default=64,
                    help="serve: most rays per batched launch, in millions (0: no cap)")
    ap.add_argument("--inflight", type=int, default=3, help="serve: launches in flight")
    ap.add_argument("--policy", type=int, default=0,
                    help="serve: admission order, 0 arrival order, 1 fewest rays first with aging")
    ap.add_argument("--max-wait-ms", type=int, default=0,
                    help="serve, policy 1: age after which a request goes first (0: 200 ms)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving block")
    ap.add_argument("--uneven-rays-per-job", type=int, default=0,
                    help="uneven: oracle rays sampled per job (0: the stored workload's)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="default run: requests per rate of the serving block")
    ap.add_argument("--tuning", type=str, default="",
                    help='batched: fixed launch shape instead of the autotuner, as JSON '
                         'rc_tuning fields, e.g. {"leaf_batch": 32}')
    ap.add_argument("--ingest", type=str, default="",
                    help="write profiles/*.json from rocprofv3 output: 'costmodel:<run dir>' "
                         "or 'traffic:<run dir>' (see profiles/*.md for the runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        return 2

    if args.workload == "uneven":
        return run_uneven(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "frame":
        return run_frame(args)
    if args.workload == "voxelize":
        return run_voxelize(args)
    if args.workload == "mesh":
        return run_mesh(args)
    if args.workload == "costmodel":
        return run_costmodel(args)
    if args.ingest:
        return ingest(args.ingest)

    import torch
    import synth
    from paper_2509_17390_amd import Context, Job

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda", 0)
    log("building scene ...")
    wc = synth.workload_config("batched_4096")
    h_mesh = args.h if args.h is not None else wc["h"]
    s = synth.indoor_scene(seed=wc["mesh_seed"], h=h_mesh, n_envs=args.envs or wc["envs"],
                           pose_seed=wc["pose_seed"])
    n_rays = s.n_rays
    log(f"mesh: {len(s.tris)} tris, {len(s.verts)} verts; rays/step {n_rays}")

    ctx = Context(0)
    verts_d = torch.from_numpy(s.verts).to(dev)
    tris_d = torch.from_numpy(s.tris).to(dev)
    scene = ctx.upload_scene(verts_d, tris_d)          # inputs resident in HBM
    pat = ctx.upload_pattern(s.dirs, s.n_az)
    poses_d = torch.from_numpy(s.poses).to(dev)
    out_r = torch.empty(n_rays, dtype=torch.float32, device=dev)
    out_h = torch.empty(n_rays, dtype=torch.int32, device=dev)
    job = [Job(scene, pat, poses_d, s.t_min, s.t_max, 0)]
    stream = torch.cuda.current_stream()

    forms = {}
    outputs = {}
    for name, fmt in (("fp32", 0), ("q8", 1)):
        # setup (untimed): build this form, autotune the launch shape on the
        # real batch, capture the launch in a graph
        ctx.build(scene, node_format=fmt, stream=stream)
        torch.cuda.synchronize()
        if args.tuning:
            ctx.reset_tuning()
            ctx.set_tuning(**json.loads(args.tuning))
            best, tune_ms = ctx.get_tuning(), float("nan")
        elif args.no_autotune:
            ctx.reset_tuning()
            best, tune_ms = ctx.get_tuning(), float("nan")
        else:
            best, tune_ms = ctx.autotune(job, out_r, out_h, reps=2, stream=stream)
        graph = ctx.graph(job, out_r, out_h)

        def step(ev=None):
            ctx.build(scene, node_format=fmt, stream=stream)
            if ev is not None:
                ev[0].record(stream)
            graph.launch(stream)
            if ev is not None:
                ev[1].record(stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(evs[i])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms_step = dt * 1e3 / args.steps
        trace_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        graph.close()
        outputs[name] = (out_r.clone(), out_h.clone())
        forms[name] = {"ms_per_step": round(ms_step, 3), "Mrays_s": round(n_rays / ms_step / 1e3, 2),
                       "frame_ms": round(trace_ms, 3),
                       "frame_Mrays_s": round(n_rays / trace_ms / 1e3, 2),
                       "build_ms": round(ms_step - trace_ms, 3), "tuning": best,
                       "autotune_best_ms": None if tune_ms != tune_ms else round(tune_ms, 3)}
        log(f"{name}: step {ms_step:.2f} ms, traversal {trace_ms:.2f} ms, tuning {best}")
    info = ctx.scene_info(scene)
    same_forms = bool(torch.equal(outputs["fp32"][1], outputs["q8"][1]) and
                      torch.equal(outputs["fp32"][0].view(torch.int32),
                                  outputs["q8"][0].view(torch.int32)))
    head = "q8"
    ms_step = forms[head]["ms_per_step"]
    trace_ms = forms[head]["frame_ms"]
    out_r, out_h = outputs[head]

    if args.calib_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written, so byte
        # counters of the traversal kernel can be scaled to bytes
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # instrumented passes (untimed): node records fetched and triangles
    # tested per ray.  The cost-model bytes use the plain FP32 tree for both
    # forms (the same denominator), so fewer bytes in the Q8 form show as a
    # gain; the Q8 form's own record counts are reported beside it.
    def stats(fmt):
        ctx.build(scene, node_format=fmt, stream=stream)
        nn = torch.empty(n_rays, dtype=torch.int32, device=dev)
        nt = torch.empty(n_rays, dtype=torch.int32, device=dev)
        r2 = torch.empty_like(out_r)
        h2 = torch.empty_like(out_h)
        ctx.raycast(job, r2, h2, stream=stream, mode="stats", out_nodes=nn, out_tris=nt)
        torch.cuda.synchronize()
        return float(nn.double().mean()), float(nt.double().mean()), bool(torch.equal(h2, out_h))

    mean_nodes, mean_tris, same = stats(0)
    q8_nodes, q8_tris, same_q8 = stats(1)
    # cost-model bytes of the timed kernel: its own (Q8) record counts with
    # the canonical record sizes
    b_ray = NODE_BYTES * q8_nodes + TRI_BYTES * q8_tris + OUT_BYTES
    b_ray_fp32 = NODE_BYTES * mean_nodes + TRI_BYTES * mean_tris + OUT_BYTES
    alg_bytes = b_ray * n_rays
    achieved = alg_bytes / (trace_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    cost_model = load_cost_model()
    counters = load_traffic(khash, n_rays, int(len(s.tris)), forms["q8"]["tuning"])
    traffic = counters["bytes_per_launch"] if counters else None
    rec_bytes = 64 * info.n_q8_nodes + 48 * info.n_tris
    log("calibrating gather and issue ceilings ...")
    cal = calibrate(torch, dev, stream, rec_bytes)
    l2_peak = cal["gather_l2_2MiB"]["GB_s"]
    valu_peak = max(cal[f"valu_mix{m}"].get("G_wave_insts_s", 0.0) for m in (0, 1)) or None

    g_range = out_r.cpu().numpy()
    g_hit = out_h.cpu().numpy()
    misses = int((g_hit < 0).sum())
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(s.verts, s.tris, s.poses, s.dirs, s.t_min, s.t_max, g_range, g_hit,
                           args.cpu_budget, wc["oracle_sample_seed"])
    ctx.close()
    del outputs, out_r, out_h, graph
    torch.cuda.empty_cache()

    serving = None
    if not args.no_serve:
        serving = serve_measure(16, args.serve_requests, [0.5, 0.9], args.inflight,
                                args.batch_cap_m, args.policy, args.max_wait_ms)

    valu = None
    if counters is not None:
        v_ach = counters["valu_insts_per_wave"] * (n_rays / 64) / (trace_ms * 1e-3) / 1e9
        valu = {"achieved": round(v_ach, 1), "unit": "G wave-instructions/s",
                "peak": round(VALU_PEAK_GWI, 1), "frac": round(v_ach / VALU_PEAK_GWI, 4),
                "calibrated_ceiling": valu_peak,
                "calibrated_source": "rc_calib_valu, independent FP32 FMAs",
                "active_lanes_of_64": counters["valu_active_threads"],
                "insts_per_wave": counters["valu_insts_per_wave"]}
    hbm = None
    if traffic is not None:
        h_ach = traffic / (trace_ms * 1e-3) / 1e9
        hbm = {"achieved": round(h_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(h_ach / HBM_PEAK_GBS, 4),
               "source": "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by a 1 GiB copy"}

    value = n_rays / (ms_step * 1e-3) / 1e6
    out = {
        "metric": "Mrays/s at 4096 envs x 32x1024 beams, 1M tris; p50/p99 request latency",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched raycast: {len(s.poses)} envs x 32x1024 beams on a "
                        f"{len(s.tris)}-triangle closed indoor mesh (marching cubes at "
                        f"{h_mesh} m), step = LBVH build (Q8 nodes) + one graph-captured "
                        f"batched launch; serving: Poisson requests on 16 resident terrains",
            "node_format": "q8",
            "envs": int(len(s.poses)), "beams": int(len(s.dirs)), "tris": int(len(s.tris)),
            "seeds": "synth/configs/batched_4096.json",
            "rays_per_step": int(n_rays), "t_range": [s.t_min, s.t_max],
        },
        "frame_only": {"ms": round(trace_ms, 3),
                       "Mrays_s": round(n_rays / (trace_ms * 1e-3) / 1e6, 2)},
        "build_ms": round(ms_step - trace_ms, 3),
        "forms": forms,
        "forms_bit_identical": same_forms,
        # the traversal is bound by vector issue and lane divergence, not by
        # memory: its node and triangle records stay in L2 and MALL.  The
        # roofline is therefore the ALU one -- the cost model's
        # lane-instructions per launch over the kernel's time, against the
        # chip's lane-instruction peak; the cost model's bytes are reported
        # beside it as demand (served mostly by the caches, so above any
        # memory level's bandwidth), with the HBM traffic the counters measure
        "roofline": dict(alu_roofline(cost_model, n_rays, q8_nodes, q8_tris, trace_ms) or
                         {"bound": "alu", "achieved": None, "peak": round(LANE_PEAK_T, 3),
                          "unit": "T lane-instructions/s", "frac": None}, **{
            "traffic": traffic,
            "kernel": "k_trace<TRACE_BVH, FMT_Q8> (graph replay)",
            "q8_mean_node_records": round(q8_nodes, 2),
            "q8_mean_tri_tests": round(q8_tris, 2),
            "demand_bytes": {"bytes_per_ray": round(b_ray, 1), "GB_s": round(achieved, 1),
                             "l2_gather_ceiling_GB_s": l2_peak,
                             "note": "cost-model bytes (64 B per node record, 40 B per "
                                     "triangle, 8 B output): lanes of a wave share most "
                                     "records, so this exceeds what any memory level "
                                     "delivers and is not a roofline fraction"},
            "fp32_tree": {"bytes_per_ray": round(b_ray_fp32, 1),
                          "mean_node_records": round(mean_nodes, 2),
                          "mean_tri_tests": round(mean_tris, 2)},
            "kernel_hash": khash,
            "hbm": hbm,
            "valu": valu,
            "calibration": cal,
            "counters": None if counters is None else {
                k: counters.get(k) for k in ("hbm_GBs", "l2_hit_pct", "valu_util_pct",
                                             "valu_active_threads", "valu_insts_per_wave",
                                             "vmem_insts_per_wave", "ta_busy_pct",
                                             "td_busy_pct", "read_bytes", "write_bytes")},
        }),
        "cpu_baseline": cpu,
        "misses": misses,
        "stats_pass_matches": same and same_q8,
        "bvh_depth": info.depth,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    return 0


def _stats_bytes(ctx, jobs, n_rays, torch, dev, stream):
    """Mean node records / triangle tests per ray of the current launch form."""
    nn = torch.empty(n_rays, dtype=torch.int32, device=dev)
    nt = torch.empty(n_rays, dtype=torch.int32, device=dev)
    r = torch.empty(n_rays, dtype=torch.float32, device=dev)
    h = torch.empty(n_rays, dtype=torch.int32, device=dev)
    ctx.raycast(jobs, r, h, stream=stream, mode="stats", out_nodes=nn, out_tris=nt)
    torch.cuda.synchronize()
    return float(nn.double().mean()), float(nt.double().mean())


def uneven_oracle_leg(w, jobs, job_meta, q8_out, per_job, seed):
    """The FP64 oracle (with its checker flags) on `per_job` seeded rays of
    every job of the uneven batch -- every scene, the multi-million-triangle
    ones included -- timed on this host's cores and compared with the GPU's
    Q8 results under the parity bar: on rays the checker does not flag,
    hit/miss agreement, equal ids and |range error| <= 1e-4 + 1e-6 t; on
    flagged rays the GPU range may not exceed the oracle's nearest hit by
    more than 1e-3 + 1e-5 t.  Counts only; the GPU tests assert."""
    import oracle
    g_r = q8_out[0].cpu().numpy()
    g_h = q8_out[1].cpu().numpy()
    rng = np.random.default_rng(seed)
    threads = oracle.default_threads()
    tot = {"rays": 0, "clean": 0, "edge_near": 0, "ambiguous": 0, "bad_hitmiss": 0,
           "bad_id": 0, "bad_range": 0, "flagged_beyond_nearest": 0, "max_range_err_m": 0.0}
    tris_tested = 0
    t0 = time.perf_counter()
    for j, (k, pi, idx) in zip(jobs, job_meta):
        n = len(idx) * len(w.patterns[pi])
        sel = np.sort(rng.choice(n, min(n, per_job), replace=False))
        v, tr = w.scenes[k]
        t, ids, flags, _, _ = oracle.raycast(v, tr, w.poses[idx], w.patterns[pi], w.t_min,
                                             w.t_max, ray_idx=sel, threads=threads, checked=True)
        gr = g_r[j.out_offset + sel].astype(np.float64)
        gh = g_h[j.out_offset + sel]
        clean = flags == 0
        oh = ids >= 0
        tol = 1e-4 + 1e-6 * np.where(oh, t, 0.0)
        err = np.where(oh & (gh >= 0), np.abs(gr - np.where(oh, t, 0.0)), 0.0)
        tot["rays"] += len(sel)
        tot["clean"] += int(clean.sum())
        tot["edge_near"] += int((flags & 1).sum())
        tot["ambiguous"] += int((flags & 2).sum())
        tot["bad_hitmiss"] += int((clean & (oh != (gh >= 0))).sum())
        tot["bad_id"] += int((clean & oh & (gh != ids)).sum())
        tot["bad_range"] += int((clean & oh & (gh == ids) & ~(err <= tol)).sum())
        tot["flagged_beyond_nearest"] += int((~clean & oh & (gh >= 0) &
                                              (gr > t + 1e-3 + 1e-5 * np.abs(t))).sum())
        if (clean & oh).any():
            tot["max_range_err_m"] = max(tot["max_range_err_m"], float(err[clean & oh].max()))
        tris_tested += len(sel) * len(tr)
    dt = time.perf_counter() - t0
    return {"value": tot["rays"] / dt / 1e6, "unit": "Mrays/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{per_job} seeded rays from each of the {len(jobs)} jobs (all scenes), "
                      f"FP64 brute force with checker flags, {tris_tested / tot['rays']:.0f} "
                      f"triangles per ray on average, {dt:.1f} s",
            "gpu_agreement": tot}


def run_uneven(args):
    """64 resident terrain scenes (50k..5M triangles, log-uniform), 1024
    environments each bound to a random scene and one of three beam patterns
    (16x360, 64x1024, 128x2048), cast in one batched launch.  Scenes and
    BVHs are resident (built once, timed separately); a step is one launch."""
    import torch
    import synth
    from paper_2509_17390_amd import Context, Job

    dev = torch.device("cuda", 0)
    wc = synth.workload_config("uneven_64")
    n_scenes = args.scenes or wc["scenes"]
    log(f"generating {n_scenes} terrains ...")
    w = synth.uneven_world(seed=wc["world_seed"], n_scenes=n_scenes, n_envs=wc["envs"],
                           tri_lo=wc["tris_range"][0], tri_hi=wc["tris_range"][1])
    tris_total = int(sum(len(t) for _, t in w.scenes))
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    sids = [ctx.upload_scene(v, t) for v, t in w.scenes]
    pids = [ctx.upload_pattern(d, na) for d, na in zip(w.patterns, w.n_az)]
    # one job per (scene, pattern) group of environments
    jobs, job_meta, off = [], [], 0
    poses_keep = []
    for k in range(n_scenes):
        for pi in range(len(w.patterns)):
            idx = np.flatnonzero((w.env_scene == k) & (w.env_pattern == pi))
            if len(idx) == 0:
                continue
            pt = torch.from_numpy(w.poses[idx]).to(dev)
            poses_keep.append(pt)
            jobs.append(Job(sids[k], pids[pi], pt, w.t_min, w.t_max, off))
            job_meta.append((k, pi, idx))
            off += len(idx) * len(w.patterns[pi])
    n_rays = off
    out_r = torch.empty(n_rays, dtype=torch.float32, device=dev)
    out_h = torch.empty(n_rays, dtype=torch.int32, device=dev)
    forms, outputs = {}, {}
    for name, fmt in (("fp32", 0), ("q8", 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sid in sids:
            ctx.build(sid, node_format=fmt, stream=stream)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        best, _ = ctx.autotune(jobs, out_r, out_h, reps=1, stream=stream)
        graph = ctx.graph(jobs, out_r, out_h)
        for _ in range(args.warmup):
            graph.launch(stream)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            graph.launch(stream)
            b.record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        graph.close()
        outputs[name] = (out_r.clone(), out_h.clone())
        nodes, tt = _stats_bytes(ctx, jobs, n_rays, torch, dev, stream)
        forms[name] = {"ms_per_step": round(ms, 3), "Mrays_s": round(n_rays / ms / 1e3, 2),
                       "kernel_ms": round(kms, 3), "build_all_scenes_ms": round(build_ms, 1),
                       "tuning": best, "mean_node_records": round(nodes, 2),
                       "mean_tri_tests": round(tt, 2)}
        log(f"uneven {name}: {ms:.2f} ms/launch, {forms[name]['Mrays_s']} Mrays/s")
    same = bool(torch.equal(outputs["fp32"][1], outputs["q8"][1]) and
                torch.equal(outputs["fp32"][0].view(torch.int32), outputs["q8"][0].view(torch.int32)))
    b_ray = NODE_BYTES * forms["q8"]["mean_node_records"] + TRI_BYTES * forms["q8"]["mean_tri_tests"] + OUT_BYTES
    kms = forms["q8"]["kernel_ms"]
    achieved = b_ray * n_rays / (kms * 1e-3) / 1e9
    scene_rec = max(64 * ctx.scene_info(sid).n_q8_nodes + 48 * ctx.scene_info(sid).n_tris
                    for sid in sids)
    cal = calibrate(torch, dev, stream, scene_rec)
    l2_peak = cal["gather_l2_2MiB"]["GB_s"]
    cpu = None
    if not args.no_cpu:
        log("oracle leg: seeded rays of every job, checker flags ...")
        cpu = uneven_oracle_leg(w, jobs, job_meta, outputs["q8"],
                                args.uneven_rays_per_job or wc["oracle_rays_per_job"],
                                wc["oracle_sample_seed"])
    out = {
        "metric": "Mrays/s, uneven batch: 64 resident scenes, 1024 envs, mixed patterns, one launch",
        "value": forms["q8"]["Mrays_s"], "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": forms["q8"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n_scenes} terrains ({tris_total} triangles in total), 1024 envs "
                               f"over {len(jobs)} jobs, patterns 16x360 / 64x1024 / 128x2048, "
                               f"step = one graph-replayed launch on resident Q8 BVHs",
                   "scenes": n_scenes, "tris_total": tris_total, "envs": 1024, "jobs": len(jobs),
                   "rays_per_step": int(n_rays), "node_format": "q8"},
        "forms": forms, "forms_bit_identical": same,
        "roofline": dict(alu_roofline(load_cost_model(), n_rays,
                                      forms["q8"]["mean_node_records"],
                                      forms["q8"]["mean_tri_tests"], kms) or
                         {"bound": "alu", "achieved": None, "peak": round(LANE_PEAK_T, 3),
                          "unit": "T lane-instructions/s", "frac": None},
                         traffic=None,
                         demand_bytes={"bytes_per_ray": round(b_ray, 1),
                                       "GB_s": round(achieved, 1),
                                       "l2_gather_ceiling_GB_s": l2_peak},
                         calibration=cal),
        "cpu_baseline": cpu,
        "misses": int((outputs["q8"][1] < 0).sum()),
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def run_costmodel(args):
    """Coherent-wave dispatches for the traversal's cost model (run under
    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU ...): 4,096 beams of the headline
    pattern from 16 poses on the headline mesh, Q8 nodes, plain beam order;
    the directions are ranked by their node and triangle counts and cut into
    eight buckets, and each bucket is cast as one dispatch in which every
    beam is repeated 64 times, so each wave casts 64 copies of one ray and
    its vector-instruction count is that ray's.  Prints one JSON line per
    dispatch with its waves, node visits and triangle tests."""
    import torch
    import synth
    from paper_2509_17390_amd import Context, Job

    wc = synth.workload_config("batched_4096")
    s = synth.indoor_scene(seed=wc["mesh_seed"], h=wc["h"], n_envs=16, pose_seed=wc["pose_seed"])
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    scene = ctx.upload_scene(s.verts, s.tris)
    ctx.build(scene, node_format=1)
    ctx.set_tuning(tile_az=0, tile_el=0)
    poses = torch.from_numpy(s.poses).to(dev)
    rng = np.random.default_rng(5)
    cand = np.ascontiguousarray(s.dirs[rng.choice(len(s.dirs), 4096, replace=False)])
    pat1 = ctx.upload_pattern(cand, 0)
    _, _, nn, nt = ctx.cast([Job(scene, pat1, poses, s.t_min, s.t_max, 0)], mode="stats")
    nn = nn.cpu().numpy().reshape(16, 4096).astype(np.int64)
    nt = nt.cpu().numpy().reshape(16, 4096).astype(np.int64)
    order = np.argsort(nn.mean(0) + 5 * nt.mean(0), kind="stable")
    for b in range(8):
        sel = order[b * 512:(b + 1) * 512]
        pat = ctx.upload_pattern(np.ascontiguousarray(np.repeat(cand[sel], 64, axis=0)), 0)
        ctx.cast([Job(scene, pat, poses, s.t_min, s.t_max, 0)])
        torch.cuda.synchronize()
        print(json.dumps({"dispatch": b, "waves": 16 * 512, "sum_nodes": int(nn[:, sel].sum()),
                          "sum_tris": int(nt[:, sel].sum())}), flush=True)
    ctx.close()
    return 0


def _counter_rows(path, name_has):
    """{dispatch id: {counter: value}} for kernels whose name contains
    name_has, from a rocprofv3 counter_collection.csv."""
    import csv
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if name_has in r["Kernel_Name"]:
                out.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = \
                    float(r["Counter_Value"])
    return out


def _find_csv(run_dir, tag):
    for dp, _, fs in os.walk(run_dir):
        for f in fs:
            if f.endswith("counter_collection.csv") and tag in os.path.join(dp, f):
                return os.path.join(dp, f)
    raise FileNotFoundError(f"no counter_collection.csv for '{tag}' under {run_dir}")


def ingest(spec):
    """Turn rocprofv3 runs (made with the commands in profiles/*.md) into the
    JSON files bench.py reads: 'costmodel:<dir>' fits the traversal's cost
    model; 'traffic:<dir>' writes the headline kernel's counters."""
    kind, _, run_dir = spec.partition(":")
    if kind == "costmodel":
        rows = _counter_rows(_find_csv(run_dir, "cm"), "k_trace<0, 1")
        lines = [json.loads(l) for l in open(os.path.join(run_dir, "cm.log"))
                 if l.startswith("{")]
        disp = sorted(rows)
        assert len(disp) == len(lines) == 8, (len(disp), len(lines))
        a = np.array([[l["waves"], l["sum_nodes"], l["sum_tris"]] for l in lines], np.float64)
        y = np.array([rows[d]["SQ_INSTS_VALU"] for d in disp])
        assert all(rows[d]["SQ_WAVES"] == l["waves"] for d, l in zip(disp, lines))
        x = np.linalg.lstsq(a, y, rcond=None)[0]
        res = float(np.abs(a @ x - y).max() / y.mean())
        out = {"C_ray": round(float(x[0]), 1), "C_node": round(float(x[1]), 1),
               "C_tri": round(float(x[2]), 1), "fit_max_rel_residual": res,
               "kernel_hash": kernel_source_hash(),
               "dispatches": [{"waves": l["waves"], "sum_nodes": l["sum_nodes"],
                               "sum_tris": l["sum_tris"],
                               "SQ_INSTS_VALU": rows[d]["SQ_INSTS_VALU"]}
                              for d, l in zip(disp, lines)],
               "note": "lane-instructions (= wave-instructions of a coherent wave) per ray, "
                       "per Q8 node visit and per triangle test; least squares over the "
                       "dispatches of bench.py --workload costmodel"}
        path = os.path.join(ROOT, "profiles", "trace_cost_model.json")
    elif kind == "traffic":
        def one(tag, name):
            rows = _counter_rows(_find_csv(run_dir, tag), name)
            keys = sorted(rows)
            return {c: float(np.mean([rows[k][c] for k in keys])) for c in rows[keys[0]]}, len(keys)

        def largest(tag, counter):
            # the 1 GiB copy: the copy dispatch with the largest count
            rows = _counter_rows(_find_csv(run_dir, tag), "copy")
            return max(rows.values(), key=lambda r: r[counter])
        tr = "k_trace<0, 1, 0, 8, 64>"
        fetch, n = one("fetch", tr)
        write, _ = one("write", tr)
        cfetch = largest("fetch", "FETCH_SIZE")
        cwrite = largest("write", "WRITE_SIZE")
        l2, _ = one("l2", tr)
        sq, _ = one("sq", tr)
        tt, _ = one("tatd", tr)
        gib = 1 << 30
        fs = gib / 1024 / cfetch["FETCH_SIZE"]
        ws = gib / 1024 / cwrite["WRITE_SIZE"]
        rd = fetch["FETCH_SIZE"] * 1024 * fs
        wr = write["WRITE_SIZE"] * 1024 * ws
        import csv
        bl = [json.loads(l) for l in open(os.path.join(run_dir, "bench.json")) if l.startswith("{")][-1]
        meta = {"rays": bl["config"]["rays_per_step"], "tris": bl["config"]["tris"],
                "tuning": bl["forms"]["q8"]["tuning"]}
        kt = None
        for dp, _, names in os.walk(run_dir):
            for f in names:
                if f.endswith("kernel_stats.csv"):
                    kt = os.path.join(dp, f)
        ns = None
        with open(kt) as fh:
            for r in csv.DictReader(fh):
                if r["Name"].startswith("void (anonymous namespace)::" + tr):
                    ns = float(r["AverageNs"])
        assert ns, "headline kernel missing from the kernel trace"
        cyc = sq["GRBM_GUI_ACTIVE"] / 8
        w = sq["SQ_WAVES"]
        out = {"kernel_hash": kernel_source_hash(), "rays": meta["rays"], "tris": meta["tris"],
               "tuning": meta["tuning"], "kernel": tr, "dispatches": n,
               "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
               "fetch_kib": fetch["FETCH_SIZE"], "write_kib": write["WRITE_SIZE"],
               "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
               "avg_kernel_ns": ns, "hbm_GBs": round((rd + wr) / ns, 1),
               "l2_hit_pct": round(100 * l2["TCC_HIT_sum"] / (l2["TCC_HIT_sum"] + l2["TCC_MISS_sum"]), 2),
               "valu_util_pct": round(100 * sq["SQ_INSTS_VALU"] * 2 / (1024 * cyc), 1),
               "valu_active_threads": round(sq["SQ_THREAD_CYCLES_VALU"] / sq["SQ_INSTS_VALU"], 2),
               "valu_insts_per_wave": round(sq["SQ_INSTS_VALU"] / w, 1),
               "salu_insts_per_wave": round(sq["SQ_INSTS_SALU"] / w, 1),
               "vmem_insts_per_wave": round((sq["SQ_INSTS_VMEM_RD"] + sq["SQ_INSTS_VMEM_WR"]) / w, 1),
               "smem_insts_per_wave": round(sq["SQ_INSTS_SMEM"] / w, 1),
               "ta_busy_pct": round(100 * tt["TA_TA_BUSY_sum"] / (256 * tt["GRBM_GUI_ACTIVE"] / 8), 1),
               "td_busy_pct": round(100 * tt["TD_TD_BUSY_sum"] / (256 * tt["GRBM_GUI_ACTIVE"] / 8), 1),
               "note": "rocprofv3 --pmc passes over bench.py --no-autotune --calib-copy: FETCH_SIZE "
                       "and WRITE_SIZE scaled by the 1 GiB copy; TCC_HIT/MISS; SQ and TA/TD "
                       "counters; VALU utilisation = 2 cycles per wave64 instruction over "
                       "1024 SIMDs x cycles"}
        path = os.path.join(ROOT, "profiles", "trace_traffic.json")
    elif kind == "mesh_traffic":
        # the last TSDF + marching-cubes call of `--workload mesh --steps 2
        # --warmup 0 --no-cpu --calib-copy` (the first marching-cubes call
        # counts twice, to size its outputs): every dispatch from its
        # smoothing pass to its triangle emission
        import csv

        def per_dispatch(tag, counter):
            out = {}
            with open(_find_csv(run_dir, tag)) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        out[int(r["Dispatch_Id"])] = (r["Kernel_Name"], float(r["Counter_Value"]))
            return out

        def short(name):
            import re
            m = re.search(r"(k_[A-Za-z0-9_]+(<[^>(]*>)?)\(", name)
            return m.group(1) if m else name[:40]

        fetch = per_dispatch("fetch", "FETCH_SIZE")
        write = per_dispatch("write", "WRITE_SIZE")
        cf = max(v for n, v in fetch.values() if "copy" in n)
        cw = max(v for n, v in write.values() if "copy" in n)
        fs, ws = (1 << 30) / 1024 / cf, (1 << 30) / 1024 / cw

        def window(d):
            ids = sorted(d)
            a = max(i for i in ids if "k_smooth" in d[i][0])
            b = next(i for i in ids if i > a and "k_mc_emit" in d[i][0])
            return [i for i in ids if a <= i <= b]
        wf, ww = window(fetch), window(write)
        assert [short(fetch[i][0]) for i in wf] == [short(write[i][0]) for i in ww]
        per = {}
        for i, j in zip(wf, ww):
            k = short(fetch[i][0])
            e = per.setdefault(k, {"dispatches": 0, "read_bytes": 0.0, "write_bytes": 0.0})
            e["dispatches"] += 1
            e["read_bytes"] += fetch[i][1] * 1024 * fs
            e["write_bytes"] += write[j][1] * 1024 * ws
        rd = sum(e["read_bytes"] for e in per.values())
        wr = sum(e["write_bytes"] for e in per.values())
        bl = [json.loads(l) for l in open(os.path.join(run_dir, "bench.json")) if l.startswith("{")][-1]
        nv = bl["config"]["voxels"]
        out = {"kernel_hash": kernel_source_hash(MESH_KERNEL_FILES), "voxels": nv,
               "dispatches": len(wf), "bytes_per_step": rd + wr, "read_bytes": rd,
               "write_bytes": wr, "bytes_per_voxel": round((rd + wr) / nv, 3),
               "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
               "per_kernel": {k: {"dispatches": e["dispatches"],
                                  "read_MB": round(e["read_bytes"] / 1e6, 2),
                                  "write_MB": round(e["write_bytes"] / 1e6, 2)}
                              for k, e in sorted(per.items(), key=lambda x: -(x[1]["read_bytes"]
                                                                              + x[1]["write_bytes"]))},
               "note": "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, over bench.py --workload mesh "
                       "--steps 2 --warmup 0 --no-cpu --calib-copy; the dispatches of its last "
                       "TSDF + marching-cubes call, scaled by the 1 GiB copy"}
        path = os.path.join(ROOT, "profiles", "tsdf_traffic.json")
    else:
        raise SystemExit(f"unknown --ingest kind '{kind}'")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({"wrote": path}))
    return 0


def serve_measure(n_scenes, n_requests, rates, inflight, batch_cap_m, policy, max_wait_ms):
    """Poisson-arriving requests against `n_scenes` resident terrain scenes
    (50k..5M triangles, log-uniform).  Each request: 1..4096 environments
    (log-uniform), a pattern of 16/32/64/128 rings x 360..2048 azimuths, a
    random scene.  Served: continuous batching on Q8 BVHs (rc_serve_*).
    Baseline: the same requests one at a time in arrival order with plain
    FP32 BVHs (rc_raycast_batch + synchronize).  Rates are fractions of the
    server's capacity, measured first with every request submitted at once.
    Returns a dict with the capacity and, per rate, p50/p99 latency and
    Mrays/s of both."""
    import threading

    import torch
    import synth
    from paper_2509_17390_amd import Context, Job
    from paper_2509_17390_amd.rcast import RC_OK, last_error

    dev = torch.device("cuda", 0)
    wc = synth.workload_config("serve_16")
    rng = np.random.default_rng(wc["size_seed"])
    log(f"serving: generating {n_scenes} terrains ...")
    sizes = np.exp(rng.uniform(np.log(5e4), np.log(5e6), n_scenes))
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    q8_ids, fp_ids, pose_pools = [], [], []
    for k, n in enumerate(sizes):
        v, t, height, boxes = synth.terrain_scene(wc["terrain_seed_base"] + k, int(n))
        a = ctx.upload_scene(v, t)
        ctx.build(a, node_format=1, stream=stream)
        b = ctx.upload_scene(v, t)
        ctx.build(b, node_format=0, stream=stream)
        q8_ids.append(a)
        fp_ids.append(b)
        pose_pools.append(synth.terrain_poses(height, boxes, 256, wc["pose_seed_base"] + k))
    torch.cuda.synchronize()
    spans = {16: (-15.0, 15.0), 32: (-16.0, 15.0), 64: (-25.0, 3.0), 128: (-22.5, 22.5)}
    bank = []
    for ne in (16, 32, 64, 128):
        for na in (360, 512, 1024, 1440, 2048):
            lo, hi = spans[ne]
            bank.append((ctx.upload_pattern(synth.lidar_pattern(ne, lo, hi, na), na), ne * na))

    def make_reqs(n, seed):
        g = np.random.default_rng(seed)
        out = []
        for _ in range(n):
            envs = int(min(4096, max(1, round(np.exp(g.uniform(0, np.log(4096)))))))
            sc = int(g.integers(n_scenes))
            pi = int(g.integers(len(bank)))
            pool = pose_pools[sc]
            poses = pool[g.integers(0, len(pool), envs)]
            out.append((sc, pi, poses, envs * bank[pi][1]))
        return out

    def serve_run(reqs, arrivals):
        ctx.serve_start(arena_bytes=48 << 30, max_inflight=inflight,
                        max_batch_rays_m=batch_cap_m, policy=policy, max_wait_ms=max_wait_ms)
        tickets = [None] * len(reqs)
        t0 = time.perf_counter()

        def submitter():
            for i, (sc, pi, poses, _) in enumerate(reqs):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = ctx.submit(q8_ids[sc], bank[pi][0], poses, 0.1, 120.0)

        th = threading.Thread(target=submitter)
        th.start()
        lat = []
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0002)
            st, l = ctx.poll(tickets[i], -1)
            assert st == RC_OK, (st, last_error())
            lat.append(l)
            ctx.release(tickets[i])
        th.join()
        wall = time.perf_counter() - t0
        stats = ctx.serve_stats()
        ctx.serve_stop()
        return np.array(lat), wall, stats

    def baseline_run(reqs, arrivals):
        lat = []
        t0 = time.perf_counter()
        for i, (sc, pi, poses, n) in enumerate(reqs):
            dt = arrivals[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            r = torch.empty(n, dtype=torch.float32, device=dev)
            h = torch.empty(n, dtype=torch.int32, device=dev)
            pd = torch.from_numpy(poses).to(dev)
            ctx.raycast([Job(fp_ids[sc], bank[pi][0], pd, 0.1, 120.0)], r, h, stream=stream)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
            del r, h, pd
        return np.array(lat), time.perf_counter() - t0

    # capacity: everything submitted at once
    calib = make_reqs(n_requests, wc["capacity_request_seed"])
    lat, wall, _ = serve_run(calib, np.zeros(len(calib)))
    rays = sum(r[3] for r in calib)
    cap_rps = len(calib) / wall
    log(f"serving capacity {cap_rps:.1f} req/s, {rays / wall / 1e6:.0f} Mrays/s saturated")
    results = []
    for k, frac in enumerate(rates):
        lam = frac * cap_rps
        reqs = make_reqs(n_requests, wc["rate_request_seed_base"] + k)
        arrivals = np.cumsum(np.random.default_rng(wc["arrival_seed_base"] + k).exponential(
            1.0 / lam, len(reqs)))
        arrivals -= arrivals[0]
        rays = sum(r[3] for r in reqs)
        sl, sw, st = serve_run(reqs, arrivals)
        bl, bw = baseline_run(reqs, arrivals)
        results.append({
            "rate_frac": frac, "lambda_req_s": round(lam, 2), "requests": len(reqs),
            "mean_rays_per_request": round(rays / len(reqs)),
            "served": {"p50_ms": round(float(np.percentile(sl, 50)), 3),
                       "p99_ms": round(float(np.percentile(sl, 99)), 3),
                       "Mrays_s": round(rays / sw / 1e6, 1), "launches": st["launches"],
                       "max_batch_requests": st["max_batch_requests"],
                       "peak_inflight": st["peak_inflight"],
                       "peak_arena_GB": round(st["peak_bytes"] / 1e9, 2)},
            "per_request_fp32": {"p50_ms": round(float(np.percentile(bl, 50)), 3),
                                 "p99_ms": round(float(np.percentile(bl, 99)), 3),
                                 "Mrays_s": round(rays / bw / 1e6, 1)},
        })
        log(json.dumps(results[-1]))
    ctx.close()
    return {
        "workload": f"Poisson requests, {n_scenes} resident terrains ({int(sizes.sum())} "
                    f"triangles, 50k..5M each), 1..4096 envs (log-uniform), 20 patterns "
                    f"(16/32/64/128 rings x 360..2048 azimuths); served = Q8 nodes, continuous "
                    f"batching; per_request_fp32 = one rc_raycast_batch per request, FP32 "
                    f"nodes, arrival order",
        "capacity_req_s": round(cap_rps, 2),
        "capacity_Mrays_s": round(sum(r[3] for r in calib) / wall / 1e6, 1),
        "batch_cap_m_rays": batch_cap_m, "max_inflight": inflight, "policy": policy,
        "max_wait_ms": max_wait_ms or 200, "rates": results,
    }


def run_serve(args):
    """Serving sweep (see serve_measure), one JSON line."""
    n_scenes = args.scenes or 16
    rates = [float(x) for x in args.rates.split(",")]
    res = serve_measure(n_scenes, args.requests, rates, args.inflight, args.batch_cap_m,
                        args.policy, args.max_wait_ms)
    head = res["rates"][-1]
    out = {
        "metric": "p50/p99 request latency and Mrays/s, served (Q8, continuous batching) vs "
                  "plain per-request FP32",
        "value": head["served"]["Mrays_s"], "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 0, "ms_per_step": head["served"]["p50_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {k: v for k, v in res.items() if k != "rates"},
        "rates": res["rates"],
    }
    print(json.dumps(out), flush=True)
    return 0


def run_frame(args):
    """Single-sensor frame rate: one environment, 128 x 2048 beams (262,144
    rays, over -22.5..+22.5 deg) on the indoor mesh polygonised at 1.45 cm
    (6.4M triangles), Q8 nodes, one graph replay per frame; also 8 poses per
    launch.  The paper reports > 500 FPS for 200k+ rays on a 6M+ triangle
    scene (RTX 6000 Ada) -- context, not a target."""
    import torch
    import synth
    from paper_2509_17390_amd import Context, Job

    dev = torch.device("cuda", 0)
    h = 0.0145 if args.h is None else args.h
    log(f"polygonising at h = {h} m ...")
    sdf, v, t = synth.indoor_mesh(1, h)
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    scene = ctx.upload_scene(v, t)
    dirs = synth.lidar_pattern(128, -22.5, 22.5, 2048)
    pat = ctx.upload_pattern(dirs, 2048)
    results = {}
    for n_env in (1, 8):
        poses = torch.from_numpy(synth.free_space_poses(sdf, n_env, 31)).to(dev)
        n_rays = n_env * len(dirs)
        out_r = torch.empty(n_rays, dtype=torch.float32, device=dev)
        out_h = torch.empty(n_rays, dtype=torch.int32, device=dev)
        job = [Job(scene, pat, poses, 0.1, 120.0)]
        for name, fmt in (("fp32", 0), ("q8", 1)):
            ctx.build(scene, node_format=fmt, stream=stream)
            torch.cuda.synchronize()
            best, _ = ctx.autotune(job, out_r, out_h, reps=2, stream=stream)
            g = ctx.graph(job, out_r, out_h)
            for _ in range(10):
                g.launch(stream)
            torch.cuda.synchronize()
            frames = 200
            t0 = time.perf_counter()
            for _ in range(frames):
                g.launch(stream)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / frames
            g.close()
            results[f"{name}_{n_env}env"] = {"ms_per_frame": round(ms, 4),
                                             "frames_per_s": round(1e3 / ms, 1),
                                             "Mrays_s": round(n_rays / ms / 1e3, 1),
                                             "rays": int(n_rays), "tuning": best}
            log(f"{name} {n_env} env: {ms:.3f} ms/frame")
    head = results["q8_1env"]
    out = {
        "metric": "frames/s, one sensor with 128x2048 beams on a 6.4M-triangle mesh",
        "value": head["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": 200,
        "warmup": 10, "ms_per_step": head["ms_per_frame"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"single-sensor frame, 262,144 rays, {len(t)}-triangle indoor "
                               f"mesh (marching cubes at {h} m), graph replay per frame",
                   "tris": int(len(t))},
        "forms": results,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


# Gaussian-to-occupancy conversion: arithmetic per Gaussian-voxel evaluation
# of the density definition: d = v - mu (3), whitened u = S^-1 R^T d (9 mul +
# 6 add), q = |u|^2 (3 mul + 2 add), exp(-q/2) (2), times alpha^2 (1),
# accumulate (1)
PAIR_FLOPS = 27
FP32_VECTOR_PEAK_TFLOPS = 157.3


def vox_cpu_baseline(params, grid, g_density, g_counts, budget_s):
    """The FP64 oracle on a seeded sample of whole tiles of the same grid (one
    call over all sampled voxels; a first call on 8 tiles sizes the sample)."""
    from oracle import gauss as og
    rng = np.random.default_rng(4321)
    tx, ty, tz = grid.tiles

    def sample(n_tiles):
        ts = np.stack([rng.integers(tx, size=n_tiles), rng.integers(ty, size=n_tiles),
                       rng.integers(tz, size=n_tiles)], axis=1)
        vox = []
        for t in ts:
            (x0, x1), (y0, y1), (z0, z1) = grid.tile_voxels(tuple(t))
            vox.append(np.stack(np.meshgrid(np.arange(x0, x1), np.arange(y0, y1),
                                            np.arange(z0, z1), indexing="ij"),
                                axis=-1).reshape(-1, 3))
        vox = np.concatenate(vox)
        t0 = time.perf_counter()
        D, E, K = og.density_at(params, grid, vox, 3.0)
        return vox, D, E, K, time.perf_counter() - t0

    _, _, _, _, dt8 = sample(8)
    n_tiles = int(min(max(8, budget_s / (dt8 / 8)), 4096))
    vox, D, E, K, dt = sample(n_tiles)
    t = vox // grid.tile
    exact = bool(np.all(K == g_counts[t[:, 2], t[:, 1], t[:, 0]]))
    g = g_density[vox[:, 2], vox[:, 1], vox[:, 0]].astype(np.float64)
    tol = 2.0 ** -24 * (16 * E + 4 * D) + (K + 1) * 2.0 ** -31
    worst = float(np.max(np.abs(g - D) / tol))
    return {"value": len(vox) / dt / 1e6, "unit": "Mvoxels/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_tiles} seeded whole tiles ({len(vox)} voxels) of the same grid: "
                      f"culling sets by testing all {len(params[0])} Gaussian boxes, FP64 "
                      f"density (numpy, one thread), {dt:.1f} s",
            "gpu_agreement": {"tiles": n_tiles, "tile_counts_exact": exact,
                              "max_err_over_tol": worst}}


def run_voxelize(args):
    """Gaussian-to-occupancy conversion (FGGS-LiDAR Sec. IV-A): one million
    3DGS-like Gaussians on the surfaces of the indoor scene, a 2 cm grid over
    the 10 x 8 x 3 m room with 10 cm margins (510 x 410 x 160 = 33.5M
    voxels, 8^3 tiles), k = 3, theta = 0.5.  A step = Gaussian boxes + LBVH
    + evaluation records, then density, occupancy and surface mask."""
    import torch
    import synth
    from oracle import gauss as og
    from paper_2509_17390_amd import Context

    dev = torch.device("cuda", 0)
    n = 1_000_000
    log("generating Gaussians ...")
    m, q, sc, a, room = synth.splat_scene(1, n)
    params = (m, q, sc, a)
    grid = og.Grid((-0.1, -0.1, -0.1), 0.02, (510, 410, 160), tile=8, theta=0.5)
    nx, ny, nz = grid.dims
    n_vox = nx * ny * nz
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    dparams = [torch.from_numpy(x).to(dev) for x in params]
    gset = ctx.upload_gaussians(*dparams)
    rg = ctx.grid(grid.origin, float(grid.h), grid.dims, float(grid.theta))
    D = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    O = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    S = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    tx, ty, tz = grid.tiles
    C = torch.empty((tz, ty, tx), dtype=torch.int32, device=dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.build_gaussians(gset, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.voxelize(gset, rg, D, O, S, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    vox_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    # the density kernel alone (no surface pass): its own events
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps)
    e0.record(stream)
    for _ in range(reps):
        ctx.voxelize(gset, rg, D, O, None, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dens_ms = e0.elapsed_time(e1) / reps
    ctx.voxelize(gset, rg, D, O, S, stream=stream)
    ctx.voxelize_counts(gset, rg, C, stream=stream)
    torch.cuda.synchronize()
    counts = C.cpu().numpy().astype(np.int64)
    # Gaussian-voxel evaluations: |C_tile| times the tile's voxels in the grid
    vx = np.minimum(8, nx - 8 * np.arange(tx))
    vy = np.minimum(8, ny - 8 * np.arange(ty))
    vz = np.minimum(8, nz - 8 * np.arange(tz))
    tile_vox = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    pairs = int((counts * tile_vox).sum())
    tflops = pairs * PAIR_FLOPS / (dens_ms * 1e-3) / 1e12
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    khash = kernel_source_hash(("gauss.hip", "gauss_internal.h", "rc_internal.h"))
    counters = None
    cp = os.path.join(ROOT, "profiles", "voxelize_counters.json")
    if os.path.exists(cp):
        with open(cp) as fh:
            c = json.load(fh)
        if c.get("kernel_hash") == khash and c.get("gaussians") == n and c.get("voxels") == n_vox:
            counters = c
    occ_n = int(O.sum().item())
    surf_n = int(S.sum().item())
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on sampled tiles ...")
        cpu = vox_cpu_baseline(params, grid, D.cpu().numpy(), counts, args.cpu_budget)
    value = n_vox / (ms_step * 1e-3) / 1e6
    out = {
        "metric": "Mvoxels/s, Gaussian-to-occupancy conversion (1M Gaussians, 33.5M voxels)",
        "value": round(value, 2), "unit": "Mvoxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Gaussian-to-occupancy: {n} 3DGS-like Gaussians on the indoor "
                               f"scene surfaces (3% floaters), grid {nx}x{ny}x{nz} at "
                               f"{float(grid.h)} m, 8^3 tiles, k = 3, theta = 0.5; step = "
                               f"boxes + LBVH + records, density + occupancy + surface",
                   "gaussians": n, "voxels": n_vox, "tiles": int(counts.size)},
        "build_ms": round(build_ms, 3), "convert_ms": round(vox_ms, 3),
        "density_kernel_ms": round(dens_ms, 3),
        "culling": {"pairs": pairs, "mean_tile_set": round(float(counts.mean()), 2),
                    "max_tile_set": int(counts.max()),
                    "nonempty_tiles": int((counts > 0).sum()),
                    "brute_force_pairs": int(n) * n_vox},
        "roofline": {"bound": "alu", "achieved": round(tflops, 2),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": None if counters is None else counters["bytes_per_launch"],
                     "kernel": "k_voxelize<0>", "flops_per_pair": PAIR_FLOPS,
                     "kernel_hash": khash,
                     "counters": None if counters is None else {
                         k: counters[k] for k in ("hbm_GBs", "valu_util_pct",
                                                  "valu_active_threads", "valu_insts_per_wave",
                                                  "read_bytes", "write_bytes")}},
        # instruction issue of the same kernel (one wave64 VALU instruction per
        # SIMD every 2 cycles, 1024 SIMDs at 2.4 GHz)
        "roofline_valu": None if counters is None else {
            "bound": "alu", "unit": "G wave-instructions/s",
            "achieved": round(counters["valu_insts_per_wave"] * counters["waves"]
                              / (dens_ms * 1e-3) / 1e9, 1),
            "peak": VALU_PEAK_GWI,
            "frac": round(counters["valu_insts_per_wave"] * counters["waves"]
                          / (dens_ms * 1e-3) / 1e9 / VALU_PEAK_GWI, 4)},
        "occupied": occ_n, "surface": surf_n,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


# components of fewer triangles are removed after decimation (specks left
# by floaters; a 30 cm object at the 6 cm decimation cell has ~150 faces)
MIN_COMPONENT_FACES = 32

# Narrow-band TSDF + marching cubes: HBM bytes per voxel of each pass as
# built (reads + writes of the dense arrays; neighbour and tile-halo
# re-reads hit the caches): for kernels of 1 to 3 steps (as here) and the
# fixed threshold one tiled pass from the mask to V~ and the packed free
# bits (else smoothing u8 -> u8 -> u16 -> V~ and the packing to 2-bit
# labels as passes of their own), then for bands of at most
# 4 shells one tiled pass from V~ and the outside bits to phi float32 (S_0
# and the shells stay in LDS; wider bands: S_0 and each shell as byte
# passes, then phi), the marching-cubes count writing mask and case bytes,
# the tile scan forming both counts from those bytes and writing each
# point's u16 vertex offset within its tile, and the emit pass reading mask
# and case (the surface points' outputs are counted separately)
TSDF_PASS_BYTES = {
    "smooth_pack_tiled": 1 + 1 + 0.25,
    "smooth_x": 1 + 1, "smooth_y": 1 + 2, "smooth_z": 2 + 1, "pack": 1 + 0.25,
    "flood_sweep": 0.375, "shells_phi_tiled": 1 + 0.125 + 4,
    "shell0": 1 + 1, "shell": 1 + 1, "phi": 1 + 0.125 + 4,
    "mc_count": 4 + 1 + 1, "mc_scans": 1 + 1 + 2, "mc_emit": 1 + 1,
}


def tsdf_bytes_per_voxel(shells: int, steps: int, quantile: bool = False) -> float:
    """Bytes per voxel of TSDF_PASS_BYTES for a band of `shells` shells and a
    smoothing kernel of `steps` steps."""
    b = TSDF_PASS_BYTES
    total = b["flood_sweep"] + b["mc_count"] + b["mc_scans"] + b["mc_emit"]
    if 1 <= steps <= 3 and not quantile:
        total += b["smooth_pack_tiled"]
    else:
        total += b["smooth_x"] + b["smooth_y"] + b["smooth_z"] + b["pack"]
    if shells <= 4:
        return total + b["shells_phi_tiled"]
    return total + b["shell0"] + shells * b["shell"] + b["phi"]


def mesh_properties(v0, t0, v1, t1):
    """What quadric-error decimation must keep, checked at full size on the
    CPU: boundary edges (a face's edge on no other face) and non-manifold
    edges stay as they were, no new non-manifold edge appears, every face
    is a triangle of distinct used vertices, and the Euler characteristic
    of the whole mesh is unchanged (the link condition keeps the topology)."""
    def edges(t):
        e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), axis=1)
        _, cnt = np.unique(e[:, 0].astype(np.int64) << 32 | e[:, 1], return_counts=True)
        return cnt

    def euler(t, nv):
        return len(np.unique(t)) - len(edges(t)) + len(t)
    c0, c1 = edges(t0), edges(t1)
    return {"faces_in": int(len(t0)), "faces_out": int(len(t1)),
            "boundary_edges_in": int((c0 == 1).sum()), "boundary_edges_out": int((c1 == 1).sum()),
            "nonmanifold_edges_in": int((c0 > 2).sum()), "nonmanifold_edges_out": int((c1 > 2).sum()),
            "euler_in": int(euler(t0, len(v0))), "euler_out": int(euler(t1, len(v1))),
            "degenerate_faces_out": int(((t1[:, 0] == t1[:, 1]) | (t1[:, 1] == t1[:, 2]) |
                                         (t1[:, 0] == t1[:, 2])).sum()),
            "all_vertices_used": bool(len(np.unique(t1)) == len(v1))}


def run_mesh(args):
    """Occupancy to mesh (FGGS-LiDAR Sec. IV-B) on the surface mask of the
    Gaussian conversion workload (1M Gaussians, 510 x 410 x 160 voxels at
    2 cm, theta = 0.2): binomial smoothing (sigma 2 cm), tau = 0.15, outside
    labelling, shells up to r = 6 cm, phi, then marching cubes at iso 0 with
    vertex normals
    (timed: the value); then decimation to 10 % and Taubin smoothing (timed
    apart); both meshes are uploaded, their BVHs built, a LiDAR frame cast
    and scored against the same frame on the ground-truth mesh (CD,
    F-score at 5 cm)."""
    import torch
    import synth
    from oracle import gauss as og
    from oracle import tsdf as ot
    from paper_2509_17390_amd import Context, Job

    dev = torch.device("cuda", 0)
    m, q, sc, a, room = synth.splat_scene(1, 1_000_000)
    grid = og.Grid((-0.1, -0.1, -0.1), 0.02, (510, 410, 160), tile=8, theta=0.2)
    nx, ny, nz = grid.dims
    n_vox = nx * ny * nz
    sigma, tau, band = 0.02, 0.15, 0.06
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    gset = ctx.upload_gaussians(*[torch.from_numpy(x).to(dev) for x in (m, q, sc, a)])
    ctx.build_gaussians(gset, stream=stream)
    rg = ctx.grid(grid.origin, float(grid.h), grid.dims, float(grid.theta))
    O = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    S = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    ctx.voxelize(gset, rg, None, O, S, stream=stream)
    phi = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    vt = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    if args.calib_copy:
        # 1 GiB read + 1 GiB written, to scale the byte counters of a
        # rocprofv3 --pmc run of this workload
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        t0 = time.perf_counter()
        ctx.tsdf(rg, S, phi, sigma, tau, band, out_vtilde=vt, stream=stream)
        t1 = time.perf_counter()
        verts, tris, _ = ctx.marching_cubes(rg, phi, 0.0, stream=stream, normals=True)
        t2 = time.perf_counter()
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, verts, tris

    for _ in range(args.warmup):
        step()
    ts, ms = [], []
    for _ in range(args.steps):
        a_ms, b_ms, verts, tris = step()
        ts.append(a_ms)
        ms.append(b_ms)
    tsdf_ms, mc_ms = float(np.median(ts)), float(np.median(ms))
    ms_step = tsdf_ms + mc_ms
    # mesh optimisation (paper defaults): quadric-error decimation to 10 % of
    # the faces in three rounds, removal of components under
    # MIN_COMPONENT_FACES triangles, then Taubin smoothing (0.5, -0.53), 10
    # iterations; the one-pass vertex clustering is timed beside it
    dec_ms, cc_ms, smo_ms, clu_ms = [], [], [], []
    for k in range(3):
        t0 = time.perf_counter()
        _, clu_tris, cell = ctx.decimate(verts, tris, 0.1, stream=stream)
        if k:
            clu_ms.append((time.perf_counter() - t0) * 1e3)
    n_clu_tris = int(clu_tris.shape[0])
    for k in range(max(3, args.steps // 2)):
        t0 = time.perf_counter()
        dverts, dtris, qem_steps = ctx.decimate_qem(verts, tris, 0.1, 3, stream=stream)
        t1 = time.perf_counter()
        cverts, ctris = ctx.remove_small_components(dverts, dtris, MIN_COMPONENT_FACES,
                                                    stream=stream)
        t2 = time.perf_counter()
        ctx.taubin(cverts, ctris, 0.5, -0.53, 10, stream=stream)
        t3 = time.perf_counter()
        if k:
            dec_ms.append((t1 - t0) * 1e3)
            cc_ms.append((t2 - t1) * 1e3)
            smo_ms.append((t3 - t2) * 1e3)
    decimate_ms, smooth_ms = float(np.median(dec_ms)), float(np.median(smo_ms))
    components_ms = float(np.median(cc_ms))
    n_dec_tris = int(dtris.shape[0])
    qem_props = mesh_properties(verts.cpu().numpy(), tris.cpu().numpy(),
                                dverts.cpu().numpy(), dtris.cpu().numpy())
    dverts, dtris = cverts, ctris
    # the meshes as LiDAR scenes: BVH build and one 8-environment frame each
    sdf = synth.indoor_sdf(1)
    poses = torch.from_numpy(synth.free_space_poses(sdf, 8, 77)).to(dev)
    dirs = synth.lidar_pattern(32, -16.0, 15.0, 1024)
    pat = ctx.upload_pattern(dirs, 1024)

    def frame(vv, tt, reps=10):
        sc_ = ctx.upload_scene(vv, tt)
        ctx.build(sc_, node_format=1, stream=stream)
        job_ = [Job(sc_, pat, poses, 0.1, 120.0)]
        r_, h_ = ctx.cast(job_)
        torch.cuda.synchronize()
        t0_ = time.perf_counter()
        for _ in range(reps):
            r_, h_ = ctx.cast(job_)
        torch.cuda.synchronize()
        return r_, h_, (time.perf_counter() - t0_) * 1e3 / reps

    rr, hh, cast_ms = frame(verts, tris)
    rr_f, hh_f, cast_f_ms = frame(dverts, dtris)
    hit_frac = float((hh >= 0).float().mean())
    # fidelity in the paper's units: the same frame on the ground-truth mesh
    # the Gaussians were drawn from; points = origin + range * direction
    sdf_gt, v_gt, t_gt = synth.indoor_mesh(1, 0.035)
    gt = ctx.upload_scene(v_gt, t_gt)
    ctx.build(gt, node_format=1, stream=stream)
    rg_gt, hg_gt = ctx.cast([Job(gt, pat, poses, 0.1, 120.0)])
    torch.cuda.synchronize()

    def points(rng_t, hit_t):
        P = poses.cpu().numpy().astype(np.float64).reshape(-1, 3, 4)
        dd = dirs.astype(np.float64)
        rr = rng_t.cpu().numpy().astype(np.float64).reshape(len(P), len(dd))
        hh_ = hit_t.cpu().numpy().reshape(len(P), len(dd))
        out = []
        for e in range(len(P)):
            d = dd @ P[e][:, :3].T
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            ok = hh_[e] >= 0
            out.append(P[e][:, 3] + rr[e][ok, None] * d[ok])
        return np.concatenate(out).astype(np.float32)

    pts_sim, pts_gt = points(rr, hh), points(rg_gt, hg_gt)
    Pd, Gd = torch.from_numpy(pts_sim).to(dev), torch.from_numpy(pts_gt).to(dev)
    fid = ctx.chamfer_fscore(Pd, Gd, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        fid = ctx.chamfer_fscore(Pd, Gd, 0.05)
    fid_ms = (time.perf_counter() - t0) * 1e3 / 5
    fid_final = ctx.chamfer_fscore(torch.from_numpy(points(rr_f, hh_f)).to(dev), Gd, 0.05)
    # iterations of the outside labelling are not visible from here: count
    # the passes as one sweep (a lower bound of the bytes)
    P = int(np.ceil(float(np.float32(band)) / float(np.float32(grid.h))))
    sv = float(np.float32(sigma)) / float(np.float32(grid.h))
    steps = max(1, int(np.floor(2.0 * sv * sv + 0.5)))
    per_vox = tsdf_bytes_per_voxel(P, steps)
    # outputs: 12 B position + 12 B normal per vertex, 12 B per triangle
    alg_bytes = int(per_vox * n_vox) + 24 * int(verts.shape[0]) + 12 * int(tris.shape[0])
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    mesh_counters = load_mesh_traffic(n_vox)
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a sub-grid ...")
        surf = S.cpu().numpy()
        sub = surf[40:104, 100:228, 150:278]            # 64 x 128 x 128 voxels
        t0 = time.perf_counter()
        phi_o, _, _, _ = ot.tsdf(sub, float(grid.h), sigma, tau, band)
        vo, to, no = ot.marching_cubes(phi_o, (0, 0, 0), float(grid.h), 0.0, normals=True)
        dt = time.perf_counter() - t0
        sub_g = ctx.grid((0, 0, 0), float(grid.h), (128, 128, 64), 0.0)
        phi_g = torch.empty((64, 128, 128), dtype=torch.float32, device=dev)
        ctx.tsdf(sub_g, torch.from_numpy(np.ascontiguousarray(sub)).to(dev), phi_g, sigma, tau,
                 band)
        vg, tg, ng = ctx.marching_cubes(sub_g, phi_g, 0.0, normals=True)
        same = bool(np.array_equal(phi_g.cpu().numpy().view(np.uint32), phi_o.view(np.uint32))
                    and np.array_equal(vg.cpu().numpy().view(np.uint32), vo.view(np.uint32))
                    and np.array_equal(ng.cpu().numpy().view(np.uint32), no.view(np.uint32))
                    and np.array_equal(tg.cpu().numpy(), to))
        from oracle import metrics as om
        from oracle import mesh as omesh
        t0 = time.perf_counter()
        ocd = om.chamfer_fscore(pts_sim, pts_gt, 0.05)
        dt_m = time.perf_counter() - t0
        # decimation + smoothing of a smaller sub-grid's mesh, both sides
        from oracle import qem as oqem
        small = surf[40:72, 100:148, 150:198]           # 32 x 48 x 48 voxels
        phi_s, _, _, _ = ot.tsdf(small, float(grid.h), sigma, tau, band)
        vo2, to2 = ot.marching_cubes(phi_s, (0, 0, 0), float(grid.h), 0.0)
        t0 = time.perf_counter()
        dvo, dto = oqem.decimate_qem(vo2, to2, 0.1, 3)
        dvo, dto, _ = omesh.remove_small_components(dvo, dto, MIN_COMPONENT_FACES)
        svo = omesh.taubin(dvo, dto, 0.5, -0.53, 10)
        dt_d = time.perf_counter() - t0
        dvg, dtg, _ = ctx.decimate_qem(torch.from_numpy(vo2).to(dev),
                                       torch.from_numpy(to2).to(dev), 0.1, 3)
        dvg, dtg = ctx.remove_small_components(dvg, dtg, MIN_COMPONENT_FACES)
        ctx.taubin(dvg, dtg, 0.5, -0.53, 10)
        torch.cuda.synchronize()
        same_opt = bool(np.array_equal(dtg.cpu().numpy(), dto)
                        and np.array_equal(dvg.cpu().numpy().view(np.uint32), svo.view(np.uint32)))
        cpu = {"value": sub.size / dt / 1e6, "unit": "Mvoxels/s", "cores": 1, "kind": "oracle",
               "sample": f"a 128 x 128 x 64 sub-grid of the same surface mask, TSDF + marching "
                         f"cubes (numpy/scipy, one thread), {dt:.1f} s",
               "gpu_agreement": {"bit_identical": same, "triangles": int(len(to)),
                                 "decimate_components_smooth_bit_identical": same_opt,
                                 "decimate_smooth_oracle_s": round(dt_d, 2),
                                 "decimate_input_triangles": int(len(to2)),
                                 "decimated_triangles": int(len(dto))},
               "fidelity_oracle": {"s": round(dt_m, 3), "chamfer": ocd[0], "fscore": ocd[5],
                                   "chamfer_rel_diff": abs(ocd[0] - fid["chamfer"]) / ocd[0],
                                   "fscore_equal": ocd[5] == fid["fscore"]}}
    value = n_vox / (ms_step * 1e-3) / 1e6
    out = {
        "metric": "Mvoxels/s, occupancy to mesh (TSDF + marching cubes, 33.5M voxels)",
        "value": round(value, 2), "unit": "Mvoxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64/f32", "data": "synthetic",
        "config": {"workload": f"occupancy to mesh: surface mask (theta 0.2) of 1M Gaussians "
                               f"on a {nx}x{ny}x{nz} grid at {float(grid.h)} m; binomial smoothing "
                               f"sigma {sigma} m, tau {tau}, band {band} m, iso 0",
                   "voxels": n_vox, "surface_voxels": int(S.sum().item())},
        "tsdf_ms": round(tsdf_ms, 3), "marching_cubes_ms": round(mc_ms, 3),
        "mesh": {"vertices": int(verts.shape[0]), "triangles": int(tris.shape[0])},
        "lidar_on_mesh": {"rays": int(8 * len(dirs)), "ms": round(cast_ms, 3),
                          "hit_fraction": round(hit_frac, 4)},
        "mesh_optimisation": {
            "decimate_ms": round(decimate_ms, 3), "components_ms": round(components_ms, 3),
            "smooth_ms": round(smooth_ms, 3), "ratio": 0.1, "rounds": 3,
            "decimation": "quadric error, parallel edge contraction (rc_decimate_qem)",
            "contraction_steps": int(qem_steps), "decimated_properties": qem_props,
            "clustering": {"ms": round(float(np.median(clu_ms)), 3),
                           "cell_m": round(float(cell), 5), "triangles": n_clu_tris},
            "decimated_triangles": n_dec_tris, "min_component_faces": MIN_COMPONENT_FACES,
            "vertices": int(dverts.shape[0]), "triangles": int(dtris.shape[0]),
            "lidar_ms": round(cast_f_ms, 3),
            "chamfer_m": fid_final["chamfer"], "fscore_at_0.05m": fid_final["fscore"]},
        "fidelity_vs_ground_truth_mesh": {
            "chamfer_m": fid["chamfer"], "fscore_at_0.05m": fid["fscore"],
            "precision": fid["precision"], "recall": fid["recall"],
            "points_sim": int(fid["n_p"]), "points_gt": int(fid["n_g"]),
            "gpu_ms": round(fid_ms, 3),
            "setup": "8 free-space poses x 32x1024 beams on the reconstructed mesh and on the "
                     "h = 3.5 cm ground-truth mesh the Gaussians were drawn from"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if mesh_counters is None else mesh_counters["bytes_per_step"],
                     "kernel": "rc_tsdf + rc_marching_cubes (all passes)",
                     "bytes_per_voxel": per_vox,
                     "measured": None if mesh_counters is None else {
                         "GB_s": round(mesh_counters["bytes_per_step"] / (ms_step * 1e-3) / 1e9, 1),
                         "frac": round(mesh_counters["bytes_per_step"] / (ms_step * 1e-3) / 1e9
                                       / HBM_PEAK_GBS, 4),
                         "bytes_per_voxel": round(mesh_counters["bytes_per_step"] / n_vox, 2),
                         "source": "rocprofv3 FETCH_SIZE + WRITE_SIZE over one TSDF + marching "
                                   "cubes call, scaled by a 1 GiB copy (profiles/tsdf_traffic.json)"}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
