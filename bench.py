#!/usr/bin/env python3
"""Throughput benchmark of the acoustic propagator on one MI355X.

Workload (one "step"): the field-scale single shot -- a seeded 620 x 1001
velocity slice at 10 m with a 40-cell sponge and a free surface, dt 0.8 ms,
nt 10000 levels (8 s), a 12 Hz Ricker source at (10 m, 5000 m), 1001
receivers at 10 m, snapshots every 100 steps over the first 5 s.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: grid-point updates per second over the padded grid
(660 x 1081 points x 9999 updates per step), the HBM-roofline position of the
time-stepping kernel, and the FP64 oracle timed on a bounded sample on the
host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_UPDATE = 16.0        # read p^n, p^{n-1}, coefficient; write p^{n+1}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--tile-x", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--time-block", type=int, default=0)
    ap.add_argument("--rows-per-thread", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-levels", type=int, default=10000)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a known-size "
                         "reference kernel for hardware traffic counters)")
    return ap.parse_args()


def kernel_source_sha():
    p = os.path.join(ROOT, "paper_2605_30541_amd", "csrc", "sg_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_src_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(v, geom, src, rec, f0, levels):
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    used = oracle.set_threads(threads)
    og = oracle.Geometry(nz=geom.nz, nx=geom.nx, dz=geom.dz, dx=geom.dx, dt=geom.dt, nt=levels,
                         nbl=geom.nbl, top_free=True, R=geom.damp_R)
    w = oracle.ricker(f0, geom.dt, levels)
    t0 = time.perf_counter()
    oracle.forward(og, v.astype(np.float64), src, w, rec)
    sec = time.perf_counter() - t0
    Nz, Nx = og.padded_shape
    rate = Nz * Nx * (levels - 1) / sec / 1e9
    return {"value": rate, "unit": "Gpt-updates/s", "cores": used, "kind": "oracle",
            "sample": "FP64 oracle, one shot of the same 620x1001 slice and acquisition, "
                      "%d of 10000 levels (%.1f s wall)" % (levels, sec)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported "
              "(shots shard across GPUs with no communication, see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

    torch.cuda.set_device(0)
    nz, nx, h, dt, nt, f0 = 620, 1001, 10.0, 8e-4, 10000, 12.0
    geom = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0,
                    snap_every=100, snap_count=63)
    v = synth.field_slice(42, nz, nx)
    src = np.array([[10.0, 5000.0]])
    rec = synth.surface_receivers(nx, h)
    plan = Plan(geom)
    if args.variant is not None:
        plan.set_tuning(variant=args.variant, tile_x=args.tile_x, tile_z=args.tile_z,
                        time_block=args.time_block, rows_per_thread=args.rows_per_thread)
    tuning = plan.get_tuning(1)
    vp = torch.from_numpy(v).cuda()
    shots = Shots(src, rec, sgwave.ricker_tensor(f0, dt, nt))
    gathers = torch.empty((1, geom.nrow, nx), dtype=torch.float32, device="cuda")
    snaps = torch.empty((1, geom.snap_count, nz, nx), dtype=torch.float32, device="cuda")
    ws = torch.empty(sgwave.sg_forward_workspace_size(plan, 1, nx), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        sgwave.sg_forward(plan, vp, shots, gathers, snaps, ws, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    Nz, Nx = plan.padded_shape
    updates = Nz * Nx * (nt - 1)
    value = updates * args.steps / (ms / 1e3) / 1e9

    # dominant kernel: the time-stepping launches, timed as one back-to-back run
    plan.set_profiling(True)
    step()
    kms, launches = plan.profile()
    plan.set_profiling(False)
    torch.cuda.synchronize()
    avg_ms = kms / launches
    bytes_per_launch = BYTES_PER_UPDATE * updates / launches
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    kernel = "k_step_naive" if tuning["variant"] == 1 else "k_step_tiled"
    traffic = traffic_record(kernel, "field_shot")
    sgwave.sg_check_finite(gathers, ws)

    out = {
        "metric": "Gpt-updates/s & %HBM roofline: fwd vs fwd+adjoint grad, 1 MI355X, <=1e-4 rel L2",
        "value": value,
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "field-scale single shot forward: 620x1001 @10 m + 40-cell sponge "
                               "(660x1081 padded), dt 0.8 ms, nt 10000, 12 Hz Ricker, 1001 receivers, "
                               "63 snapshots every 100 steps",
                   "shots": 1, "padded_points": Nz * Nx, "updates_per_step": updates,
                   "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "launches_per_step": launches,
                     "avg_launch_us": avg_ms * 1e3,
                     "bytes_per_update": BYTES_PER_UPDATE},
        "cpu_baseline": None,
    }
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(v, geom, src, rec, f0, args.cpu_sample_levels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
