#!/usr/bin/env python3
"""Throughput benchmark of the acoustic propagator on one MI355X.

Workload (one "step"): the batched forward of 8 seeded field slices of
uneven size (nz 400-620, nx 601-1001 at 10 m, 40-cell sponge, free surface;
sizes from rng(42), slice i seeded 42 + i) x 64 shots each at 10 m depth
evenly spaced on [1.1 km, W - 1.1 km], dt 0.8 ms, nt 10000 levels (8 s), a
12 Hz Ricker, receivers on every surface column, all shots of all slices in
one time-blocked launch per time block, replayed from a hipGraph with the
batch-autotuned tiling.  Inputs are resident in HBM before the timed region.

Prints one JSON line: grid-point updates per second over the padded grids
(points x 9999 updates x 64 shots summed over the slices), the HBM-roofline
position of the time-stepping kernel (k_tiled_batch), and the FP64 oracle
timed on a bounded sample of the same workload on the host cores.  Beside
it, on the same GPU: the field-scale single shot (620 x 1001), the
forward + adjoint-gradient rate (16 shots on that slice, checkpoints every
100 levels), the full-density batched gradient (4 slices x 100 shots), the
paper's production shape (4 slices of 619 x 1000, 64 shots, 8001 levels,
gathers decimated by 14), the physics-residual pass and the builder modules.
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
LEGS = ("batch", "field_shot", "gradient", "batched_gradient", "paper", "residual", "builder")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", choices=LEGS, default=None,
                    help="run one workload only (for profiling runs); 'batch' is the headline")
    ap.add_argument("--levels", type=int, default=10000,
                    help="time levels of the headline batch (shorter runs for counter profiles)")
    ap.add_argument("--batch-tuning", type=str, default="",
                    help="tile_x,tile_z,time_block (tiled) or s<strip_width>,<segment rows>,<time_block> "
                         "(column sweep) for the headline batch instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-slices", type=int, default=3)
    ap.add_argument("--shots-per-wave", type=int, default=25)
    ap.add_argument("--grad-tuning", type=str, default="s128,96,3",
                    help="tuning of the forward and recompute passes of the 16-shot gradient, in the "
                         "form of --batch-tuning (the adjoint always runs the tiled kernel; default: column "
                         "sweep, 128-column strips, 96-row segments, time block 3, the fastest measured; "
                         "'' = tiled)")
    ap.add_argument("--batched-grad-tuning", type=str, default="s256,160,4",
                    help="the same for the full-density batched gradient (default: column sweep, 256-column "
                         "strips, 160-row segments, time block 4, the fastest measured; '' = tiled)")
    ap.add_argument("--field-tuning", type=str, default="",
                    help="tile_x,tile_z,time_block for the single field shot instead of the autotuner "
                         "(profiling runs: keeps the autotuner's trial launches out of the counters)")
    ap.add_argument("--field-steps", type=int, default=20, help="timed repetitions of the single field shot")
    ap.add_argument("--grad-levels", type=int, default=10000,
                    help="time levels of the two gradient workloads (shorter runs for counter profiles: "
                         "the launches and their grids are those of the full run)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a known-size "
                         "reference kernel for hardware traffic counters)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_sha(kernel: str):
    """sha256[:16] of the source file holding a kernel."""
    f = "sg_sweep.hip" if kernel.startswith("k_sweep") else "sg_kernels.hip"
    p = os.path.join(ROOT, "paper_2605_30541_amd", "csrc", f)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_record(kernel: str, workload: str, tuning):
    """Counter record (profiles/<kernel>_<workload>_traffic.json) of a kernel
    on a workload under `tuning`, if it was taken on the current kernel
    source; else None."""
    p = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(p):
        return None
    recs = json.load(open(p))
    key = "%d,%d,%d,%d" % (tuning["variant"], tuning["tile_x"], tuning["tile_z"], tuning["time_block"])
    rec = recs.get("by_tuning", {}).get(key)
    if rec is None or recs.get("kernel_src_sha") != kernel_source_sha(kernel):
        return None
    return dict(rec, source=recs.get("source"))


def kernel_shape(tuning):
    """Template arguments <K, NWX, NWZ> of the tiled kernel a tuning runs."""
    k = tuning.get("rows_per_thread") or 8
    return {(128, 64, 8): "8, 2, 8", (64, 128, 16): "16, 1, 8", (64, 64, 8): "8, 1, 8",
            (128, 64, 16): "16, 2, 4"}.get((tuning["tile_x"], tuning["tile_z"], k), "?")


def batch_items(levels):
    """The headline batch: 8 uneven slices x 64 shots; returns (items, padded
    points x shots, [(geom, v, src, rec)] per slice)."""
    import torch
    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots
    dt = 8e-4
    items, points, cases = [], 0, []
    for i, (nz, nx) in enumerate(synth.uneven_sizes(42, 8)):
        geom = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=dt, nt=levels, nbl=40, vmax_hint=4500.0)
        plan = Plan(geom)
        W = (nx - 1) * 10.0
        src = synth.shot_line(64, 1100.0, W - 1100.0)
        rec = synth.surface_receivers(nx, 10.0)
        v = synth.field_slice(42 + i, nz, nx)
        shots = Shots(src, rec, sgwave.ricker_tensor(12.0, dt, levels))
        gathers = torch.empty((64, geom.nrow, nx), dtype=torch.float32, device="cuda")
        items.append((plan, torch.from_numpy(v).cuda(), shots, gathers, None))
        Nz, Nx = plan.padded_shape
        points += Nz * Nx * 64
        cases.append((geom, v, src, rec))
    return items, points, cases


def parse_tuning(spec):
    """tile_x,tile_z,time_block (tiled) or s<strip>,<segment rows>,<time block> (column sweep)."""
    if not spec:
        return None
    parts = [int(x) for x in spec.replace("s", "").split(",")]
    if spec.startswith("s") or len(parts) == 2:
        z = parts[1] if len(parts) == 3 else 0
        return dict(variant=3, tile_x=parts[0], tile_z=z, time_block=parts[-1], rows_per_thread=0)
    return dict(variant=2, tile_x=parts[0], tile_z=parts[1], time_block=parts[2], rows_per_thread=0)


def batch_headline(args):
    """Times K replays of the headline batch (after W untimed ones), and the
    average launch of its time-stepping kernel from events on the stream the
    graph is launched on."""
    import torch
    from paper_2605_30541_amd import sgwave
    levels = args.levels
    items, points, cases = batch_items(levels)
    ws = torch.empty(sgwave.sg_batch_workspace_size(items), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    if args.batch_tuning:
        tuning = parse_tuning(args.batch_tuning)
    else:
        tuning = sgwave.sg_batch_autotune(items, ws, 32)          # untimed
    log("headline batch: tuning %s" % tuning)

    def step():
        sgwave.sg_batch_forward(items, ws, tuning, stream)

    for _ in range(args.warmup):
        step()                     # the first one records and instantiates the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(args.steps):
        step()
        torch.cuda.synchronize()   # (progress line per step; a step is seconds of GPU work)
        log("headline batch: step %d of %d done" % (k + 1, args.steps))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for it in items:
        sgwave.sg_check_finite(it[3], ws)
    updates = points * (levels - 1)
    value = updates * args.steps / (ms / 1e3) / 1e9
    tb = tuning["time_block"] or 3
    launches = -(-(levels - 1) // tb)
    # each replay is `launches` time-stepping launches (plus one small record
    # launch for the last level): their average duration, gaps included
    avg_ms = ms / args.steps / launches
    bytes_per_launch = BYTES_PER_UPDATE * updates / launches
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    shape = kernel_shape(tuning)
    kname = ("k_sweep_batch<%d, %d>" % (tuning["tile_x"] // 64, tb) if tuning["variant"] == 3
             else "k_tiled_batch<%s, 0, true>" % shape)
    rec = traffic_record("k_sweep_batch" if tuning["variant"] == 3 else "k_tiled_batch", "uneven_batch", tuning)
    traffic = None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": kname, "launches_per_step": launches,
            "avg_launch_us": avg_ms * 1e3, "bytes_per_update": BYTES_PER_UPDATE,
            "algorithmic_bytes_per_launch": bytes_per_launch}
    if rec is not None:
        traffic = rec["hbm_bytes_per_launch"]
        roof["traffic"] = traffic
        roof["measured_hbm_GBs"] = traffic / (avg_ms / 1e3) / 1e9
        roof["measured_hbm_frac"] = roof["measured_hbm_GBs"] / HBM_PEAK_GBS
        if rec.get("valu_insts_per_update") is not None:
            roof["valu_insts_per_update"] = rec["valu_insts_per_update"]
        roof["counters"] = rec.get("source")
    return {"value": value, "ms": ms, "tuning": tuning, "roofline": roof, "updates_per_step": updates,
            "points": points}, cases


def cpu_baseline(cases, nslices):
    """The FP64 oracle on a bounded sample of the headline workload: shot 0
    of each of the first `nslices` slices over all levels."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    used = oracle.set_threads(threads)
    upd, sec = 0, 0.0
    for geom, v, src, rec in cases[:nslices]:
        og = oracle.Geometry(nz=geom.nz, nx=geom.nx, dz=geom.dz, dx=geom.dx, dt=geom.dt, nt=geom.nt,
                             nbl=geom.nbl, top_free=True, R=geom.damp_R)
        w = oracle.ricker(12.0, geom.dt, geom.nt)
        t0 = time.perf_counter()
        oracle.forward(og, v.astype(np.float64), src[:1], w, rec)
        sec += time.perf_counter() - t0
        Nz, Nx = og.padded_shape
        upd += Nz * Nx * (geom.nt - 1)
    return {"value": upd / sec / 1e9, "unit": "Gpt-updates/s", "cores": used, "kind": "oracle",
            "sample": "FP64 oracle, shot 0 of each of the first %d of the 8 slices, all %d levels "
                      "(%.1f s wall)" % (nslices, cases[0][0].nt, sec)}


def field_shot_rate(steps=20, tuning=None):
    """The field-scale single shot: a 620 x 1001 slice (seed 42) at 10 m with a
    40-cell sponge, dt 0.8 ms, nt 10000, a 12 Hz Ricker at (10 m, 5000 m), 1001
    receivers, 63 snapshots every 100 levels; single-call path, autotuned
    unless a tuning is given."""
    import numpy as np
    import torch
    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots
    nz, nx, h, dt, nt, f0 = 620, 1001, 10.0, 8e-4, 10000, 12.0
    geom = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0,
                    snap_every=100, snap_count=63)
    v = synth.field_slice(42, nz, nx)
    plan = Plan(geom)
    vp = torch.from_numpy(v).cuda()
    shots = Shots(np.array([[10.0, 5000.0]]), synth.surface_receivers(nx, h), sgwave.ricker_tensor(f0, dt, nt))
    gathers = torch.empty((1, geom.nrow, nx), dtype=torch.float32, device="cuda")
    snaps = torch.empty((1, geom.snap_count, nz, nx), dtype=torch.float32, device="cuda")
    ws = torch.empty(sgwave.sg_forward_workspace_size(plan, 1, nx), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    if tuning:
        plan.set_tuning(**tuning)
    else:
        sgwave.sg_autotune(plan, vp, shots, 64, ws, stream)
    tuning = plan.get_tuning(1)

    def step():
        sgwave.sg_forward(plan, vp, shots, gathers, snaps, ws, stream)
    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    Nz, Nx = plan.padded_shape
    updates = Nz * Nx * (nt - 1)
    plan.set_profiling(True)
    step()
    kms, launches = plan.profile()
    plan.set_profiling(False)
    torch.cuda.synchronize()
    avg_ms = kms / launches
    achieved = BYTES_PER_UPDATE * updates / launches / (avg_ms / 1e3) / 1e9
    sgwave.sg_check_finite(gathers, ws)
    return {"workload": "field-scale single shot forward: 620x1001 @10 m + 40-cell sponge (660x1081 padded), "
                        "dt 0.8 ms, nt 10000, 12 Hz Ricker, 1001 receivers, 63 snapshots every 100 steps",
            "ms": ms, "value": updates / (ms / 1e3) / 1e9, "unit": "Gpt-updates/s", "tuning": tuning,
            "kernel": "k_tiled", "avg_launch_us": avg_ms * 1e3, "launches": launches,
            "hbm_algorithmic_GBs": achieved, "frac_of_hbm_peak": achieved / HBM_PEAK_GBS}, v


def gradient_rate(v, fwd_rate, tuning=None, nt=10000):
    """Forward with checkpoints + adjoint gradient: 16 shots on the field
    slice (1D-smoothed start model), checkpoints every 100 levels."""
    import numpy as np
    import torch
    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots
    nz, nx, h, dt, nshot, ckpt = 620, 1001, 10.0, 8e-4, 16, 100
    geom = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0)
    plan = Plan(geom)
    if tuning:
        plan.set_tuning(**tuning)
    v0 = torch.from_numpy(synth.smoothed_1d(v, 500.0, h)).cuda()
    shots = Shots(synth.shot_line(nshot, 1100.0, 8900.0), synth.surface_receivers(nx, h),
                  sgwave.ricker_tensor(12.0, dt, nt))
    ws = torch.empty(sgwave.sg_grad_workspace_size(plan, nshot, nx, ckpt), dtype=torch.uint8, device="cuda")
    gathers = torch.empty((nshot, geom.nrow, nx), dtype=torch.float32, device="cuda")
    resid = torch.randn((nshot, geom.nrow, nx), dtype=torch.float32, device="cuda")
    grad = torch.empty_like(v0)

    def run():
        sgwave.sg_forward_ckpt(plan, v0, shots, ckpt, gathers, ws)
        sgwave.sg_adjoint_gradient(plan, v0, shots, ckpt, resid, grad, ws)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    Nz, Nx = plan.padded_shape
    rate = Nz * Nx * (nt - 1) * nshot / (ms / 1e3) / 1e9
    sgwave.sg_check_finite(grad, ws)
    return {"workload": "forward with checkpoints + adjoint-state gradient, 16 shots on the 620x1001 "
                        "slice, nt %d, checkpoints every 100 levels (segment recompute)" % nt,
            "tuning": {"forward_and_recompute": tuning or "tiled 128x64, time block 3",
                       "adjoint": "tiled 128x64, time block 3"},
            "ms": ms, "value": rate, "unit": "Gpt-steps/s (padded points x time steps x shots)",
            "ratio_to_forward_value": rate / fwd_rate if fwd_rate else None}


def paper_workload_rate(fwd_rate):
    """The paper's production shape on the batched path: 4 field slices of
    619 x 1000 at 10 m with a 60-cell sponge, dt 1 ms, 8001 levels (8 s), 64
    shots each at 10 m uniform in [1.1 km, W - 1.1 km], 1000 receivers at
    10 m, gathers decimated by k = 14 (572 saved samples per trace)."""
    import torch
    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots
    nz, nx, h, dt, nt, k, nshot = 619, 1000, 10.0, 1e-3, 8001, 14, 64
    items, pts = [], 0
    for i in range(4):
        geom = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=60, vmax_hint=4500.0, rec_every=k)
        plan = Plan(geom)
        shots = Shots(synth.shot_line(nshot, 1100.0, (nx - 1) * h - 1100.0), synth.surface_receivers(nx, h),
                      sgwave.ricker_tensor(10.25, dt, nt))
        vp = torch.from_numpy(synth.field_slice(42 + i, nz, nx)).cuda()
        items.append((plan, vp, shots, torch.empty((nshot, geom.nrow, nx), dtype=torch.float32, device="cuda"), None))
        Nz, Nx = plan.padded_shape
        pts += Nz * Nx * nshot
    ws = torch.empty(sgwave.sg_batch_workspace_size(items), dtype=torch.uint8, device="cuda")
    tuning = sgwave.sg_batch_autotune(items, ws, 32)   # untimed
    sgwave.sg_batch_forward(items, ws, tuning)           # warm-up: records the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sgwave.sg_batch_forward(items, ws, tuning)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for it in items:
        sgwave.sg_check_finite(it[3], ws)
    rate = pts * (nt - 1) / (ms / 1e3) / 1e9
    return {"workload": "4 field slices 619x1000 @10 m + 60-cell sponge (679x1120 padded) x 64 shots, dt 1 ms, "
                        "nt 8001, 1000 receivers, gathers decimated by 14 -> [64][572][1000] per slice",
            "ms": ms, "value": rate, "unit": "Gpt-updates/s", "tuning": tuning,
            "ratio_to_forward_value": rate / fwd_rate if fwd_rate else None}


def copy_reference(mib):
    """A device-to-device copy of `mib` MiB: a kernel of known traffic that
    calibrates the hardware byte counters."""
    if mib <= 0:
        return
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()


def residual_rate(passes=10):
    """Physics-residual pass (App. F.5) over the paper's saved wavefield stack
    of one shot: 572 frames (8001 levels decimated by 14) of 619 x 1000, free
    top, frame spacing 14 ms.  Seeded random frames: the pass does the same
    work for any values.  Algorithmic traffic: every frame and the velocity
    read once (4 B per cell), the sums written (16 B per frame)."""
    import torch
    from paper_2605_30541_amd import sgwave
    T, nz, nx = 572, 619, 1000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    frames = torch.randn((T, nz, nx), dtype=torch.float32, device="cuda", generator=gen)
    vp = torch.empty((nz, nx), dtype=torch.float32, device="cuda").uniform_(1500.0, 4500.0, generator=gen)
    sgwave.wave_residual(frames, vp, 10.0, 10.0, 14e-3)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(passes):
        res2, dtt2 = sgwave.wave_residual(frames, vp, 10.0, 10.0, 14e-3)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / passes
    ratio = float(torch.sqrt(res2.sum() / dtt2.sum()))
    algo = 4.0 * (T + 1) * nz * nx + 16.0 * T
    del frames
    return {"workload": "572 frames of 619x1000 (one shot's wavefields, 8001 levels decimated by 14), free top",
            "ms": ms, "frames_per_s": T / (ms / 1e3), "hbm_algorithmic_GBs": algo / (ms / 1e3) / 1e9,
            "frac_of_hbm_peak": algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, "residual_ratio": ratio}


def builder_rate(passes=3):
    """Builder modules at the paper's model shape, 619 x 1000 x 1000 voxels at
    10 m (App. C): a 4-octave fractal-noise displacement (max 90 m) and the
    Squish warp it drives, then one listric normal fault across the model;
    and a Deposit band of 40 beds, 200 cells at 2.5 m over the same area.
    The input is a seeded layered volume built on the device.  Algorithmic
    traffic: each voxel read and written once (8 B)."""
    import numpy as np
    import torch
    from paper_2605_30541_amd import sgwave
    nz, ny, nx, h = 619, 1000, 1000, 10.0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13)
    z = torch.arange(nz, device="cuda", dtype=torch.float32)[:, None, None]
    x = torch.arange(nx, device="cuda", dtype=torch.float32)[None, None, :]
    y = torch.arange(ny, device="cuda", dtype=torch.float32)[None, :, None]
    v = (1600.0 + 4.0 * z + 150.0 * torch.remainder(torch.floor((z + 3.0 * torch.sin(x / 40.0 + y / 55.0)) / 12.0), 3.0)
         ).contiguous()
    lattice = torch.rand((4, 8, 8), device="cuda", generator=gen) * 2.0 - 1.0
    fault = dict(cz=3000.0, cy=5000.0, cx=5000.0, azimuth_deg=30.0, dip_deg=60.0, radius=6000.0, slip=120.0,
                 direction=1, die_r=1500.0, die_strike=4500.0, die_theta_deg=35.0)
    shift = sgwave.fractal_noise2d(lattice, ny, nx, h, h, 2500.0, 4000.0, 20.0, 90.0)
    out = sgwave.squish(v, h, shift)
    out2 = sgwave.fault(out, h, h, h, fault, 1500.0)     # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(passes):
        shift = sgwave.fractal_noise2d(lattice, ny, nx, h, h, 2500.0, 4000.0, 20.0, 90.0)
        out = sgwave.squish(v, h, shift, stream=None)
    ev[1].record()
    ev[2].record()
    for _ in range(passes):
        out2 = sgwave.fault(out, h, h, h, fault, 1500.0)
    ev[3].record()
    torch.cuda.synchronize()
    ms_sq = ev[0].elapsed_time(ev[1]) / passes
    ms_f = ev[2].elapsed_time(ev[3]) / passes
    # a subsidiary-size fault (R 800 m, die-off 150 m / 400 m / 20 deg): only its box is processed
    small = dict(cz=3000.0, cy=4000.0, cx=6000.0, azimuth_deg=45.0, dip_deg=60.0, radius=800.0, slip=30.0,
                 direction=-1, die_r=150.0, die_strike=400.0, die_theta_deg=20.0)
    out3 = sgwave.fault(out, h, h, h, small, 1500.0)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(passes):
        out3 = sgwave.fault(out, h, h, h, small, 1500.0)
    ev[1].record()
    torch.cuda.synchronize()
    ms_fs = ev[0].elapsed_time(ev[1]) / passes
    del out3
    # the primary and its Riedel-shear subsidiaries (25 candidates, the paper's 20-30 per primary;
    # subsidiaries at 0.15 of the primary's size, 0.2-0.5 of its slip, 500 m apart) in one sequence
    cfg = dict(synthetic_fraction=0.85, hangingwall_fraction=0.75, synthetic_offset_deg=15.0,
               antithetic_offset_deg=165.0, along_strike=3000.0, across_min=300.0, across_max=2000.0,
               size_scale=0.15, slip_min=0.2, slip_max=0.5, min_distance=500.0)
    subs = sgwave.riedel_subsidiaries(fault, cfg, np.random.default_rng(17).random((25, 5)))
    seq = [fault] + subs
    ws = torch.empty_like(out)
    out3 = sgwave.fault_sequence(out, h, h, h, seq, 1500.0, ws=ws)
    torch.cuda.synchronize()
    ev[0].record()
    out3 = sgwave.fault_sequence(out, h, h, h, seq, 1500.0, ws=ws)
    ev[1].record()
    torch.cuda.synchronize()
    ms_seq = ev[0].elapsed_time(ev[1])
    del out3, ws
    nvox = nz * ny * nx
    moved = float((out2 != out).float().mean())
    del v, out, out2
    # Deposit: a 200-cell band of 40 beds over the same 1000 x 1000 area
    tb, nb = 200, 40
    thick = torch.clamp(torch.randn(nb, device="cuda", generator=gen) * 1.5 + tb / nb, min=0.5)
    vbed = torch.randn(nb, device="cuda", generator=gen) * 150.0 + 2600.0
    eta = torch.stack([sgwave.fractal_noise2d(torch.rand((3, 8, 8), device="cuda", generator=gen) * 2.0 - 1.0,
                                              ny, nx, h, h, 1500.0, 2000.0, 10.0 * i, 1.0) for i in range(nb - 1)])
    tex = torch.rand((16, 16, 16), device="cuda", generator=gen) * 2.0 - 1.0
    off = torch.rand(nb, device="cuda", generator=gen) * 500.0
    dargs = (tb, ny, nx, h / 4, h, h, thick, vbed, 0.3, eta, 3.0, tex, (12.0, 400.0, 400.0), off, 50.0, 0.1, 0.1)
    band = sgwave.deposit(*dargs)     # warm-up
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(passes):
        band = sgwave.deposit(*dargs)
    ev[1].record()
    torch.cuda.synchronize()
    ms_d = ev[0].elapsed_time(ev[1]) / passes
    del band, eta
    # the same band with simplex contact and texture fields, and the sinusoidal bedform mode
    perm_b = torch.randperm(256, device="cuda", generator=gen).to(torch.int32)
    perm_t = torch.randperm(256, device="cuda", generator=gen).to(torch.int32)
    sargs = (tb, ny, nx, h / 4, h, h, thick, vbed, 0.3, perm_b, (40.0, 1500.0, 2000.0), 3.0, perm_t,
             (12.0, 400.0, 400.0), off, 50.0, 0.1, 0.1)
    freq = torch.rand(tb, device="cuda", generator=gen) * 0.08 + 0.04
    rug = sgwave.fractal_noise2d(torch.rand((3, 8, 8), device="cuda", generator=gen) * 2.0 - 1.0, ny, nx, h, h,
                                 1500.0, 2000.0, 0.0, 1.0)
    wargs = (tb, ny, nx, h / 4, h, h, 2600.0, 0.3, freq, 4.0, 150.0, 60.0, 0.8, rug, 0.1, perm_t,
             (12.0, 400.0, 400.0), 50.0, 0.1, 0.1)
    band = sgwave.deposit_simplex(*sargs)
    band = sgwave.deposit_sinusoidal(*wargs)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(passes):
        band = sgwave.deposit_simplex(*sargs)
    ev[1].record()
    ev[2].record()
    for _ in range(passes):
        band = sgwave.deposit_sinusoidal(*wargs)
    ev[3].record()
    torch.cuda.synchronize()
    ms_ds = ev[0].elapsed_time(ev[1]) / passes
    ms_dw = ev[2].elapsed_time(ev[3]) / passes
    del band, rug
    # SaltSDT: three rotated ellipsoids (radii 0.8-2 km); each body's field from
    # the GRF step (sg_grf: white noise on the 1024^3 periodic grid, spectral
    # exponent p = 2, correlation lengths l_k = max(r_k f_k, 5) cells with
    # f = (0.2, 0.2, 0.3)), a = 0.15, water above 1500 m/s
    nbody = 3
    v = (1500.0 + 3.0 * z).expand(nz, ny, nx).contiguous()
    centres = np.array([[3000.0, 4000.0, 5000.0], [4200.0, 7000.0, 2500.0], [2000.0, 2500.0, 7500.0]])
    radii = np.array([[1500.0, 2000.0, 1800.0], [1000.0, 1400.0, 900.0], [800.0, 900.0, 1200.0]])
    grid, gbytes = sgwave.grf_grid(nz, ny, nx)
    gws = torch.empty(gbytes, dtype=torch.uint8, device="cuda")
    grf = torch.empty((nbody, nz, ny, nx), dtype=torch.float32, device="cuda")
    ms_grf = 0.0
    for i in range(nbody):
        noise = torch.randn(grid, dtype=torch.float32, device="cuda", generator=gen)
        ell = tuple(max(r / h * f, 5.0) for r, f in zip(radii[i], (0.2, 0.2, 0.3)))
        torch.cuda.synchronize()
        ev[0].record()
        grf[i] = sgwave.grf(noise, (nz, ny, nx), ell, 2.0, ws=gws)
        ev[1].record()
        torch.cuda.synchronize()
        ms_grf += ev[0].elapsed_time(ev[1])
        del noise
    del gws
    ang = np.array([[0.3, -0.2, 0.8], [-0.5, 0.1, 0.3], [0.2, 0.4, -1.0]])
    rots = []
    for a, b, c in ang:
        ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
        rots.append(np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]]) @ np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
                    @ np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]]))
    sargs = (v, h, h, h, centres, radii, np.array(rots), grf, 0.15, 4500.0, 1500.0, 1000)
    salted, smask = sgwave.salt_sdt(*sargs)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    salted, smask = sgwave.salt_sdt(*sargs)
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    salt_frac = float(smask.float().mean())
    del v, grf, salted, smask
    return {"workload": "619x1000x1000 voxels @10 m; squish 90 m max shift, 4 octaves; one fault "
                        "(R 6 km, slip 120 m, die-off 1.5 km / 4.5 km / 35 deg)",
            "salt_bodies": nbody, "grf_ms_per_body": ms_grf / nbody,
            "grf_grid": list(grid), "salt_ms": ms_s, "salt_Gvoxel_per_s": nvox / (ms_s / 1e3) / 1e9,
            "salt_fraction": salt_frac,
            "squish_ms": ms_sq, "squish_Gvoxel_per_s": nvox / (ms_sq / 1e3) / 1e9,
            "squish_frac_of_hbm_peak": 8.0 * nvox / (ms_sq / 1e3) / 1e9 / HBM_PEAK_GBS,
            "fault_ms": ms_f, "fault_Gvoxel_per_s": nvox / (ms_f / 1e3) / 1e9, "small_fault_ms": ms_fs,
            "fault_moved_fraction": moved, "fault_sequence_faults": len(seq), "fault_sequence_ms": ms_seq,
            "deposit_simplex_ms": ms_ds, "deposit_sinusoidal_ms": ms_dw,
            "deposit_band": "200 x 1000 x 1000 cells (2.5 m vertical), 40 beds", "deposit_ms": ms_d,
            "deposit_Gvoxel_per_s": tb * ny * nx / (ms_d / 1e3) / 1e9}


def batched_gradient_rate(fwd_rate, shots_per_wave, tuning=None, nt=10000):
    """4 field slices of uneven size (nz 500-620, nx 801-1001) x 100 shots
    spread evenly over the full width, nt 10000 at 0.8 ms, receivers on every
    column: forward with checkpoints every 100 levels, segment recompute and
    adjoint for all slices in one launch per time block, in waves of
    `shots_per_wave` shots per slice; random residuals stand in for dJ/dd."""
    import torch
    from paper_2605_30541_amd import sgwave, synth
    from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots
    dt, nshot, ckpt = 8e-4, 100, 100
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    items, pts = [], 0
    for i, (nz, nx) in enumerate(synth.uneven_sizes(42, 4, nz_range=(500, 620), nx_range=(801, 1001))):
        geom = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0)
        plan = Plan(geom)
        W = (nx - 1) * 10.0
        shots = Shots(synth.shot_line(nshot, 0.0, W), synth.surface_receivers(nx, 10.0),
                      sgwave.ricker_tensor(12.0, dt, nt))
        v0 = torch.from_numpy(synth.smoothed_1d(synth.field_slice(42 + i, nz, nx), 500.0, 10.0)).cuda()
        resid = torch.randn((nshot, geom.nrow, nx), dtype=torch.float32, device="cuda", generator=gen)
        items.append((plan, v0, shots, resid, torch.empty_like(v0)))
        Nz, Nx = plan.padded_shape
        pts += Nz * Nx * nshot
    ws = torch.empty(sgwave.sg_batch_grad_workspace_size(items, ckpt, shots_per_wave), dtype=torch.uint8,
                     device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sgwave.sg_batch_adjoint_gradient(items, ws, ckpt, shots_per_wave, tuning=tuning)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for it in items:
        sgwave.sg_check_finite(it[4], ws)
    rate = pts * (nt - 1) / (ms / 1e3) / 1e9
    return {"workload": "4 uneven field slices (nz 500-620, nx 801-1001, 40-cell sponge) x 100 shots, nt %d, "
                        "forward with checkpoints every 100 levels + segment recompute + adjoint, "
                        "%d shots per slice per wave" % (nt, shots_per_wave),
            "ms": ms, "value": rate, "unit": "Gpt-steps/s (padded points x time steps x shots)",
            "forward_tuning": tuning, "workspace_GB": ws.numel() / 1e9, "ratio_to_forward_value": rate / fwd_rate if fwd_rate else None}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported "
              "(shots shard across GPUs with no communication, see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    want = (lambda leg: args.only in (None, leg))
    out = {}
    if args.only not in (None, "batch"):
        # a profiling run of one sub-workload: print its record only
        if args.only == "field_shot":
            out["field_shot"], _ = field_shot_rate(args.field_steps, parse_tuning(args.field_tuning))
        elif args.only == "gradient":
            from paper_2605_30541_amd import synth
            out["gradient"] = gradient_rate(synth.field_slice(42, 620, 1001), None, parse_tuning(args.grad_tuning),
                                            args.grad_levels)
        elif args.only == "batched_gradient":
            out["batched_gradient"] = batched_gradient_rate(None, args.shots_per_wave,
                                                            parse_tuning(args.batched_grad_tuning), args.grad_levels)
        elif args.only == "paper":
            out["paper_workload"] = paper_workload_rate(None)
        elif args.only == "residual":
            out["physics_residual"] = residual_rate()
        elif args.only == "builder":
            out["builder"] = builder_rate()
        copy_reference(args.copy_mib)
        print(json.dumps(out), flush=True)
        return

    head, cases = batch_headline(args)
    value = head["value"]
    log("headline batch: %.1f Gpt-updates/s" % value)
    out = {
        "metric": "Gpt-updates/s & %HBM roofline: fwd vs fwd+adjoint grad, 1 MI355X, <=1e-4 rel L2",
        "value": value,
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched forward: 8 field slices of uneven size (nz 400-620 x nx 601-1001 @10 m, "
                               "seeds 42-49, 40-cell sponge, free surface) x 64 shots each, dt 0.8 ms, nt %d, "
                               "12 Hz Ricker, receivers on every surface column, one launch per time block "
                               "replayed from a hipGraph, batch-autotuned tiling" % args.levels,
                   "slices": 8, "shots_per_slice": 64, "padded_points_x_shots": head["points"],
                   "updates_per_step": head["updates_per_step"], "tuning": head["tuning"]},
        "roofline": head["roofline"],
        "cpu_baseline": None,
    }
    if args.only is None:
        out["field_shot"], v = field_shot_rate(args.field_steps, parse_tuning(args.field_tuning))
        log("field shot: %.1f Gpt-updates/s" % out["field_shot"]["value"])
        out["gradient"] = gradient_rate(v, value, parse_tuning(args.grad_tuning), args.grad_levels)
        log("gradient: %.1f Gpt-steps/s" % out["gradient"]["value"])
        out["batched_gradient"] = batched_gradient_rate(value, args.shots_per_wave,
                                                        parse_tuning(args.batched_grad_tuning), args.grad_levels)
        log("batched gradient: %.1f Gpt-steps/s" % out["batched_gradient"]["value"])
        out["paper_workload"] = paper_workload_rate(value)
        log("paper-shaped batch: %.1f Gpt-updates/s" % out["paper_workload"]["value"])
        out["physics_residual"] = residual_rate()
        log("physics residual: %.3f ms per 572-frame stack" % out["physics_residual"]["ms"])
        out["builder"] = builder_rate()
        log("builder: squish %.2f ms, fault %.1f ms per 619x1000x1000 volume, deposit %.2f ms per band" % (
            out["builder"]["squish_ms"], out["builder"]["fault_ms"], out["builder"]["deposit_ms"]))
    copy_reference(args.copy_mib)
    if not args.no_cpu_baseline and args.levels == 10000:
        log("timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_sample_slices)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
