"""GPU parity of the batched path at the full sizes of its workloads, in the
launch configuration the benchmark times (batch-autotuned tiling, hipGraph
replay, gradient in shot waves):

* uneven field slices (the 8-slice batched forward's generator: sizes from
  rng(42) with nz 400-620, nx 601-1001, slice i seeded 42 + i), 10000 levels
  of 0.8 ms, shots of the workload's 64-shot line, receivers on every column;
* the full-density batched gradient (slices of nz 500-620, nx 801-1001,
  shots spread over the full width, checkpoints every 100 levels, two shots
  per slice per wave) against the oracle's gradients stored by
  golden/make_batched_gradient.py;
* the paper's production shape (619 x 1000 at 10 m, 60-cell sponge, dt 1 ms,
  8001 levels, gathers and snapshots every 14 levels) on the batched path.

Relative L2 <= 1e-4 against the FP64 oracle for every compared gather,
snapshot and gradient."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave, synth
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_batched_gradient as c5golden  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-4
GOLDEN_C5 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_gradient_c5.npz")


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))


def rel_l2(a, b):
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _batch(full, tuning):
    import torch
    ws = torch.empty(sgwave.sg_batch_workspace_size(full), dtype=torch.uint8, device="cuda")
    if tuning is None:
        tuning = sgwave.sg_batch_autotune(full, ws, 32)
    sgwave.sg_batch_forward(full, ws, tuning)
    torch.cuda.synchronize()
    return tuning


@pytest.mark.parametrize("given", [None, dict(variant=3, tile_x=256, tile_z=320, time_block=4)],
                         ids=["autotuned", "sweep-s256z320b4"])
def test_uneven_slices_batched_full_length_against_oracle(given):
    """Three slices of the batched forward's generator (419 x 681, 571 x 638,
    544 x 812) x 4 shots of each slice's 64-shot line (shots 0, 21, 42, 63), all
    10000 levels in one batched call with the autotuned tiling, and with the
    tiling the benchmark's autotuner picks for the full batch: two shots of the
    largest slice against the oracle, every shot of every slice finite and
    equal to its single-slice call under the same tiling."""
    import torch
    dt, nt, pick = 8e-4, 10000, [0, 21, 42, 63]
    full, cases = [], []
    for i, (nz, nx) in enumerate(synth.uneven_sizes(42, 8)[:3]):
        g = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0)
        v = synth.field_slice(42 + i, nz, nx)
        src = synth.shot_line(64, 1100.0, (nx - 1) * 10.0 - 1100.0)[pick]
        rec = synth.surface_receivers(nx, 10.0)
        shots = Shots(src, rec, sgwave.ricker_tensor(12.0, dt, nt))
        gathers = torch.full((len(pick), g.nrow, nx), float("nan"), device="cuda")
        full.append((Plan(g), torch.from_numpy(v).cuda(), shots, gathers, None))
        cases.append((g, v, src, rec))
    tuning = _batch(full, given)
    print("batch tiling:", tuning, flush=True)
    for (plan, vp, shots, gathers, _), (g, v, src, rec) in zip(full, cases):
        assert torch.isfinite(gathers).all()
        plan.set_tuning(**tuning)
        single = torch.empty_like(gathers)
        ws = torch.empty(sgwave.sg_forward_workspace_size(plan, shots.nshot, shots.nrec), dtype=torch.uint8,
                         device="cuda")
        sgwave.sg_forward(plan, vp, shots, single, None, ws)
        torch.cuda.synchronize()
        plan.clear_tuning()
        assert torch.equal(single, gathers)
    g, v, src, rec = cases[2]
    got = full[2][3].cpu().numpy()
    og = oracle.Geometry(nz=g.nz, nx=g.nx, dz=g.dz, dx=g.dx, dt=g.dt, nt=g.nt, nbl=g.nbl)
    for k in (0, 3):
        od, _ = oracle.forward(og, v.astype(np.float64), src[k:k + 1], oracle.ricker(12.0, dt, nt), rec)
        e = rel_l2(got[k], od[0])
        print("slice 2 shot %d: 10000-level gather rel-L2 %.3e" % (pick[k], e), flush=True)
        assert e <= TOL


@pytest.mark.parametrize("tuning", [None, dict(variant=3, tile_x=256, tile_z=160, time_block=3),
                                    dict(variant=3, tile_x=256, tile_z=160, time_block=4)],
                         ids=["tiled", "sweep-s256z160b3", "sweep-s256z160b4"])
def test_full_density_batched_gradient_against_stored_oracle_gradients(tuning):
    """Two slices of the full-density batched-gradient workload (510 x 888
    with 4 shots including both edge shots, 593 x 973 with 2), 10000 levels,
    checkpoints every 100, two shots per slice per wave, through
    sg_batch_adjoint_gradient: with the default tiling, and with the forward
    and the recompute on the column sweep (the adjoint stays on the tiled
    kernel) at time blocks 3 and 4, the latter as the benchmark runs it.  The
    GPU forms each residual from its own FP32
    gathers on the true and start models; the reference gradients and misfits
    are the FP64 oracle's."""
    import torch
    ref = np.load(GOLDEN_C5)
    h, dt, nt, ckpt = 10.0, 8e-4, 10000, 100
    w = sgwave.ricker_tensor(12.0, dt, nt)
    items, misfits = [], []
    for i in range(2):
        nz, nx, v_true, v0, src, rec = c5golden.slice_case(i)
        g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, vmax_hint=4500.0)
        plan = Plan(g)
        shots = Shots(src, rec, w)
        ws = torch.empty(sgwave.sg_forward_workspace_size(plan, shots.nshot, nx), dtype=torch.uint8, device="cuda")
        d_obs = torch.empty((shots.nshot, g.nrow, nx), dtype=torch.float32, device="cuda")
        d = torch.empty_like(d_obs)
        vp = torch.from_numpy(v0).cuda()
        sgwave.sg_forward(plan, torch.from_numpy(v_true).cuda(), shots, d_obs, None, ws)
        sgwave.sg_forward(plan, vp, shots, d, None, ws)
        resid = d - d_obs
        del d, d_obs, ws
        misfits.append(0.5 * float((resid.double() ** 2).sum()))
        items.append((plan, vp, shots, resid, torch.full_like(vp, float("nan"))))
    ws = torch.empty(sgwave.sg_batch_grad_workspace_size(items, ckpt, 2), dtype=torch.uint8, device="cuda")
    sgwave.sg_batch_adjoint_gradient(items, ws, ckpt, 2, tuning=tuning)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        e_m = abs(misfits[i] - float(ref["misfit%d" % i])) / float(ref["misfit%d" % i])
        e = rel_l2(it[4].cpu().numpy(), ref["grad%d" % i])
        print("slice %d (%d shots): misfit rel err %.3e, gradient rel-L2 %.3e" % (i, it[2].nshot, e_m, e),
              flush=True)
        assert e_m <= TOL
        assert e <= TOL


@pytest.mark.parametrize("given", [None, dict(variant=3, tile_x=256, tile_z=0, time_block=5)],
                         ids=["autotuned", "sweep-s256z0b5"])
def test_paper_shape_on_the_batched_path_against_oracle(given):
    """Two 619 x 1000 slices (seeds 7 and 8) at 10 m, 60-cell sponge, dt 1 ms,
    8001 levels, 1000 receivers, gathers decimated by k = 14 (572 samples per
    trace) and snapshots every 14 levels over the first 5 s (358 frames), two
    shots per slice in one batched call with the autotuned tiling, and with
    the tiling the benchmark's autotuner picks for the full paper-shaped batch:
    one shot per slice against the oracle, its gathers and all 358 snapshots."""
    import torch
    nz, nx, h = 619, 1000, 10.0
    srcs = [synth.shot_line(64, 1100.0, (nx - 1) * h - 1100.0)[[5, 40]],
            synth.shot_line(64, 1100.0, (nx - 1) * h - 1100.0)[[17, 58]]]
    full, cases = [], []
    for i, seed in enumerate((7, 8)):
        g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=1e-3, nt=8001, nbl=60, vmax_hint=4500.0, rec_every=14,
                     snap_every=14, snap_count=358)
        assert g.nrow == 572
        v = synth.field_slice(seed, nz, nx)
        rec = synth.surface_receivers(nx, h)
        shots = Shots(srcs[i], rec, sgwave.ricker_tensor(10.25, g.dt, g.nt))
        gathers = torch.empty((2, g.nrow, nx), dtype=torch.float32, device="cuda")
        snaps = torch.empty((2, g.snap_count, nz, nx), dtype=torch.float32, device="cuda")
        full.append((Plan(g), torch.from_numpy(v).cuda(), shots, gathers, snaps))
        cases.append((g, v, srcs[i], rec))
    tuning = _batch(full, given)
    print("batch tiling:", tuning, flush=True)
    for i, k in ((0, 0), (1, 1)):
        g, v, src, rec = cases[i]
        og = oracle.Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=g.dt, nt=g.nt, nbl=g.nbl)
        od, os_ = oracle.forward(og, v.astype(np.float64), src[k:k + 1], oracle.ricker(10.25, g.dt, g.nt), rec,
                                 rec_every=14, snap_every=14, snap_count=358)
        gd = full[i][3][k].cpu().numpy()
        e = rel_l2(gd, od[0])
        worst = 0.0
        for j in range(1, 358):
            s = full[i][4][k, j].cpu().numpy()
            worst = max(worst, rel_l2(s, os_[0, j]))
        del os_
        print("slice %d shot %d: gather rel-L2 %.3e, worst of 357 snapshots %.3e" % (i, k, e, worst), flush=True)
        assert e <= TOL and worst <= TOL
        assert np.all(full[i][4][k, 0].cpu().numpy() == 0.0)
