"""Host run-ahead of the hot calls: three back-to-back forward calls on one
plan and one workspace, each with its own source position and outputs,
return before the GPU has finished them (the per-call tables go through the
plan's pinned staging slots, none of which has to be waited for), and every
result matches the FP64 oracle (relative L2 <= 1e-4)."""
import os
import time

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave, synth
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("batched", [False, True])
def test_three_back_to_back_calls_run_ahead_of_the_gpu(batched):
    import torch
    oracle.set_threads(min(16, os.cpu_count() or 1))
    nz, nx, h, nt = 300, 420, 10.0, 3000
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=8e-4, nt=nt, nbl=30, vmax_hint=4500.0)
    plan = Plan(g)
    v = synth.field_slice(5, nz, nx)
    vp = torch.from_numpy(v).cuda()
    rec = synth.surface_receivers(nx, h)
    w = sgwave.ricker_tensor(15.0, g.dt, nt)
    xs = (1005.0, 2330.0, 3610.0)
    shots = [Shots(np.array([[10.0 + 7.5 * k, x]]), rec, w) for k, x in enumerate(xs)]
    outs = [torch.empty((1, g.nrow, nx), dtype=torch.float32, device="cuda") for _ in xs]
    stream = torch.cuda.current_stream()
    if batched:
        ws = torch.empty(sgwave.sg_batch_workspace_size([(plan, vp, shots[0], outs[0], None)]), dtype=torch.uint8,
                         device="cuda")
        call = lambda k: sgwave.sg_batch_forward([(plan, vp, shots[k], outs[k], None)], ws, None, stream)
    else:
        ws = torch.empty(sgwave.sg_forward_workspace_size(plan, 1, nx), dtype=torch.uint8, device="cuda")
        call = lambda k: sgwave.sg_forward(plan, vp, shots[k], outs[k], None, ws, stream)
    call(0)                       # records the launch graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(3):
        call(k)
    host_s = time.perf_counter() - t0
    busy = not stream.query()
    e0 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    torch.cuda.synchronize()
    print("three calls enqueued in %.2f ms; stream still busy: %s" % (host_s * 1e3, busy), flush=True)
    assert busy
    og = oracle.Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=g.dt, nt=nt, nbl=g.nbl)
    for k, sh in enumerate(shots):
        od, _ = oracle.forward(og, v.astype(np.float64), sh.src_zx, oracle.ricker(15.0, g.dt, nt), rec)
        e = rel_l2(outs[k][0].cpu().numpy(), od[0])
        print("call %d (source x = %.0f m): rel-L2 %.2e" % (k, xs[k], e), flush=True)
        assert e <= TOL
