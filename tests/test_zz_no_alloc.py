"""The no-allocation forward (sg_forward_noalloc, static device scratch)
against sg_forward with a caller workspace, through the C ABI: two calls in a
row, the second on a smaller grid with fewer shots, each equal to sg_forward
bit for bit (same kernels and tiling) and the smaller one also within 1e-4
relative L2 of the FP64 oracle; a call needing more than the static scratch
is refused with SG_ENOSPACE and writes nothing."""
import os

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave, synth
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu


def _case(nz, nx, nshot, nt, snaps, seed):
    import torch
    g = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=8e-4, nt=nt, nbl=15, vmax_hint=4500.0,
                 snap_every=40 if snaps else 0, snap_count=(nt - 1) // 40 + 1 if snaps else 0)
    plan = Plan(g)
    v = synth.field_slice(seed, nz, nx)
    src = synth.shot_line(nshot, 0.2 * (nx - 1) * 10.0, 0.8 * (nx - 1) * 10.0)
    rec = synth.surface_receivers(nx, 10.0)
    shots = Shots(src, rec, sgwave.ricker_tensor(14.0, g.dt, nt))
    return g, plan, v, src, rec, shots, torch.from_numpy(v).cuda()


def _outputs(g, nshot, nx):
    import torch
    gathers = torch.full((nshot, g.nrow, nx), float("nan"), device="cuda")
    snaps = torch.full((nshot, g.snap_count, g.nz, g.nx), float("nan"), device="cuda") if g.snap_count else None
    return gathers, snaps


def test_noalloc_forward_equals_the_workspace_forward_twice():
    import torch
    oracle.set_threads(min(16, os.cpu_count() or 1))
    for (nz, nx, nshot, nt, snaps, seed) in ((180, 300, 3, 700, True, 3), (64, 128, 1, 400, False, 4)):
        g, plan, v, src, rec, shots, vp = _case(nz, nx, nshot, nt, snaps, seed)
        ga, sa = _outputs(g, nshot, nx)
        sgwave.sg_forward_noalloc(plan, vp, shots, ga, sa)
        gb, sb = _outputs(g, nshot, nx)
        ws = torch.empty(sgwave.sg_forward_workspace_size(plan, nshot, nx), dtype=torch.uint8, device="cuda")
        sgwave.sg_forward(plan, vp, shots, gb, sb, ws)
        torch.cuda.synchronize()
        print("%d x %d, %d shots: equal gathers %s" % (nz, nx, nshot, torch.equal(ga, gb)), flush=True)
        assert torch.equal(ga, gb)
        if snaps:
            assert torch.equal(sa, sb)
        og = oracle.Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=g.dt, nt=nt, nbl=g.nbl)
        od, _ = oracle.forward(og, v.astype(np.float64), src, oracle.ricker(14.0, g.dt, nt), rec)
        got = ga.cpu().numpy().astype(np.float64)
        for k in range(nshot):
            e = np.linalg.norm(got[k] - od[k]) / np.linalg.norm(od[k])
            assert e <= 1e-4, e


def test_noalloc_refuses_inputs_beyond_the_static_scratch():
    import torch
    g, plan, v, src, rec, shots, vp = _case(1400, 2000, 3, 50, False, 5)
    need = sgwave.sg_forward_workspace_size(plan, 3, 2000)
    assert need > (64 << 20)
    ga, _ = _outputs(g, 3, 2000)
    with pytest.raises(sgwave.SGError) as e:
        sgwave.sg_forward_noalloc(plan, vp, shots, ga, None)
    assert e.value.status == sgwave.SG_ENOSPACE
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(ga).all()
