"""GPU parity on the degenerate and boundary cases of the method, against the
FP64 oracle (relative L2 <= 1e-4, exact zeros where the result is zero):
grids smaller than one tile, a single time step, no receivers, a time step at
the paper's CFL bound, a decimation longer than the record, zero sources and
zero residuals."""
import os

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu
TOL = 1e-4
TUNINGS = [dict(variant=1), dict(variant=2, tile_x=128, tile_z=64, time_block=4),
           dict(variant=2, tile_x=64, tile_z=64, time_block=1), dict(variant=2, tile_x=64, tile_z=64, time_block=3)]
TIDS = ["naive", "t128x64b4", "t64x64b1", "t64x64b3"]


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        assert np.all(np.asarray(a) == 0.0)
        return 0.0
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / nb)


def grid_receivers(nz, nx, h):
    """A receiver on every grid node."""
    zz, xx = np.meshgrid(np.arange(nz) * h, np.arange(nx) * h, indexing="ij")
    return np.stack([zz.ravel(), xx.ravel()], 1)


def both(g: Geometry, v, src, rec, wl, tuning):
    import torch
    plan = Plan(g)
    plan.set_tuning(**tuning)
    w = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(wl), np.float32)).cuda()
    gd, gs = sgwave.forward(plan, torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda(), Shots(src, rec, w))
    torch.cuda.synchronize()
    og = oracle.Geometry(nz=g.nz, nx=g.nx, dz=g.dz, dx=g.dx, dt=g.dt, nt=g.nt, nbl=g.nbl,
                         top_free=g.top == sgwave.SG_TOP_FREE, R=g.damp_R)
    od, os_ = oracle.forward(og, np.asarray(v, np.float64), src, np.atleast_2d(wl).astype(np.float64), rec,
                             rec_every=g.rec_every, snap_every=g.snap_every or 1, snap_count=g.snap_count)
    return (gd.cpu().numpy() if gd is not None else None, gs.cpu().numpy() if gs is not None else None), (od, os_)


@pytest.mark.parametrize("tuning", TUNINGS, ids=TIDS)
@pytest.mark.parametrize("nz,nx,nbl,nt,top", [(5, 7, 0, 2, sgwave.SG_TOP_FREE), (5, 7, 3, 40, sgwave.SG_TOP_FREE),
                                              (3, 200, 2, 60, sgwave.SG_TOP_ABSORBING),
                                              (150, 4, 5, 50, sgwave.SG_TOP_FREE)],
                         ids=["5x7-rigid-1step", "5x7-sponge3", "3x200-absorbing", "150x4"])
def test_grids_smaller_than_a_tile(nz, nx, nbl, nt, top, tuning):
    """Padded grids far smaller than one loaded tile (every tile is an edge
    tile, the halo reaches past every side), down to a single time step; a
    receiver on every node and every level as a snapshot."""
    h = 10.0
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=1e-3, nt=nt, nbl=nbl, top=top, vmax_hint=2500.0,
                 snap_every=1, snap_count=nt)
    rng = np.random.default_rng(nz * 1000 + nx)
    v = rng.uniform(1500.0, 2500.0, (nz, nx)).astype(np.float32)
    src = np.array([[(nz // 2) * h + 3.0, (nx // 2) * h + 1.5]])
    wl = oracle.ricker(40.0, 1e-3, nt, t0=0.01)
    (gd, gs), (od, os_) = both(g, v, src, grid_receivers(nz, nx, h), wl, tuning)
    e = rel_l2(gd[0], od[0])
    print("gather rel-L2 %.3e" % e, flush=True)
    assert e <= TOL
    for j in range(nt):
        assert rel_l2(gs[0, j], os_[0, j]) <= TOL, j


@pytest.mark.parametrize("tuning", TUNINGS[:2], ids=TIDS[:2])
def test_snapshots_only_without_receivers(tuning):
    g = Geometry(nz=40, nx=90, dz=10.0, dx=10.0, dt=1e-3, nt=120, nbl=10, vmax_hint=3000.0,
                 snap_every=20, snap_count=6)
    v = np.full((40, 90), 2500.0, np.float32)
    v[20:] = 3000.0
    (gd, gs), (od, os_) = both(g, v, np.array([[50.0, 455.0]]), np.zeros((0, 2)), oracle.ricker(20.0, 1e-3, 120),
                               tuning)
    assert gd is None
    for j in range(6):
        assert rel_l2(gs[0, j], os_[0, j]) <= TOL, j


@pytest.mark.parametrize("tuning", TUNINGS[:2], ids=TIDS[:2])
def test_time_step_at_the_paper_cfl_bound(tuning):
    """dt equal to the paper's bound at vmax (accepted by the plan) on a
    homogeneous 4500 m/s model: stable and at parity over 800 steps."""
    h, vmax = 10.0, 4500.0
    dt = sgwave.sg_cfl_dt_max(h, h, vmax)
    g = Geometry(nz=60, nx=80, dz=h, dx=h, dt=dt, nt=800, nbl=15, vmax_hint=vmax)
    v = np.full((60, 80), vmax, np.float32)
    rec = np.stack([np.full(80, 10.0), np.arange(80) * h], 1)
    (gd, _), (od, _) = both(g, v, np.array([[300.0, 400.0]]), rec, oracle.ricker(15.0, dt, 800), tuning)
    assert np.all(np.isfinite(gd))
    e = rel_l2(gd[0], od[0])
    print("gather rel-L2 %.3e" % e, flush=True)
    assert e <= TOL


def test_decimation_longer_than_the_record_keeps_level_zero_only():
    g = Geometry(nz=30, nx=40, dz=10.0, dx=10.0, dt=1e-3, nt=50, nbl=5, vmax_hint=2000.0, rec_every=53)
    (gd, _), (od, _) = both(g, np.full((30, 40), 2000.0, np.float32), np.array([[100.0, 200.0]]),
                            np.array([[10.0, 50.0], [20.0, 300.0]]), oracle.ricker(20.0, 1e-3, 50),
                            TUNINGS[1])
    assert gd.shape == (1, 1, 2) and od.shape == (1, 1, 2)
    assert np.all(gd == 0.0) and np.all(od == 0.0)


@pytest.mark.parametrize("tuning", TUNINGS, ids=TIDS)
def test_zero_wavelet_gives_exact_zeros(tuning):
    g = Geometry(nz=50, nx=70, dz=10.0, dx=10.0, dt=1e-3, nt=90, nbl=8, vmax_hint=3000.0,
                 snap_every=30, snap_count=3)
    (gd, gs), _ = both(g, np.full((50, 70), 3000.0, np.float32), np.array([[15.0, 345.0], [250.0, 100.0]]),
                       grid_receivers(5, 7, 10.0), np.zeros((2, 90)), tuning)
    assert np.all(gd == 0.0) and np.all(gs == 0.0)


def _gradient(g, v, src, rec, wl, resid, ckpt):
    import torch
    plan = Plan(g)
    vp = torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda()
    shots = Shots(src, rec, torch.from_numpy(np.ascontiguousarray(np.atleast_2d(wl), np.float32)).cuda())
    ws = torch.empty(sgwave.sg_grad_workspace_size(plan, shots.nshot, shots.nrec, ckpt), dtype=torch.uint8,
                     device="cuda")
    gathers = torch.empty((shots.nshot, g.nrow, shots.nrec), dtype=torch.float32, device="cuda")
    sgwave.sg_forward_ckpt(plan, vp, shots, ckpt, gathers, ws)
    grad = torch.empty_like(vp)
    sgwave.sg_adjoint_gradient(plan, vp, shots, ckpt, torch.from_numpy(resid).cuda(), grad, ws)
    torch.cuda.synchronize()
    return grad.cpu().numpy()


def test_zero_residual_gives_an_exactly_zero_gradient():
    g = Geometry(nz=40, nx=60, dz=10.0, dx=10.0, dt=1e-3, nt=150, nbl=8, vmax_hint=3000.0)
    rec = np.stack([np.full(60, 10.0), np.arange(60) * 10.0], 1)
    grad = _gradient(g, np.full((40, 60), 2500.0), np.array([[20.0, 300.0]]), rec, oracle.ricker(20.0, 1e-3, 150),
                     np.zeros((1, g.nrow, 60), np.float32), 13)
    assert np.all(grad == 0.0)


@pytest.mark.parametrize("nt,ckpt", [(3, 0), (3, 1), (17, 5)])
def test_short_records_gradient(nt, ckpt):
    """Gradients over very short records (two updates), checkpoint spacing 1
    and a spacing that does not divide the record, on a small grid."""
    h = 10.0
    g = Geometry(nz=12, nx=15, dz=h, dx=h, dt=1e-3, nt=nt, nbl=3, vmax_hint=3000.0)
    rng = np.random.default_rng(nt)
    v = rng.uniform(2000.0, 3000.0, (12, 15))
    src = np.array([[40.0, 70.0]])
    rec = grid_receivers(12, 15, h)
    wl = rng.standard_normal(nt)
    resid = rng.standard_normal((1, g.nrow, rec.shape[0])).astype(np.float32)
    og = oracle.Geometry(nz=12, nx=15, dz=h, dx=h, dt=1e-3, nt=nt, nbl=3)
    ref = oracle.gradient(og, v, src, wl[None], rec, resid.astype(np.float64))
    got = _gradient(g, v, src, rec, wl, resid, ckpt)
    e = rel_l2(got, ref)
    print("gradient rel-L2 %.3e" % e, flush=True)
    assert e <= TOL


def test_binding_rejects_mismatched_device_tensors():
    """Wrong dtype, shape, contiguity or wavelet length are refused by the
    binding with ValueError before anything reaches the library."""
    import torch
    g = Geometry(nz=30, nx=40, dz=10.0, dx=10.0, dt=1e-3, nt=50, nbl=5, vmax_hint=3000.0)
    plan = Plan(g)
    src = np.array([[10.0, 200.0]])
    rec = np.stack([np.full(40, 10.0), np.arange(40) * 10.0], 1)
    w = torch.zeros((1, g.nt), dtype=torch.float32, device="cuda")
    vp = torch.full((g.nz, g.nx), 2000.0, device="cuda")
    ws = torch.empty(sgwave.sg_forward_workspace_size(plan, 1, 40), dtype=torch.uint8, device="cuda")
    gathers = torch.empty((1, g.nrow, 40), device="cuda")
    sh = Shots(src, rec, w)
    bad = [
        dict(vp=vp.double()),                                          # float64 velocity
        dict(vp=vp[:, :39]),                                           # short rows
        dict(vp=torch.full((g.nx, g.nz), 2000.0, device="cuda").t()),  # transposed view
        dict(gathers=torch.empty((1, g.nrow - 1, 40), device="cuda")), # short gathers
        dict(shots=Shots(src, rec, w[:, :g.nt - 1])),                  # short wavelet
        dict(shots=Shots(src, rec, torch.zeros((2, g.nt), device="cuda"))),   # 2 wavelet rows, 1 shot
        dict(ws=torch.empty(64, dtype=torch.float32, device="cuda")),  # workspace not bytes
    ]
    for case in bad:
        args = dict(vp=vp, shots=sh, gathers=gathers, ws=ws)
        args.update(case)
        with pytest.raises(ValueError):
            sgwave.sg_forward(plan, args["vp"], args["shots"], args["gathers"], None, args["ws"])
    sgwave.sg_forward(plan, vp, sh, gathers, None, ws)       # the good call passes
    torch.cuda.synchronize()
