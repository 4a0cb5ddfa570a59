"""GPU parity of the column-sweep forward kernel (tuning variant 3): the same
update expression as the tiled kernel, so every gather and snapshot equals
the tiled kernel's bit for bit, and the FP64 oracle's to relative L2 <= 1e-4.
Covers strips of 128 and 256 columns with time blocks 1..6, the whole height
or segments of 8 to 45 rows (several per strip, receivers and sources in
every segment), free and
absorbing tops, sources and receivers on and next to the free-surface rows,
off-grid positions, decimated receivers, snapshots, grids narrower than a
strip or only a few rows high, and the batched launch over uneven slices."""
import os

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave, synth
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu
TOL = 1e-4
TILED = dict(variant=2, tile_x=64, tile_z=64, time_block=3)


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        assert np.all(np.asarray(a) == 0.0)
        return 0.0
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / nb)


def run(g, v, src, rec, wl, tuning):
    import torch
    plan = Plan(g)
    plan.set_tuning(**tuning)
    w = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(wl), np.float32)).cuda()
    gd, gs = sgwave.forward(plan, torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda(), Shots(src, rec, w))
    torch.cuda.synchronize()
    return (gd.cpu().numpy() if gd is not None else None, gs.cpu().numpy() if gs is not None else None)


def run_oracle(g, v, src, rec, wl):
    og = oracle.Geometry(nz=g.nz, nx=g.nx, dz=g.dz, dx=g.dx, dt=g.dt, nt=g.nt, nbl=g.nbl,
                         top_free=g.top == sgwave.SG_TOP_FREE, R=g.damp_R)
    return oracle.forward(og, np.asarray(v, np.float64), src, np.atleast_2d(wl).astype(np.float64), rec,
                          rec_every=g.rec_every, snap_every=g.snap_every or 1, snap_count=g.snap_count)


def check(g, v, src, rec, wl, tuning):
    a = run(g, v, src, rec, wl, tuning)
    b = run(g, v, src, rec, wl, TILED)
    ref = run_oracle(g, v, src, rec, wl)
    for k in range(len(src)):
        if a[0] is not None:
            assert np.array_equal(a[0][k], b[0][k]), "gathers differ from the tiled kernel"
            assert rel_l2(a[0][k], ref[0][k]) <= TOL
        if a[1] is not None:
            assert np.array_equal(a[1], b[1]), "snapshots differ from the tiled kernel"
            for j in range(1, a[1].shape[1]):
                assert rel_l2(a[1][k, j], ref[1][k, j]) <= TOL


SWEEPS = [dict(variant=3, tile_x=128, time_block=tb) for tb in (1, 2, 3, 4, 5, 6)] + \
         [dict(variant=3, tile_x=256, time_block=tb) for tb in (1, 3, 4, 6)] + \
         [dict(variant=3, tile_x=256, tile_z=z, time_block=tb) for z, tb in ((8, 1), (17, 4), (30, 6), (45, 3))]
SIDS = ["s128b%d" % t for t in (1, 2, 3, 4, 5, 6)] + ["s256b%d" % t for t in (1, 3, 4, 6)] + \
       ["s256z%db%d" % zt for zt in ((8, 1), (17, 4), (30, 6), (45, 3))]


@pytest.mark.parametrize("tuning", SWEEPS, ids=SIDS)
@pytest.mark.parametrize("top", [sgwave.SG_TOP_FREE, sgwave.SG_TOP_ABSORBING], ids=["free", "absorbing"])
def test_sweep_equals_tiled_and_oracle(tuning, top):
    """A ragged field slice (91 x 301 at 10 m, 12-cell sponge), three shots:
    one on row 1, one off-grid at 23.4 m depth, one off-grid at 503.3 m;
    receivers on row 1 at every column plus off-grid ones from 17.5 m to 555.5
    m depth, one on the last row and a vertical array with a receiver in every
    row (base rows on every segment's last rows); snapshots every 37 levels."""
    nz, nx, h, nt = 91, 301, 10.0, 260
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=8e-4, nt=nt, nbl=12, vmax_hint=4500.0, top=top,
                 snap_every=37, snap_count=7)
    v = synth.field_slice(11, nz, nx)
    src = np.array([[10.0, 400.0], [23.4, 1513.7], [503.3, 2907.0]])
    rec = np.concatenate([synth.surface_receivers(nx, h),
                          np.array([[17.5, 55.5], [41.0, 1777.7], [17.5, 2996.0], [0.0, 1200.0],
                                    [400.0, 1500.0], [555.5, 2222.2], [899.0, 640.0]]),
                          np.stack([np.arange(nz - 1) * 10.0 + 2.5, np.full(nz - 1, 1733.3)], 1)])
    wl = np.stack([oracle.ricker(14.0 + 3 * k, g.dt, nt) for k in range(3)])
    check(g, v, src, rec, wl, tuning)


@pytest.mark.parametrize("tuning", [dict(variant=3, tile_x=128, time_block=4),
                                    dict(variant=3, tile_x=256, time_block=2)], ids=["s128b4", "s256b2"])
@pytest.mark.parametrize("nz,nx,nbl,nt,rec_every", [(5, 7, 0, 30, 1), (3, 200, 2, 60, 3), (150, 4, 5, 50, 1),
                                                     (40, 390, 30, 120, 7)])
def test_sweep_small_and_narrow_grids(tuning, nz, nx, nbl, nt, rec_every):
    """Grids narrower than a strip, only a few rows high, a sponge wider than
    the physical grid, decimated receivers."""
    g = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=1e-3, nt=nt, nbl=nbl, vmax_hint=3500.0, rec_every=rec_every)
    v = synth.flat_layers(nz, nx, 10.0, [0.0, 10.0 * (nz // 2)], [1800.0, 3200.0])
    src = np.array([[min(10.0, 10.0 * (nz - 1)), 10.0 * (nx // 2)]])
    rec = np.stack([np.full(nx, min(10.0, 10.0 * (nz - 1))), np.arange(nx) * 10.0], 1)
    check(g, v, src, rec, oracle.ricker(20.0, g.dt, nt), tuning)


@pytest.mark.parametrize("tuning", [dict(variant=3, tile_x=128, time_block=3),
                                    dict(variant=3, tile_x=256, time_block=5),
                                    dict(variant=3, tile_x=256, tile_z=20, time_block=4)],
                         ids=["s128b3", "s256b5", "s256z20b4"])
def test_sweep_batched_uneven_slices(tuning):
    """The batched launch over four uneven slices with 3, 1, 2, 2 shots:
    equal to the tiled batch bit for bit and to the oracle."""
    import torch
    sizes, nshots, nt = [(50, 70), (41, 93), (66, 155), (30, 330)], [3, 1, 2, 2], 300
    items, cases = [], []
    for i, ((nz, nx), ns) in enumerate(zip(sizes, nshots)):
        g = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=8e-4, nt=nt, nbl=12, vmax_hint=4500.0,
                     snap_every=50, snap_count=6)
        v = synth.field_slice(20 + i, nz, nx)
        W = (nx - 1) * 10.0
        src = synth.shot_line(ns, 0.2 * W, 0.8 * W, depth=12.5)
        rec = synth.surface_receivers(nx, 10.0)
        wl = np.stack([oracle.ricker(15.0 + 2 * j, g.dt, nt) for j in range(ns)])
        items.append((Plan(g), torch.from_numpy(v).cuda(), Shots(src, rec, torch.from_numpy(wl.astype(np.float32)).cuda())))
        cases.append((g, v, src, rec, wl))
    a = sgwave.batch_forward(items, tuning)
    b = sgwave.batch_forward(items, TILED)
    torch.cuda.synchronize()
    for (ga, sa), (gb, sb), (g, v, src, rec, wl) in zip(a, b, cases):
        assert torch.equal(ga, gb) and torch.equal(sa, sb)
        od, os_ = run_oracle(g, v, src, rec, wl)
        ga, sa = ga.cpu().numpy(), sa.cpu().numpy()
        for k in range(len(src)):
            assert rel_l2(ga[k], od[k]) <= TOL
            for j in range(1, os_.shape[1]):
                assert rel_l2(sa[k, j], os_[k, j]) <= TOL


def _receivers(layout, nx):
    """surface: every column at 10 m; vertical: off-grid ones plus a column
    of eight receivers (more nodes in one column than a thread keeps);
    dense: every column at three off-grid depths (more nodes per strip than
    the adjoint sums in LDS)."""
    surf = synth.surface_receivers(nx, 10.0)
    if layout == "surface":
        return surf
    if layout == "vertical":
        col = np.stack([np.arange(8) * 31.0 + 15.0, np.full(8, 733.0)], 1)
        odd = np.array([[17.5, 55.5], [41.0, 1177.7], [0.0, 120.0], [555.5, 222.2], [689.0, 640.0]])
        return np.concatenate([surf[::3], col, odd])
    x = np.arange(nx - 1) * 10.0 + 3.3
    return np.concatenate([np.stack([np.full(nx - 1, d), x], 1) for d in (12.5, 27.5, 44.0)])


@pytest.mark.parametrize("tuning", [dict(variant=3, tile_x=128, time_block=4),
                                    dict(variant=3, tile_x=256, tile_z=24, time_block=3),
                                    dict(variant=3, tile_x=128, tile_z=8, time_block=6)],
                         ids=["s128b4", "s256z24b3", "s128z8b6"])
@pytest.mark.parametrize("layout,top", [("surface", sgwave.SG_TOP_FREE), ("vertical", sgwave.SG_TOP_FREE),
                                        ("dense", sgwave.SG_TOP_ABSORBING), ("surface", sgwave.SG_TOP_ABSORBING),
                                        ("dense", sgwave.SG_TOP_FREE)],
                         ids=["surface", "vertical", "dense-absorbing", "surface-absorbing", "dense-free"])
def test_gradient_with_sweep_forward_and_recompute(tuning, layout, top):
    """Forward with checkpoints and the segment recompute on the column sweep,
    the adjoint on the tiled kernel: gathers and gradient equal the all-tiled
    gradient calls bit for bit (same ring values, same adjoint) and the
    oracle's gradient to 1e-4; the batched form (shot waves) equals the
    all-tiled batched form bit for bit.  Receiver layouts: a surface line,
    receivers at many depths incl. a column of eight, three dense off-grid
    lines; both tops."""
    import torch
    nz, nx, nt, ckpt = 70, 150, 260, 29
    g = Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=8e-4, nt=nt, nbl=12, vmax_hint=4500.0, rec_every=2, top=top)
    v = synth.field_slice(31, nz, nx)
    src = np.array([[10.0, 300.0], [37.5, 1111.0]])
    rec = _receivers(layout, nx)
    wl = np.stack([oracle.ricker(16.0, g.dt, nt), oracle.ricker(19.0, g.dt, nt)])
    w = torch.from_numpy(wl.astype(np.float32)).cuda()
    vp = torch.from_numpy(v).cuda()
    rng = np.random.default_rng(5)
    nrec = len(rec)
    resid_np = rng.standard_normal((2, g.nrow, nrec)).astype(np.float32)
    resid = torch.from_numpy(resid_np).cuda()
    out = {}
    for name, tn in (("sweep", tuning), ("tiled", None)):
        plan = Plan(g)
        if tn:
            plan.set_tuning(**tn)
        sh = Shots(src, rec, w)
        ws = torch.empty(sgwave.sg_grad_workspace_size(plan, 2, nrec, ckpt), dtype=torch.uint8, device="cuda")
        gathers = torch.empty((2, g.nrow, nrec), device="cuda")
        grad = torch.empty_like(vp)
        sgwave.sg_forward_ckpt(plan, vp, sh, ckpt, gathers, ws)
        sgwave.sg_adjoint_gradient(plan, vp, sh, ckpt, resid, grad, ws)
        torch.cuda.synchronize()
        out[name] = (gathers.cpu().numpy(), grad.cpu().numpy())
    assert np.array_equal(out["sweep"][0], out["tiled"][0])
    og = oracle.Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=g.dt, nt=nt, nbl=12,
                         top_free=top == sgwave.SG_TOP_FREE)
    ref = oracle.gradient(og, v.astype(np.float64), src, wl, rec, resid_np.astype(np.float64), rec_every=2)
    e = rel_l2(out["sweep"][1], ref)
    print("%s %s: gradient vs oracle %.2e" % (layout, tuning, e), flush=True)
    assert np.array_equal(out["sweep"][1], out["tiled"][1])
    assert e <= TOL
    # batched form, one shot per wave
    items_out = []
    for tn in (tuning, None):
        plan = Plan(g)
        items = [(plan, vp, Shots(src, rec, w), resid, torch.empty_like(vp))]
        wsb = torch.empty(sgwave.sg_batch_grad_workspace_size(items, ckpt, 1), dtype=torch.uint8, device="cuda")
        sgwave.sg_batch_adjoint_gradient(items, wsb, ckpt, 1, tuning=tn)
        torch.cuda.synchronize()
        items_out.append(items[0][4].cpu().numpy())
    assert np.array_equal(items_out[0], items_out[1])
    assert rel_l2(items_out[0], ref) <= TOL
