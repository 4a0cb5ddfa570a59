"""GPU parity at the largest grids the plan accepts, where the oracle cannot
run the whole domain: 18000 x 16000 cells (a stored field of 289 M cells,
above 2^28, so the FP64 imaging accumulator's byte offsets pass 2^31).

Over nt steps a wave moves at most 4 cells per step (the stencil's reach), so
with the source and receivers deep inside the grid nothing reaches a boundary:
the oracle on a 401 x 401 crop around them computes exactly the same gathers
and the same gradient, and the gradient outside the crop is exactly zero."""
import os

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_largest_grid_forward_and_gradient_match_the_oracle_on_a_crop():
    import torch
    nz, nx, h, dt, nt, ckpt, nbl = 18000, 16000, 10.0, 1e-3, 24, 8, 20
    zc, xc, half = 9000, 8000, 200
    assert 4 * nt + 12 < half                                  # nothing reaches the crop's edges
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, vmax_hint=3000.0)
    plan = Plan(g)
    Nz, Nx = plan.padded_shape
    pitch = -(-(Nx + 8) // 32) * 32
    assert (Nz + 8) * pitch > (1 << 28)
    print("largest grid: %d x %d physical, padded %d x %d" % (nz, nx, Nz, Nx), flush=True)

    # smooth velocity in [2000, 3000] m/s, built on the device
    zz = torch.arange(nz, device="cuda", dtype=torch.float64)[:, None]
    xx = torch.arange(nx, device="cuda", dtype=torch.float64)[None, :]
    vp = (2500.0 + 300.0 * torch.sin(zz / 37.0) * torch.cos(xx / 53.0) + 150.0 * torch.sin((zz + xx) / 11.0)).float()
    del zz, xx
    rng = np.random.default_rng(2024)
    src = np.array([[zc * h + 3.0, xc * h - 4.5]])
    rec = np.stack([(zc + rng.integers(-10, 11, 6)) * h + rng.uniform(0, h, 6),
                    (xc + rng.integers(-10, 11, 6)) * h + rng.uniform(0, h, 6)], 1)
    wl = rng.standard_normal(nt)
    resid = rng.standard_normal((1, nt, rec.shape[0])).astype(np.float32)
    shots = Shots(src, rec, torch.from_numpy(wl[None].astype(np.float32)).cuda())

    ws = torch.empty(sgwave.sg_grad_workspace_size(plan, 1, rec.shape[0], ckpt), dtype=torch.uint8, device="cuda")
    print("workspace %.1f GB" % (ws.numel() / 1e9), flush=True)
    gathers = torch.empty((1, nt, rec.shape[0]), dtype=torch.float32, device="cuda")
    sgwave.sg_forward_ckpt(plan, vp, shots, ckpt, gathers, ws)
    grad = torch.empty_like(vp)
    sgwave.sg_adjoint_gradient(plan, vp, shots, ckpt, torch.from_numpy(resid).cuda(), grad, ws)
    torch.cuda.synchronize()
    print("GPU forward + gradient done", flush=True)
    del ws

    z0, x0 = zc - half, xc - half
    crop = (slice(z0, z0 + 2 * half + 1), slice(x0, x0 + 2 * half + 1))
    v_crop = vp[crop].double().cpu().numpy()
    g_crop = grad[crop].cpu().numpy()
    outside = grad.clone()
    outside[crop] = 0.0
    assert float(outside.abs().max()) == 0.0
    del outside

    og = oracle.Geometry(nz=2 * half + 1, nx=2 * half + 1, dz=h, dx=h, dt=dt, nt=nt, nbl=0)
    off = np.array([z0 * h, x0 * h])
    od, _ = oracle.forward(og, v_crop, src - off, wl[None], rec - off)
    ograd = oracle.gradient(og, v_crop, src - off, wl[None], rec - off, resid.astype(np.float64))
    e_d = rel_l2(gathers.cpu().numpy()[0], od[0])
    e_g = rel_l2(g_crop, ograd)
    print("gathers rel-L2 %.3e, gradient rel-L2 %.3e" % (e_d, e_g), flush=True)
    assert e_d <= TOL and e_g <= TOL
