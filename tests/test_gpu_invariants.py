"""Invariants of the discrete scheme checked on the GPU path itself, in FP32
(the FP64 oracle is pinned to them in the CPU tests): source-receiver
reciprocity with the sponge and off-grid positions (the Laplacian with its
boundary rules is symmetric, the damping diagonal, and a source and a receiver
use the same bilinear weights), and invariance under a horizontal flip of the
model and the acquisition (the stencil pairs x+m with x-m symmetrically)."""
import numpy as np
import pytest

from paper_2605_30541_amd import sgwave, synth
from paper_2605_30541_amd.sgwave import Geometry, Plan, Shots

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _shot(geom, v, src, rec):
    import torch
    plan = Plan(geom)
    vp = torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda()
    g, _ = sgwave.forward(plan, vp, Shots(np.asarray(src, np.float64).reshape(-1, 2),
                                          np.asarray(rec, np.float64).reshape(-1, 2),
                                          sgwave.ricker_tensor(15.0, geom.dt, geom.nt)))
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("top", [sgwave.SG_TOP_FREE, sgwave.SG_TOP_ABSORBING])
def test_source_receiver_reciprocity_on_the_gpu(top):
    geom = Geometry(nz=80, nx=130, dz=10.0, dx=10.0, dt=1e-3, nt=700, nbl=20, top=top, vmax_hint=4500.0)
    v = synth.field_slice(11, 80, 130)
    a, b = np.array([123.0, 217.5]), np.array([431.7, 1004.2])      # off-grid, (z, x) in metres
    ab = _shot(geom, v, a, b)[0, :, 0]
    ba = _shot(geom, v, b, a)[0, :, 0]
    e = _rel(ab, ba)
    print("reciprocity (top %d): rel %.2e, peak %.3e" % (top, e, np.abs(ba).max()), flush=True)
    assert np.abs(ba).max() > 0
    assert e <= 1e-5


def test_horizontal_flip_invariance_on_the_gpu():
    nz, nx, h = 70, 121, 10.0
    geom = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=1e-3, nt=600, nbl=20, vmax_hint=4500.0)
    v = synth.field_slice(12, nz, nx)
    rec = synth.surface_receivers(nx, h)
    W = (nx - 1) * h
    src = np.array([30.0, 413.7])
    g = _shot(geom, v, src, rec)[0]
    gf = _shot(geom, v[:, ::-1], np.array([src[0], W - src[1]]), rec)[0]
    e = _rel(gf[:, ::-1], g)
    print("horizontal flip: rel %.2e" % e, flush=True)
    assert e <= 1e-5
