"""Pins of the oracle's adjoint and velocity gradient (no GPU): the dot-product
test of the transpose, central finite differences of the misfit, and
invariance to the checkpoint spacing of the recompute."""
import numpy as np
import pytest

import oracle
from oracle import Geometry
from test_oracle_scheme import layered


def _setup(seed=0, nz=22, nx=30, nt=260, nbl=8, top_free=True):
    h, dt = 10.0, 1e-3
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, top_free=top_free)
    v = layered(nz, nx, h, seed=seed, noise=0.05)
    rng = np.random.default_rng(seed + 100)
    rec = np.stack([np.full(nx - 1, 10.0), np.arange(nx - 1) * h + 3.3], 1)
    return g, v, rng, rec


@pytest.mark.parametrize("top_free,rec_every", [(True, 1), (True, 3), (False, 2)])
def test_adjoint_dot_product(top_free, rec_every):
    """<F w, r> == <w, F^T r> for random off-grid point sources and data."""
    g, v, rng, rec = _setup(seed=1, top_free=top_free)
    nshot, nsrc = 2, 3
    src = np.stack([rng.uniform(0, (g.nz - 1) * g.dz, (nshot, nsrc)),
                    rng.uniform(0, (g.nx - 1) * g.dx, (nshot, nsrc))], -1)
    wl = rng.standard_normal((nshot, nsrc, g.nt))
    d, _ = oracle.forward(g, v, src, wl, rec, rec_every=rec_every)
    r = rng.standard_normal(d.shape)
    _, wg = oracle.gradient(g, v, src, wl, rec, r, rec_every=rec_every, want_wavelet_grad=True)
    lhs, rhs = float(np.sum(d * r)), float(np.sum(wl * wg))
    assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(d) * np.linalg.norm(r))
    assert abs(lhs) > 1e-6 * np.linalg.norm(d) * np.linalg.norm(r)


def test_gradient_matches_central_differences():
    g, v, rng, rec = _setup(seed=2, nt=300)
    src = np.array([[10.0, 73.0], [10.0, 211.0]])
    w = oracle.ricker(15.0, g.dt, g.nt)
    v_true = v.copy()
    v_true[9:14, 10:18] *= 1.08
    d_obs, _ = oracle.forward(g, v_true, src, w, rec)

    def J(vv):
        d, _ = oracle.forward(g, vv, src, w, rec)
        return oracle.misfit(d, d_obs)
    d, _ = oracle.forward(g, v, src, w, rec)
    grad = oracle.gradient(g, v, src, w, rec, d - d_obs)
    gmax = np.abs(grad).max()
    assert gmax > 0
    cells = [(0, 5), (1, 0), (g.nz - 1, g.nx - 1), (g.nz - 1, 3), (7, g.nx - 1), (4, 0)]
    cells += [tuple(x) for x in np.stack([rng.integers(0, g.nz, 14), rng.integers(0, g.nx, 14)], 1)]
    for (iz, ix) in cells:
        eps = 1e-5 * v[iz, ix]   # FD truncation error ~ eps^2 (checked: x100 per decade)
        vp, vm = v.copy(), v.copy()
        vp[iz, ix] += eps
        vm[iz, ix] -= eps
        fd = (J(vp) - J(vm)) / (2 * eps)
        if iz == 0:
            # the free surface pins row 0: v there moves nothing
            assert grad[iz, ix] == 0.0 and abs(fd) <= 1e-12 * gmax
            continue
        assert abs(fd - grad[iz, ix]) <= 1e-6 * max(abs(grad[iz, ix]), 1e-3 * gmax), (iz, ix, fd, grad[iz, ix])


def test_gradient_is_linear_in_residual_and_independent_of_checkpointing():
    g, v, rng, rec = _setup(seed=3, nt=157)
    src = np.array([[20.0, 101.0]])
    w = oracle.ricker(20.0, g.dt, g.nt)
    r = rng.standard_normal((1, g.nt, rec.shape[0]))
    g_def = oracle.gradient(g, v, src, w, rec, r)
    for ck in (1, 2, 7, 156, 400):
        assert np.array_equal(oracle.gradient(g, v, src, w, rec, r, ckpt=ck), g_def), ck
    g2 = oracle.gradient(g, v, src, w, rec, 2.5 * r)
    assert np.allclose(g2, 2.5 * g_def, rtol=1e-12, atol=1e-12 * np.abs(g_def).max())


def test_gradient_sums_over_shots():
    g, v, rng, rec = _setup(seed=4, nt=120)
    src = np.array([[10.0, 61.0], [30.0, 222.0], [10.0, 150.0]])
    w = oracle.ricker(20.0, g.dt, g.nt)
    r = rng.standard_normal((3, g.nt, rec.shape[0]))
    total = oracle.gradient(g, v, src, w, rec, r)
    parts = sum(oracle.gradient(g, v, src[i:i + 1], w, rec, r[i:i + 1]) for i in range(3))
    assert np.allclose(total, parts, rtol=1e-12, atol=1e-13 * np.abs(total).max())
