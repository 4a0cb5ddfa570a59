"""Pins of the oracle's discrete scheme against closed forms, invariants and an
independent formulation (no GPU).

Each test is built so that a plausible slip in the oracle (a wrong stencil
weight or index, a wrong sign of the free-surface ghosts, the source entering
at the wrong time level or with the wrong cell scaling, an asymmetric
injection/sampling pair, a sponge in the wrong units) fails at least one.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import hankel1

import oracle
from oracle import Geometry


def layered(nz, nx, dz, seed=0, noise=0.03, vals=(1500.0, 2200.0, 3000.0)):
    rng = np.random.default_rng(seed)
    v = np.empty((nz, nx))
    edges = np.linspace(0, nz, len(vals) + 1).astype(int)
    for i, val in enumerate(vals):
        v[edges[i]:edges[i + 1]] = val
    v *= 1.0 + noise * rng.uniform(-1, 1, size=v.shape)
    return v


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- Laplacian

def test_laplacian_exact_on_polynomials_in_interior():
    g = Geometry(nz=30, nx=34, dz=2.0, dx=5.0, dt=1e-3, nt=2, nbl=0, top_free=False)
    v = np.full((g.nz, g.nx), 2000.0)
    Z, X = np.meshgrid(np.arange(g.nz) * g.dz, np.arange(g.nx) * g.dx, indexing="ij")
    for (a, b) in ((2, 0), (0, 2), (4, 3), (9, 0), (0, 9), (5, 6)):
        s = 1.0 / (Z.max() ** a * X.max() ** b + 1.0)
        p = s * Z ** a * X ** b
        exact = s * (a * (a - 1) * Z ** max(a - 2, 0) * X ** b * (a >= 2)
                     + b * (b - 1) * Z ** a * X ** max(b - 2, 0) * (b >= 2))
        lap = oracle.apply_laplacian(g, v, p)
        inner = (slice(4, -4), slice(4, -4))
        scale = np.abs(exact[inner]).max() + np.abs(p[inner]).max() / min(g.dz, g.dx) ** 2
        assert np.abs(lap[inner] - exact[inner]).max() <= 1e-11 * scale, (a, b)


def test_laplacian_rigid_outside_and_odd_mirror_at_free_top():
    rng = np.random.default_rng(3)
    g_rigid = Geometry(nz=12, nx=14, dz=10.0, dx=10.0, dt=1e-3, nt=2, nbl=0, top_free=False)
    v = np.full((12, 14), 2000.0)
    p = rng.standard_normal((12, 14))
    # rigid: same as embedding in a larger zero field
    big = np.zeros((12 + 8, 14 + 8))
    big[4:-4, 4:-4] = p
    gb = Geometry(nz=20, nx=22, dz=10.0, dx=10.0, dt=1e-3, nt=2, nbl=0, top_free=False)
    lb = oracle.apply_laplacian(gb, np.full((20, 22), 2000.0), big)[4:-4, 4:-4]
    assert np.allclose(oracle.apply_laplacian(g_rigid, v, p), lb, rtol=0, atol=1e-14)
    # free top: same as embedding in a field extended by the odd mirror about row 0
    g_free = Geometry(nz=12, nx=14, dz=10.0, dx=10.0, dt=1e-3, nt=2, nbl=0, top_free=True)
    p[0] = 0.0
    ext = np.zeros((12 + 11, 14 + 8))
    ext[11:, 4:-4] = p
    ext[:11, 4:-4] = -p[:0:-1]
    ge = Geometry(nz=23, nx=22, dz=10.0, dx=10.0, dt=1e-3, nt=2, nbl=0, top_free=False)
    le = oracle.apply_laplacian(ge, np.full((23, 22), 2000.0), ext)[11:, 4:-4]
    lf = oracle.apply_laplacian(g_free, v, p)
    assert np.allclose(lf[1:], le[1:], rtol=0, atol=1e-14)


# ----------------------------------------------------------- free surface

def test_free_surface_equals_odd_image_domain():
    """A free-surface run equals a run on the domain mirrored about z=0 with the
    sponge mirrored onto the top, a source +w at z_s and an image source -w at
    -z_s (method of images; App. E.2 'sign-flipped reflection')."""
    nz, nx, h = 24, 40, 10.0
    v = layered(nz, nx, h, seed=1)
    nt, dt, nbl = 260, 1e-3, 8
    w = oracle.ricker(18.0, dt, nt)
    src = np.array([[23.0, 187.0]])
    rec = np.stack([np.full(nx, 15.0), np.arange(nx) * h + 1.5], 1)[:-1]
    gf = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, top_free=True)
    d_free, s_free = oracle.forward(gf, v, src, w, rec, snap_every=13, snap_count=20)

    vm = np.concatenate([v[:0:-1], v], axis=0)             # rows -(nz-1)..nz-1
    gm = Geometry(nz=2 * nz - 1, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, top_free=False)
    z0 = (nz - 1) * h
    srcm = np.array([[[z0 + src[0, 0], src[0, 1]], [z0 - src[0, 0], src[0, 1]]]])
    wm = np.stack([w, -w])[None]
    recm = rec.copy()
    recm[:, 0] += z0
    d_img, s_img = oracle.forward(gm, vm, srcm, wm, recm, snap_every=13, snap_count=20)
    assert np.abs(d_free).max() > 0
    assert np.abs(d_free - d_img).max() <= 1e-12 * np.abs(d_free).max()
    assert np.abs(s_free - s_img[:, :, nz - 1:]).max() <= 1e-12 * np.abs(s_free).max()
    # z = 0 stays exactly zero in the image run too (odd symmetry)
    assert np.abs(s_img[:, :, nz - 1]).max() == 0.0


# ----------------------------------------------------------- energy

def _test_laplacian_matrix(nz, nx, dz, dx, free_top):
    """Independent sparse L: weights from the Taylor system, zero outside the
    grid, odd mirror about row 0 under a free top (row 0 itself excluded)."""
    from test_oracle_host import _taylor_weights
    c = [float(x) for x in _taylor_weights(4)]
    idx = lambda i, j: i * nx + j
    rows, cols, vals = [], [], []
    for i in range(nz):
        for j in range(nx):
            if free_top and i == 0:
                continue
            for m in range(-4, 5):
                wz, wx = c[abs(m)] / dz ** 2, c[abs(m)] / dx ** 2
                # z direction
                ii = i + m
                if 0 <= ii < nz:
                    rows.append(idx(i, j)); cols.append(idx(ii, j)); vals.append(wz)
                elif ii < 0 and free_top:
                    rows.append(idx(i, j)); cols.append(idx(-ii, j)); vals.append(-wz)
                jj = j + m
                if 0 <= jj < nx:
                    rows.append(idx(i, j)); cols.append(idx(i, jj)); vals.append(wx)
    L = sp.csr_matrix((vals, (rows, cols)), shape=(nz * nx, nz * nx))
    if free_top:   # row 0 carries p = 0: drop its column as well
        keep = np.ones(nz * nx)
        keep[:nx] = 0
        L = sp.diags(keep) @ L @ sp.diags(keep)
    return L


@pytest.mark.parametrize("free_top", [False, True])
def test_discrete_energy_is_conserved_without_sponge(free_top):
    nz, nx, h, dt, nt = 26, 30, 10.0, 1e-3, 400
    v = layered(nz, nx, h, seed=2, noise=0.05)
    w = oracle.ricker(20.0, dt, nt)
    w[90:] = 0.0                                    # source off after n = 90
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=0, top_free=free_top)
    _, snaps = oracle.forward(g, v, [[104.0, 143.0]], w, [[50.0, 50.0]], snap_every=1, snap_count=nt)
    P = snaps[0].reshape(nt, -1)
    L = _test_laplacian_matrix(nz, nx, h, h, free_top)
    m = 1.0 / v.ravel() ** 2
    E = np.array([np.sum(m * ((P[n + 1] - P[n]) / dt) ** 2) - P[n + 1] @ (L @ P[n])
                  for n in range(100, nt - 1)])
    assert E[0] > 0
    assert np.abs(E - E[0]).max() <= 1e-10 * E[0]


# ----------------------------------------------------------- reciprocity

def test_source_receiver_reciprocity_with_sponge_and_free_surface():
    nz, nx, h, dt, nt = 30, 44, 10.0, 1e-3, 500
    v = layered(nz, nx, h, seed=4, noise=0.05)
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=10, top_free=True)
    w = oracle.ricker(15.0, dt, nt)
    A, B = np.array([13.0, 61.7]), np.array([204.0, 377.2])
    dAB, _ = oracle.forward(g, v, A, w, B[None])
    dBA, _ = oracle.forward(g, v, B, w, A[None])
    assert np.abs(dAB).max() > 1e-3 * np.abs(w).max()
    assert np.abs(dAB - dBA).max() <= 1e-12 * np.abs(dAB).max()


# ----------------------------------------------------------- symmetries

def test_horizontal_flip_and_time_shift_are_exact():
    nz, nx, h, dt, nt = 20, 36, 10.0, 1e-3, 240
    v = layered(nz, nx, h, seed=5, noise=0.05)
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=6, top_free=True)
    w = oracle.ricker(15.0, dt, nt)
    src = np.array([[20.0, 123.4]])
    rec = np.stack([np.full(nx, 10.0), np.arange(nx) * h], 1)
    d, _ = oracle.forward(g, v, src, w, rec)
    W = (nx - 1) * h
    df, _ = oracle.forward(g, v[:, ::-1], [[20.0, W - 123.4]], w, rec[::-1])
    assert np.abs(d - df).max() <= 1e-13 * np.abs(d).max()
    j = 17
    ws = np.concatenate([np.zeros(j), w[:-j]])
    ds, _ = oracle.forward(g, v, src, ws, rec)
    assert np.array_equal(ds[0, j:], d[0, :-j])
    assert np.all(ds[0, :j] == 0)


# ----------------------------------------------------------- CFL

def _cfl_run(courant):
    n, h, vel = 40, 10.0, 2000.0
    dt = courant * h / vel
    nt = 500
    g = Geometry(nz=n, nx=n, dz=h, dx=h, dt=dt, nt=nt, nbl=0, top_free=False)
    rng = np.random.default_rng(11)
    zz, xx = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij")
    src = np.stack([zz.ravel(), xx.ravel()], 1)[None]
    wl = np.zeros((1, n * n, nt))
    wl[0, :, 0] = rng.standard_normal(n * n)          # random kick at n = 0
    _, snaps = oracle.forward(g, np.full((n, n), vel), src, wl, [[200.0, 200.0]],
                              snap_every=50, snap_count=10)
    return np.abs(snaps[0]).reshape(10, -1).max(1)


def test_cfl_von_neumann_threshold():
    stable = _cfl_run(0.99 * oracle.von_neumann_courant())
    unstable = _cfl_run(1.02 * oracle.von_neumann_courant())
    assert stable[-1] < 10 * stable[1]
    assert unstable[-1] > 1e6 * unstable[1]
    # the paper's (more conservative) bound is stable as well
    paper = _cfl_run(oracle.cfl_smax())
    assert paper[-1] < 10 * paper[1]


# ----------------------------------------------------------- Green's function

def _green_trace(h, dt, T, c, f0, r):
    """Oracle trace at distance r (along x) from a point source in a homogeneous
    medium large enough that nothing reflects inside the window."""
    nt = int(round(T / dt)) + 1
    half = int(math.ceil((c * T + r) / h)) // 2 + 6
    n = 2 * half + 1
    g = Geometry(nz=n, nx=n + int(round(r / h)), dz=h, dx=h, dt=dt, nt=nt, nbl=4, top_free=False)
    w = oracle.ricker(f0, dt, nt)
    zs, xs = half * h, half * h
    d, _ = oracle.forward(g, np.full((g.nz, g.nx), c), [[zs, xs]], w, [[zs, xs + r]])
    return d[0, :, 0], w


def _green_analytic(w, dt, c, r):
    """p = G *_t w with the 2D free-space Green's function of
    v^-2 p_tt - lap p = delta(x) delta(t); evaluated in frequency as
    (i/4) H0^(1)(omega r / c) under the e^{-i omega t} convention."""
    nt = len(w)
    nf = 8 * nt
    Wf = np.fft.rfft(w, n=nf)
    om = 2 * np.pi * np.fft.rfftfreq(nf, dt)
    G = np.zeros_like(Wf)
    G[1:] = np.conj(0.25j * hankel1(0, om[1:] * r / c))   # numpy's forward FFT uses e^{-i omega t}
    return np.fft.irfft(G * Wf, n=nf)[:nt]


def test_green_function_convergence():
    c, f0, r, T = 2000.0, 10.0, 200.0, 0.35
    errs = []
    for h, dt in ((10.0, 2.5e-3), (5.0, 1.25e-3)):
        tr, w = _green_trace(h, dt, T, c, f0, r)
        ref = _green_analytic(w, dt, c, r)
        # causality of the analytic trace: silent before the first arrival
        assert np.abs(ref[: int(0.5 * r / c / dt)]).max() < 1e-3 * np.abs(ref).max()
        errs.append(rel(tr, ref))
    assert errs[0] < 2e-2 and errs[1] < 5e-3, errs
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, errs          # second order in time


# ----------------------------------------------------------- sponge

def test_sponge_suppresses_edge_reflection():
    """The Cerjan sponge (units reading: eta in s/m^2 = paper value x 1e-3)
    leaves a reflection that falls as the layer widens, about 1 % at the
    paper's 60 cells for a receiver 50 m from the edge; a rigid edge reflects at
    order one.  A stiff sponge (the literal-SI reading) would reflect off its
    own front and would not fall like this."""
    c, h, dt, f0 = 2000.0, 10.0, 1e-3, 15.0
    nt = 700
    w = oracle.ricker(f0, dt, nt)
    n = 60

    def run(nbl, pad):
        g = Geometry(nz=n + 2 * pad, nx=n + 2 * pad, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, top_free=False)
        o = pad * h
        d, _ = oracle.forward(g, np.full((g.nz, g.nx), c), [[300.0 + o, 300.0 + o]],
                              w, [[300.0 + o, 50.0 + o]])
        return d[0, :, 0]
    ref = run(0, 120)                              # edges 1.2 km away: no reflection in window
    direct = np.abs(ref).max()
    refl = {nbl: np.abs(run(nbl, 0) - ref).max() / direct for nbl in (0, 20, 40, 60)}
    assert refl[0] > 0.3
    assert refl[20] > refl[40] > refl[60]
    assert refl[40] < 3e-2 and refl[60] < 1e-2, refl


# ----------------------------------------------------------- brute force

def _bruteforce_gathers(nz, nx, dz, dx, dt, nt, nbl, v, src, w, rec):
    """Independent formulation: assemble the whole space-time system of the
    scheme as one sparse lower block-triangular matrix and solve it directly."""
    from test_oracle_host import _taylor_weights
    c = [float(x) for x in _taylor_weights(4)]
    Nz, Nx = nz + nbl, nx + 2 * nbl
    N = Nz * Nx
    vp = v[np.clip(np.arange(Nz), 0, nz - 1)][:, np.clip(np.arange(Nx) - nbl, 0, nx - 1)]
    cd = 1.5 * math.log(1e3) / nbl

    def prof(d, h_):
        r = d / nbl
        return np.where(d > 0, cd / h_ * (r - np.sin(2 * np.pi * r) / (2 * np.pi)) * 1e-3, 0.0)
    I, J = np.meshgrid(np.arange(Nz), np.arange(Nx), indexing="ij")
    eta = prof(nbl - J, dx) + prof(J - (nbl + nx - 1), dx) + prof(I - (nz - 1), dz)
    gam = eta * vp ** 2 * dt / 2
    a, b = 1 / (1 + gam), (1 - gam) / (1 + gam)
    W = a * dt ** 2 * vp ** 2
    L = _test_laplacian_matrix(Nz, Nx, dz, dx, True)

    def point(z, x):
        fz, fx = z / dz, x / dx
        iz, ix = int(fz), int(fx)
        out = np.zeros(N)
        for di, wz in ((0, 1 - (fz - iz)), (1, fz - iz)):
            for dj, wx in ((0, 1 - (fx - ix)), (1, fx - ix)):
                if wz * wx:
                    out[(iz + di) * Nx + ix + dj + nbl] += wz * wx
        return out
    s_vec = point(*src) / (dx * dz)
    r_mat = np.stack([point(*q) for q in rec])
    keep = np.ones(N)
    keep[:Nx] = 0                                   # free top: row 0 pinned
    K = nt - 1                                      # unknown levels 1..nt-1
    I_N = sp.identity(N, format="csr")
    A = sp.diags(keep) @ (sp.diags(2 * a.ravel()) + sp.diags(W.ravel()) @ L)
    B = sp.diags(keep * b.ravel())
    blocks = [[None] * K for _ in range(K)]
    for k in range(K):
        blocks[k][k] = I_N
        if k >= 1:
            blocks[k][k - 1] = -A
        if k >= 2:
            blocks[k][k - 2] = B
    M = sp.bmat(blocks, format="csc")
    rhs = np.concatenate([keep * W.ravel() * s_vec * w[n] for n in range(K)])
    p = spla.spsolve(M, rhs).reshape(K, N)
    d = np.zeros((nt, len(rec)))
    d[1:] = p @ r_mat.T
    return d


def test_bruteforce_space_time_system():
    nz, nx, h, dt, nt, nbl = 6, 7, 10.0, 1e-3, 40, 3
    v = layered(nz, nx, h, seed=9, noise=0.1)
    w = oracle.ricker(40.0, dt, nt)
    src = (12.5, 31.0)
    rec = [(10.0, 0.0), (20.0, 44.0), (37.5, 60.0), (0.0, 20.0)]
    g = Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=nbl, top_free=True)
    d, _ = oracle.forward(g, v, [list(src)], w, rec)
    ref = _bruteforce_gathers(nz, nx, h, h, dt, nt, nbl, v, src, w, rec)
    assert np.abs(ref).max() > 0
    assert np.abs(d[0] - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("top_free", [True, False])
def test_wave_residual_closed_form_on_a_separable_mode(top_free):
    """u = cos(w t) sin(kz z) cos(kx x) (odd about z = 0, so the free-surface
    mirror holds exactly): the discrete second difference in time and the
    8th-order Laplacian act as multiplications by closed-form symbols, so
    R = u [(2 cos(w dt) - 2) / dt^2 - v^2 (sum_m c_m 2 (cos(m kz dz) - 1) / dz^2
    + sum_m c_m 2 (cos(m kx dx) - 1) / dx^2)] at every evaluated cell."""
    nz, nx, T, dz, dx, dt, vel = 30, 41, 7, 8.0, 11.0, 1.3e-3, 2300.0
    w, kz, kx = 2 * np.pi * 17.0, 2 * np.pi / 97.0, 2 * np.pi / 131.0
    t = np.arange(T)[:, None, None] * dt
    z = np.arange(nz)[None, :, None] * dz
    x = np.arange(nx)[None, None, :] * dx
    u = np.cos(w * t) * np.sin(kz * z) * np.cos(kx * x)
    c = [float(q) for q in oracle.fd_coefficients()]
    sym_t = (2 * np.cos(w * dt) - 2) / dt ** 2
    sym_l = sum(c[m] * 2 * (np.cos(m * kz * dz) - 1) for m in range(1, 5)) / dz ** 2 + \
        sum(c[m] * 2 * (np.cos(m * kx * dx) - 1) for m in range(1, 5)) / dx ** 2
    res2, dtt2 = oracle.wave_residual(u, np.full((nz, nx), vel), dz, dx, dt, top_free=top_free)
    z0 = 1 if top_free else 4
    for k in range(1, T - 1):
        cells = u[k, z0:nz - 4, 4:nx - 4]
        assert res2[k] == pytest.approx(np.sum((cells * (sym_t - vel ** 2 * sym_l)) ** 2), rel=1e-9)
        assert dtt2[k] == pytest.approx(np.sum((cells * sym_t) ** 2), rel=1e-9)
    assert res2[0] == res2[-1] == 0.0 and dtt2[0] == dtt2[-1] == 0.0


def test_wave_residual_vanishes_on_the_schemes_own_frames():
    """Frames of the scheme itself (rigid boundary, no sponge: a = 1,
    W = (v dt)^2) at the time step of the scheme satisfy the discrete wave
    equation exactly once the source has stopped: the residual is round-off."""
    nz, nx, dt, nt = 40, 50, 1e-3, 90
    g = oracle.Geometry(nz=nz, nx=nx, dz=10.0, dx=10.0, dt=dt, nt=nt, nbl=0, top_free=True)
    rng = np.random.default_rng(3)
    v = rng.uniform(2000.0, 3000.0, (nz, nx))
    wl = np.zeros(nt)
    wl[:25] = oracle.ricker(60.0, dt, 25)
    _, snaps = oracle.forward(g, v, np.array([[200.0, 250.0]]), wl[None], np.zeros((0, 2)),
                              snap_every=1, snap_count=nt)
    res2, dtt2 = oracle.wave_residual(snaps[0], v, 10.0, 10.0, dt, top_free=True)
    late = slice(30, nt - 1)
    assert np.sum(dtt2[late]) > 0
    assert np.sqrt(np.sum(res2[late]) / np.sum(dtt2[late])) < 1e-9
    # while the source acts the residual is the source term, not round-off
    assert np.sqrt(res2[10] / dtt2[10]) > 1e-3
