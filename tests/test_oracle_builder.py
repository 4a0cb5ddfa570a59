"""Pins of the builder oracle (Squish, Alg. 2; Fault, Alg. 3; the windowed-sinc
pull sampling) against what holds independently of its code: exact samples at
integer positions, analytic band-limited functions, exact shifts, rotation
invariants of the fault map, first-order symmetry of the fault slip, the
amplitude bound and lattice values of the fractal noise."""
import math

import numpy as np
import pytest

from oracle import builder as B


def test_sinc_is_exact_at_integer_positions_and_on_constants():
    rng = np.random.default_rng(1)
    V = rng.standard_normal((17, 3, 11))
    z, y, x = np.meshgrid(np.arange(17.0), np.arange(3.0), np.arange(11.0), indexing="ij")
    assert np.abs(B.sinc_sample_3d(V, z, y, x) - V).max() < 1e-14
    C = np.full((9, 4, 6), 2.5)
    s = rng.uniform(-3, 12, (50,))
    assert np.abs(B.sinc_sample_3d(C, s, s * 0.3, s * 0.5) - 2.5).max() < 1e-14


@pytest.mark.parametrize("period", [4.0, 8.0, 16.0, 64.0])
def test_sinc_reproduces_a_band_limited_cosine(period):
    """Interior samples of cos(2 pi z / P) at fractional positions against the
    function itself.  The window's error stays below 1e-3 of the amplitude
    from 4 to 64 samples per period; a plain truncated sinc (no window) is off
    by 7e-3 to 2e-1 and a window misplaced by one tap by ~1e-2."""
    n = 256
    z = np.arange(n, dtype=np.float64)
    V = np.cos(2 * np.pi * z / period)[:, None, None]
    s = np.linspace(60.3, 180.7, 301)
    got = B.sinc_sample_3d(V, s, np.zeros_like(s), np.zeros_like(s))
    err = np.abs(got - np.cos(2 * np.pi * s / period)).max()
    assert err < 1.2e-3, err


def test_sinc_weights_are_symmetric_about_the_sample_position():
    """Mirroring the axis mirrors the sample: the taps are centred."""
    rng = np.random.default_rng(6)
    v = rng.standard_normal(40)
    V, W = v[:, None, None], v[::-1].copy()[:, None, None]
    s = rng.uniform(5, 34, 50)
    a = B.sinc_sample_3d(V, s, 0 * s, 0 * s)
    b = B.sinc_sample_3d(W, 39 - s, 0 * s, 0 * s)
    assert np.abs(a - b).max() < 1e-13


def test_squish_shifts_columns_exactly_by_whole_cells_and_keeps_zero_shift():
    rng = np.random.default_rng(2)
    V = rng.standard_normal((40, 2, 5))
    dz = 12.5
    assert np.abs(B.squish(V, dz, np.zeros((2, 5))) - V).max() < 1e-14
    shift = np.array([[3, -2, 0, 5, 1], [-4, 2, 7, 0, -1]], np.float64) * dz
    out = B.squish(V, dz, shift)
    for iy in range(2):
        for ix in range(5):
            k = int(shift[iy, ix] / dz)
            zs = np.arange(40) + k
            ok = (zs >= 0) & (zs < 40)
            # (sin(pi k) is zero only to rounding: exact to 1e-13)
            assert np.abs(out[ok, iy, ix] - V[zs[ok], iy, ix]).max() < 1e-13
            # past the ends the edge value is replicated
            assert np.abs(out[~ok, iy, ix] - V[np.clip(zs[~ok], 0, 39), iy, ix]).max(initial=0.0) < 1e-13


def test_squish_of_a_smooth_profile_samples_it_at_the_shifted_depth():
    dz = 10.0
    z = np.arange(200) * dz
    prof = 2000.0 + 1.5 * z + 80.0 * np.sin(2 * np.pi * z / 600.0)
    V = np.broadcast_to(prof[:, None, None], (200, 3, 4)).copy()
    shift = np.array([[13.7, -42.2, 0.0, 77.1], [5.5, -5.5, 120.3, -0.4], [33.3, 1.0, -90.9, 64.0]])
    out = B.squish(V, dz, shift)
    zz = z[30:170, None, None] + shift[None]
    ref = 2000.0 + 1.5 * zz + 80.0 * np.sin(2 * np.pi * zz / 600.0)
    # (a 15 m/s-per-cell trend: the window's first-moment bias, ~5e-3 cells, leaves < 0.1 m/s;
    # a wrong sign or unit of the shift would be off by hundreds)
    assert np.abs(out[30:170] - ref).max() < 0.1         # of values ~2000-4600


def test_fractal_noise_hits_lattice_values_and_stays_in_bounds():
    rng = np.random.default_rng(3)
    lat = rng.uniform(-1, 1, (1, 5, 7))
    # one octave, azimuth 0, grid spacing = wavelength: every node is a lattice node
    dzf = B.fractal_noise2d(lat, 5, 7, 100.0, 100.0, 100.0, 100.0, 0.0, 30.0)
    assert np.abs(dzf - 30.0 * lat[0]).max() < 1e-12
    lat4 = rng.uniform(-1, 1, (4, 6, 6))
    f = B.fractal_noise2d(lat4, 50, 60, 10.0, 10.0, 170.0, 230.0, 37.0, 25.0)
    assert np.abs(f).max() <= 25.0 + 1e-12
    assert f.std() > 1.0
    # the lattice is periodic: a whole lattice period further gives the same field
    per_x = 6 * 230.0
    g = B.fractal_noise2d(lat4, 1, 60, 10.0, 10.0, 170.0, 230.0, 0.0, 25.0)
    lat_shift = B.fractal_noise2d(lat4, 1, 60 + int(per_x / 10.0), 10.0, 10.0, 170.0, 230.0, 0.0, 25.0)
    assert np.abs(lat_shift[0, int(per_x / 10.0):] - g[0]).max() < 1e-9


FAULT = dict(cz=300.0, cy=200.0, cx=400.0, azimuth_deg=25.0, dip_deg=55.0, radius=900.0, slip=60.0,
             direction=1, die_r=250.0, die_strike=300.0, die_theta_deg=25.0)


def _frame(p):
    a, th, R = math.radians(p["azimuth_deg"]), math.radians(p["dip_deg"]), p["radius"]
    n = np.array([math.sin(a), math.cos(a)])
    s = np.array([math.cos(a), -math.sin(a)])
    ct = np.array([p["cz"] - R * math.sin(th), p["cy"] - R * math.cos(th) * n[0], p["cx"] - R * math.cos(th) * n[1]])
    return n, s, ct


def test_fault_with_zero_slip_or_outside_the_taper_is_the_identity():
    rng = np.random.default_rng(4)
    V = rng.standard_normal((40, 30, 50))
    p = dict(FAULT, slip=0.0)
    assert np.abs(B.fault(V, 10.0, 10.0, 10.0, p, 1500.0) - V).max() < 1e-14
    (sz, sy, sx), w = B.fault_source(V.shape, 10.0, 10.0, 10.0, FAULT)
    out = B.fault(V, 10.0, 10.0, 10.0, FAULT, 1500.0)
    assert 0 < np.count_nonzero(w) < w.size
    assert np.abs(out[w == 0] - V[w == 0]).max() < 1e-13
    assert w.max() <= 1.0 and w.min() >= 0.0


def test_fault_map_is_a_rotation_about_the_cylinder_axis():
    """p_fwd = 2p - src keeps each voxel's distance to the axis and its
    along-strike offset, and turns it by -chi d w s / R."""
    shape, h = (40, 30, 50), 10.0
    (sz, sy, sx), w = B.fault_source(shape, h, h, h, FAULT)
    Z, Y, X = np.meshgrid(np.arange(40) * h, np.arange(30) * h, np.arange(50) * h, indexing="ij")
    fz, fy, fx = 2 * Z - sz, 2 * Y - sy, 2 * X - sx
    n, s, ct = _frame(FAULT)

    def cyl(z, y, x):
        hh = (y - ct[1]) * n[0] + (x - ct[2]) * n[1]
        vv = z - ct[0]
        return np.hypot(hh, vv), np.arctan2(vv, hh), (y - ct[1]) * s[0] + (x - ct[2]) * s[1]

    r0, t0, a0 = cyl(Z, Y, X)
    r1, t1, a1 = cyl(fz, fy, fx)
    assert np.abs(r1 - r0).max() < 1e-9
    assert np.abs(a1 - a0).max() < 1e-9
    chi = np.where(r0 >= FAULT["radius"], 1.0, -1.0)
    expect = -chi * FAULT["direction"] * w * FAULT["slip"] / FAULT["radius"]
    assert np.abs((t1 - t0) - expect).max() < 1e-12
    # the two walls move in opposite senses; the largest displacement is about the slip
    disp = np.sqrt((fz - Z) ** 2 + (fy - Y) ** 2 + (fx - X) ** 2)
    assert 0.7 * FAULT["slip"] < disp.max() <= 1.5 * FAULT["slip"]


def test_fault_direction_reverses_the_slip_to_first_order():
    shape, h = (30, 20, 40), 10.0
    Z, Y, X = np.meshgrid(np.arange(30) * h, np.arange(20) * h, np.arange(40) * h, indexing="ij")
    (az, ay, ax), _ = B.fault_source(shape, h, h, h, FAULT)
    (bz, by, bx), _ = B.fault_source(shape, h, h, h, dict(FAULT, direction=-1))
    # (src+ - p) + (src- - p) = O(theta_shift^2 r)
    th = FAULT["slip"] / FAULT["radius"]
    resid = np.abs(az + bz - 2 * Z) + np.abs(ay + by - 2 * Y) + np.abs(ax + bx - 2 * X)
    assert resid.max() < 4 * th * th * 2000.0
    assert np.abs(az - Z).max() > 10.0


def test_fault_fills_voxels_pulled_from_outside_the_model_depth():
    """A fault through a thin model: where the pull source depth falls outside
    [0, nz) cells the fill value appears, and only there."""
    rng = np.random.default_rng(5)
    V = 2000.0 + rng.uniform(0, 100, (20, 4, 40))
    p = dict(FAULT, cz=10.0, cy=20.0, cx=200.0, slip=150.0, die_r=400.0, die_strike=1000.0, die_theta_deg=60.0)
    (sz, _, _), _ = B.fault_source(V.shape, 10.0, 10.0, 10.0, p)
    out = B.fault(V, 10.0, 10.0, 10.0, p, -1.0)
    outside = (sz / 10.0 < 0) | (sz / 10.0 >= 20)
    assert (sz / 10.0 < 0).any()
    assert np.all(out[outside] == -1.0) and np.all(out[~outside] > 1000.0)


def test_value_noise3d_hits_lattice_values_and_is_periodic():
    rng = np.random.default_rng(7)
    lat = rng.uniform(-1, 1, (3, 4, 5))
    z, y, x = np.meshgrid(np.arange(3) * 20.0, np.arange(4) * 50.0, np.arange(5) * 70.0, indexing="ij")
    assert np.abs(B.value_noise3d(lat, z, y, x, 20.0, 50.0, 70.0) - lat).max() < 1e-12
    p = rng.uniform(0, 500, (3, 40))
    a = B.value_noise3d(lat, p[0], p[1], p[2], 20.0, 50.0, 70.0)
    b = B.value_noise3d(lat, p[0] + 3 * 20.0, p[1] + 4 * 50.0, p[2] + 5 * 70.0, 20.0, 50.0, 70.0)
    assert np.abs(a - b).max() < 1e-9
    assert np.abs(a).max() <= np.abs(lat).max() + 1e-12


def _walk_bed(thick, z):
    """Bed of depth z by walking the beds (thicknesses in cells)."""
    top = 0.0
    for k, h in enumerate(thick):
        if z < top + h or k == len(thick) - 1:
            return k
        top += h


def test_deposit_without_noise_is_beds_plus_trend_under_the_taper():
    """a_B = a_eta = 0: each voxel is the mean velocity plus the depth trend
    plus the taper times its bed's deviation; the bed of a depth found by
    walking the beds; at depth 0 the taper is 0, inside the untapered middle
    it is 1 (the bed velocity itself plus the trend)."""
    rng = np.random.default_rng(8)
    t, ny, nx, dz = 60, 2, 3, 5.0
    thick = np.array([9.0, 12.0, 7.5, 11.0, 10.0, 10.5])
    vbed = rng.normal(2500, 100, 6)
    V = B.deposit(t, ny, nx, dz, 10.0, 10.0, thick, vbed, 0.5, rng.uniform(-1, 1, (5, ny, nx)), 0.0,
                  rng.uniform(-1, 1, (4, 4, 4)), (40.0, 300.0, 300.0), np.zeros(6), 0.0, 0.2, 0.25)
    vbar = vbed.mean()
    assert np.all(V[0] == vbar)
    for z in range(t):
        tau = min(z / (0.2 * t), 1.0) * min((t - z) / (0.25 * t), 1.0)
        ref = vbar + 0.5 * z * dz + tau * (vbed[_walk_bed(thick, z)] - vbar)
        assert np.abs(V[z] - ref).max() < 1e-9, z
    for z in range(12, 45):                      # tau = 1 there
        assert np.abs(V[z] - (vbed[_walk_bed(thick, z)] + 0.5 * z * dz)).max() < 1e-9


def test_deposit_boundary_noise_moves_bed_contacts_within_the_band():
    rng = np.random.default_rng(9)
    t, ny, nx = 50, 3, 4
    thick = np.array([10.0, 10.0, 10.0, 10.0, 10.0])
    vbed = np.array([2000.0, 2400.0, 2800.0, 3200.0, 3600.0])
    eta = np.full((4, ny, nx), 0.5)
    eta[:, 1, 2] = -1.0
    V = B.deposit(t, ny, nx, 5.0, 10.0, 10.0, thick, vbed, 0.0, eta, 4.0,
                  np.zeros((2, 2, 2)), (40.0, 300.0, 300.0), np.zeros(5), 0.0, 1e-9, 1e-9)
    # with the taper 1 below depth 0 a contact moves by a_B * eta = +2 or -4 cells
    # (depth 0 has taper 0: the mean velocity)
    col = V[:, 0, 0]
    assert col[0] == 2800.0
    assert np.all(col[1:12] == 2000.0) and np.all(col[12:22] == 2400.0)
    col = V[:, 1, 2]
    assert np.all(col[1:6] == 2000.0) and np.all(col[6:16] == 2400.0)


def _salt(V, centres, radii, rots, grf, a, vw=0.0, minv=1, h=10.0):
    return B.salt_sdt(V, h, h, h, centres, radii, rots, grf, a, 4500.0, vw, minv)


def test_salt_ellipsoid_volume_and_rotation():
    """No field: the salt is the rasterised ellipsoid (after the cleanup, which
    a large smooth body survives up to a few boundary voxels): its volume
    matches 4/3 pi abc; a rotation that permutes the axes permutes the radii."""
    V = np.full((60, 60, 60), 2500.0)
    zero = np.zeros((1, 60, 60, 60))
    c = (295.0, 305.0, 300.0)
    _, K = _salt(V, [c], [(200.0, 150.0, 120.0)], [np.eye(3)], zero, 0.0)
    assert abs(K.sum() - 4 / 3 * np.pi * 20 * 15 * 12) < 0.03 * K.sum()
    perm = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], np.float64)   # body axis 0 = world y, ...
    _, K1 = _salt(V, [c], [(150.0, 120.0, 200.0)], [perm], zero, 0.0)
    _, K2 = _salt(V, [c], [(200.0, 150.0, 120.0)], [np.eye(3)], zero, 0.0)
    # perm maps world (z, y, x) offsets to body (y, x, z): radii (ry, rx, rz) = (150, 120, 200)
    # along world (y, x, z) are the same ellipsoid as (200, 150, 120) along (z, y, x)
    assert np.array_equal(K1, K2)


def test_salt_constant_field_moves_the_boundary_by_amplitude_times_mean_radius():
    """phi is a signed distance: with grf = 1 everywhere the boundary moves out
    by amplitude * rbar, a sphere of radius R becomes one of R (1 + a)."""
    V = np.full((64, 64, 64), 2500.0)
    R, a = 150.0, 0.3
    _, K = _salt(V, [(315.0, 315.0, 315.0)], [(R, R, R)], [np.eye(3)], np.ones((1, 64, 64, 64)), a)
    vol = 4 / 3 * np.pi * (R * (1 + a) / 10.0) ** 3
    assert abs(K.sum() - vol) < 0.03 * vol
    _, K0 = _salt(V, [(315.0, 315.0, 315.0)], [(R, R, R)], [np.eye(3)], np.zeros((1, 64, 64, 64)), a)
    assert K0.sum() < K.sum() and np.all(K[K0])


def test_salt_water_small_bodies_empty_and_covering_bodies():
    V = np.full((40, 40, 40), 2500.0)
    V[:10] = 1500.0                                     # water layer
    zero = np.zeros((2, 40, 40, 40))
    big, tiny = (120.0, 120.0, 120.0), (25.0, 25.0, 25.0)
    out, K = _salt(V, [(100.0, 200.0, 200.0), (300.0, 80.0, 80.0)], [big, tiny], [np.eye(3)] * 2, zero, 0.0,
                   vw=1600.0, minv=100)
    assert not K[:10].any() and np.all(out[:10] == 1500.0)     # water is never salted
    assert K[10:20, 15:25, 15:25].any()                         # the big body below the water stays
    assert not K[25:35, 5:12, 5:12].any()                       # the tiny one (~65 voxels) is dropped
    assert np.all(out[K] == 4500.0) and np.all(out[~K] == V[~K])
    # a body outside the model changes nothing; one covering it salts everything below the water
    # except the outer one-voxel shell (the closing ends with an erosion, and outside the volume
    # counts as empty)
    o2, K2 = _salt(V, [(5000.0, 5000.0, 5000.0)], [big], [np.eye(3)], zero[:1], 0.0, vw=1600.0)
    assert not K2.any() and np.array_equal(o2, V)
    o3, K3 = _salt(V, [(200.0, 200.0, 200.0)], [(1e5, 1e5, 1e5)], [np.eye(3)], zero[:1], 0.0, vw=1600.0)
    inner = np.zeros(V.shape, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert np.array_equal(K3, inner & (V >= 1600.0))


def test_fault_labels_take_the_voxel_nearest_the_source():
    """Nearest-neighbour pull of integer fields: each moved voxel gets the label
    of the voxel centre nearest its source (brute force over all centres, the
    y and x sources past the volume landing on its faces), fill where the
    source depth leaves the volume, its own label outside the taper."""
    shape, h = (12, 7, 9), 10.0
    L = np.arange(np.prod(shape), dtype=np.int64).reshape(shape)    # every label unique
    p = dict(cz=30.0, cy=30.0, cx=40.0, azimuth_deg=20.0, dip_deg=55.0, radius=300.0, slip=35.0, direction=1,
             die_r=150.0, die_strike=200.0, die_theta_deg=60.0)
    out = B.fault_labels(L, h, h, h, p, -1)
    (sz, sy, sx), w = B.fault_source(shape, h, h, h, p)
    sz, sy, sx = sz / h, sy / h, sx / h
    Z, Y, X = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    moved = fill = 0
    for idx in zip(*np.nonzero(w > 0)):
        s = np.array([sz[idx], sy[idx], sx[idx]])
        if not 0.0 <= s[0] < shape[0]:
            assert out[idx] == -1
            fill += 1
            continue
        d = (Z - s[0]) ** 2 + (Y - s[1]) ** 2 + (X - s[2]) ** 2
        best = np.argmin(d)
        if np.sort(d.ravel())[1] - d.ravel()[best] > 1e-9:      # no tie
            assert out[idx] == L.ravel()[best], idx
            moved += 1
    assert moved > 100 and fill > 0
    assert np.array_equal(out[w == 0], L[w == 0])
    assert np.array_equal(B.fault_labels(L, h, h, h, dict(p, slip=0.0), -1), L)


@pytest.mark.parametrize("c", [0.6, 2.5, -1.8])
def test_rough_fault_surface_moves_the_fault_by_the_noise(c):
    """A rough surface of zero amplitude is the smooth fault; with a constant
    lattice c the noise is exactly c, so the slip changes side exactly where
    the distance from the axis crosses R + amplitude * c (not at R), also for
    a lattice outside [-1, 1] (the paper perturbs the radius by the noise
    itself; nothing bounds it)."""
    shape, h = (40, 6, 50), 10.0
    p = dict(cz=150.0, cy=25.0, cx=250.0, azimuth_deg=0.0, dip_deg=50.0, radius=400.0, slip=30.0, direction=1,
             die_r=200.0, die_strike=500.0, die_theta_deg=80.0)
    lat = np.random.default_rng(3).uniform(-1, 1, (3, 4, 5))
    (s0, w0) = B.fault_source(shape, h, h, h, p)
    (s1, w1) = B.fault_source(shape, h, h, h, dict(p, rough_lattice=lat, rough_amplitude=0.0,
                                                   rough_lam_strike=100.0, rough_lam_dip=80.0))
    assert all(np.array_equal(a, b) for a, b in zip(s0, s1)) and np.array_equal(w0, w1)
    A = 50.0
    rough = dict(p, rough_lattice=np.full((2, 3, 3), c), rough_amplitude=A, rough_lam_strike=100.0,
                 rough_lam_dip=80.0)
    (sz, sy, sx), w = B.fault_source(shape, h, h, h, rough)
    # geometry of the frame, from the fault's definition: axis offset R cos(dip) along n = (0, 1) in (y, x)
    R, dip = p["radius"], math.radians(p["dip_deg"])
    Z, Y, X = np.meshgrid(*[np.arange(n) * h for n in shape], indexing="ij")
    hh, vv = X - (p["cx"] - R * math.cos(dip)), Z - (p["cz"] - R * math.sin(dip))
    r = np.hypot(hh, vv)
    moved = w > 0
    # the displacement's rotation sense: its component along the tangent (-sin t, cos t) in (h, v)
    dh, dv = X - sx, Z - sz          # p - src = (p_fwd - p)
    t = np.arctan2(vv, hh)
    tang = -np.sin(t) * dh + np.cos(t) * dv
    far = r >= R + A * c
    band = moved & (np.abs(tang) > 1e-9)
    assert band.sum() > 200
    # rotation -chi * direction: chi = +1 beyond the surface, -1 inside it
    assert np.all(np.sign(tang[band]) == np.where(far[band], -1.0, 1.0) * p["direction"])
    # voxels between R and R + A c changed side: the smooth fault had them on the other one
    between = band & (r >= min(R, R + A * c)) & (r < max(R, R + A * c))
    assert between.sum() > 20


@pytest.mark.parametrize("o", range(4))
def test_fractal_octave_frequency_and_weight(o):
    """Octave o of the fractal noise runs at frequency 2^o with weight 2^-o of
    the sum sum_k 2^-k: a lattice that is non-zero only in octave o gives
    exactly (2^-o / sum_k 2^-k) times that octave's lattice value at every node
    of the 2^o-refined grid (the fade is 0 there).  A linear frequency ladder
    (o + 1) misses the nodes of octaves 2 and 3; weights growing with o, or
    no normalisation, scale every octave wrongly."""
    rng = np.random.default_rng(20 + o)
    noct, gy, gx = 4, 5, 7
    lat = np.zeros((noct, gy, gx))
    lat[o] = rng.uniform(-1, 1, (gy, gx))
    f = 2.0 ** o
    i = np.arange(-3, 3 * gx + 2)
    j = np.arange(-2, 2 * gy + 3)
    U, Wd = np.meshgrid(i / f, j / f)
    got = B.fractal_value(lat, U, Wd)
    weight = (1.0 / f) / sum(2.0 ** -k for k in range(noct))
    ref = weight * lat[o][np.mod(j, gy)[:, None], np.mod(i, gx)[None, :]]
    assert np.abs(got - ref).max() < 1e-13
    # the octaves add: the sum of one-octave fields is the field of the sum
    full = rng.uniform(-1, 1, (noct, gy, gx))
    u, w = rng.uniform(-5, 20, 300), rng.uniform(-5, 20, 300)
    parts = sum(B.fractal_value(np.where(np.arange(noct)[:, None, None] == k, full, 0.0), u, w) for k in range(noct))
    assert np.abs(B.fractal_value(full, u, w) - parts).max() < 1e-13


def test_fractal_noise_azimuth_rotates_the_lattice():
    """Azimuth 90 deg, one octave, grid spacing = wavelength: the along-azimuth
    coordinate is y and the across coordinate is -x, so the field at node
    (y, x) is the lattice value at row -x, column y (periodic)."""
    rng = np.random.default_rng(24)
    lat = rng.uniform(-1, 1, (1, 6, 6))
    ny, nx = 9, 11
    got = B.fractal_noise2d(lat, ny, nx, 50.0, 50.0, 50.0, 50.0, 90.0, 7.0)
    y, x = np.arange(ny)[:, None], np.arange(nx)[None, :]
    assert np.abs(got - 7.0 * lat[0][np.mod(-x, 6), np.mod(y, 6)]).max() < 1e-12


@pytest.mark.parametrize("which", ["fractal", "value3d"])
def test_noise_is_twice_continuously_differentiable_across_lattice_nodes(which):
    """The fade between lattice nodes has zero first and second derivatives at
    both ends, so the noise is C2 across nodes; midway between two nodes it is
    their mean.  Linear interpolation (a kink) or the cubic smoothstep (a jump
    of the second derivative) fails it."""
    rng = np.random.default_rng(25)
    h = 1e-4
    if which == "fractal":
        lat = rng.uniform(-1, 1, (1, 4, 8))
        f = lambda u: B.fractal_value(lat, u, np.full_like(u, 2.0))
        row = lat[0][2]
    else:
        lat = rng.uniform(-1, 1, (3, 3, 8))
        f = lambda u: B.value_noise3d(lat, np.full_like(u, 10.0), np.full_like(u, 20.0), u * 30.0, 10.0, 20.0, 30.0)
        row = lat[1, 1]
    for node in range(1, 7):
        d2 = []
        for side in (-1, 1):
            x = node + side * 2 * h
            v = f(np.array([x - h, x, x + h]))
            d2.append((v[0] - 2 * v[1] + v[2]) / h ** 2)
        scale = np.abs(np.diff(row)).max()
        assert abs(d2[0] - d2[1]) < 0.05 * scale, (node, d2)
        assert abs(d2[0]) < 0.05 * scale and abs(d2[1]) < 0.05 * scale
        mid = f(np.array([node + 0.5]))[0]
        assert mid == pytest.approx(0.5 * (row[node] + row[node + 1]), abs=1e-13)


def test_deposit_texture_restarts_at_each_bed_start_with_its_offset():
    """Alg. 1's texture term a_eta eta_3D(z - S_l, y, x), with the per-bed
    depth offset into the shared field: with a_B = 0 the bed starts S_l are
    the cumulative thicknesses; with dy, dx equal to the lattice spacing and
    lam_z = 2 dz every sample sits on a lattice node (even z - S_l) or midway
    between two (odd: their mean), so each voxel has a closed form.  Sampling
    at absolute depth (bed starts not multiples of the lattice period), in
    cells instead of metres, or without the offsets fails it."""
    rng = np.random.default_rng(26)
    t, ny, nx, dz, dy, dx = 64, 3, 5, 4.0, 30.0, 25.0
    lam = (2 * dz, dy, dx)
    thick = np.array([7.0, 11.0, 9.0, 13.0, 10.0, 14.0])
    starts = np.concatenate([[0.0], np.cumsum(thick)[:-1]])
    vbed = rng.normal(2600, 120, thick.size)
    gz, gy, gx = 5, 4, 6
    lat = rng.uniform(-1, 1, (gz, gy, gx))
    koff = np.array([0, 3, 1, 4, 2, 7])
    a_eta, beta = 35.0, 0.3
    V = B.deposit(t, ny, nx, dz, dy, dx, thick, vbed, beta, np.zeros((thick.size - 1, ny, nx)), 0.0, lat, lam,
                  koff * lam[0], a_eta, 1e-9, 1e-9)
    vbar = vbed.mean()
    y, x = np.arange(ny)[:, None], np.arange(nx)[None, :]
    for z in range(1, t):
        bed = int(np.searchsorted(starts, z, side="right") - 1)
        q2 = (z - int(starts[bed])) + 2 * koff[bed]          # twice the lattice coordinate
        a = lat[(q2 // 2) % gz][y % gy, x % gx]
        b = lat[(q2 // 2 + 1) % gz][y % gy, x % gx]
        eta = a if q2 % 2 == 0 else 0.5 * (a + b)
        ref = vbar + beta * z * dz + (vbed[bed] - vbar) + a_eta * eta
        assert np.abs(V[z] - ref).max() < 1e-9, z


def test_grf_with_p2_has_the_exponential_covariance_along_each_axis():
    """Alg. 4's spectrum with p = 2 is the Matern spectrum of smoothness 1/2 in
    3D, whose covariance is exp(-|h| / ell) (closed form): the normalised
    field's correlation at lag h along axis k is exp(-h / ell_k), for
    anisotropic correlation lengths.  (Amplitude P instead of sqrt(P) gives
    0.86 at h = ell instead of 0.37; lengths on the wrong axes or a wrong
    frequency order fail the per-axis checks.)  The grid's missing
    wavenumbers past the Nyquist limit and the sampling error leave < 0.05."""
    rng = np.random.default_rng(40)
    n = 128
    ell = (6.0, 9.0, 13.0)
    acc = {k: np.zeros(4) for k in range(3)}
    reps = 3
    for _ in range(reps):
        xi = B.grf(rng.standard_normal((n, n, n)), (n, n, n), ell, 2.0)
        assert abs(xi.mean()) < 1e-12 and abs(xi.std() - 1.0) < 1e-12
        for k in range(3):
            for i, f in enumerate((0.5, 1.0, 1.5, 2.0)):
                h = int(round(f * ell[k]))
                acc[k][i] += np.mean(xi * np.roll(xi, -h, axis=k)) / reps
    for k in range(3):
        for i, f in enumerate((0.5, 1.0, 1.5, 2.0)):
            h = round(f * ell[k])
            assert abs(acc[k][i] - np.exp(-h / ell[k])) < 0.05, (k, h, acc[k][i])


def test_grf_special_cases_and_axis_assignment():
    """ell = 0 makes P = 1: the field is the (cropped, normalised) noise
    itself; transposing the noise's axes with the lengths transposes the
    field; the periodic grid is the next power of two."""
    rng = np.random.default_rng(41)
    assert B.grf_grid(37, 50, 64) == (64, 64, 64) and B.grf_grid(1, 2, 3) == (1, 2, 4)
    shape = (20, 33, 12)
    noise = rng.standard_normal(B.grf_grid(*shape))
    xi = B.grf(noise, shape, (0.0, 0.0, 0.0), 1.7)
    cut = noise[:20, :33, :12]
    assert np.abs(xi - (cut - cut.mean()) / cut.std()).max() < 1e-12
    cube = (32, 32, 32)
    n3 = rng.standard_normal(cube)
    a = B.grf(n3, cube, (2.0, 5.0, 3.0), 1.3)
    b = B.grf(np.transpose(n3, (2, 0, 1)).copy(), cube, (3.0, 2.0, 5.0), 1.3)
    assert np.abs(np.transpose(a, (2, 0, 1)) - b).max() < 1e-10


def test_grf_spectrum_follows_p_of_k_in_every_band():
    """The measured spectrum of the field, |FFT xi|^2 averaged over four
    realisations and over twelve bands of the anisotropic radius
    s = |(k_z l_z, k_y l_y, k_x l_x)|, divided by P(k) = (1 + s^2)^-p, is flat
    (white noise times P): every band within 5 % of the mean.  Wavenumbers in
    cycles instead of radians, the exponent doubled, or the lengths on the
    wrong axes leave bands 10-90 % off."""
    rng = np.random.default_rng(42)
    n, ell, p = 64, (3.0, 5.0, 2.0), 1.5
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    s2 = (kz * ell[0]) ** 2 + (ky * ell[1]) ** 2 + (kx * ell[2]) ** 2
    power = np.zeros_like(s2)
    for _ in range(4):
        power += np.abs(np.fft.fftn(B.grf(rng.standard_normal((n, n, n)), (n, n, n), ell, p))) ** 2
    ratio = power / (1.0 + s2) ** (-p)
    s = np.sqrt(s2)
    edges = np.quantile(s[s2 > 0], np.linspace(0.0, 1.0, 13))
    bands = np.array([ratio[(s > a) & (s <= b)].mean() for a, b in zip(edges[:-1], edges[1:])])
    assert np.abs(bands / bands.mean() - 1.0).max() < 0.05, bands / bands.mean()


# -- 3D simplex noise and the Deposit forms built on it ----------------------

def _corner(i, j, k):
    """Unskewed position of the skewed-lattice corner (i, j, k)."""
    s = (i + j + k) / 6.0
    return np.array([i - s, j - s, k - s], np.float64)


def _simplex_grad_at(perm, c, h=1e-6):
    """Central-difference gradient of the field at point c."""
    g = np.zeros(3)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        g[ax] = (B.simplex_noise3d(perm, *(c + e)) - B.simplex_noise3d(perm, *(c - e))) / (2 * h)
    return g


def test_simplex_noise_vanishes_at_corners_with_a_cube_edge_gradient_there():
    """At every lattice corner the field is 0 (only the corner's own kernel
    reaches it: the nearest other corners are sqrt(3/4) away, beyond the
    radius sqrt(0.6)), and its gradient is 32 * 0.6^4 * g with g one of the
    twelve edge midpoints (|g| = sqrt 2).  A wrong skew or unskew factor
    moves the zeros; a wrong falloff radius, power or scale changes the
    gradient."""
    rng = np.random.default_rng(50)
    perm = rng.permutation(256)
    edges = {tuple(g) for g in ([a, b, 0] for a in (-1, 1) for b in (-1, 1))} | \
            {tuple(g) for g in ([a, 0, b] for a in (-1, 1) for b in (-1, 1))} | \
            {tuple(g) for g in ([0, a, b] for a in (-1, 1) for b in (-1, 1))}
    seen = set()
    for i, j, k in rng.integers(-300, 300, (60, 3)):
        c = _corner(i, j, k)
        assert abs(B.simplex_noise3d(perm, *c)) < 1e-13
        g = _simplex_grad_at(perm, c) / (32.0 * 0.6 ** 4)
        gr = tuple(int(v) for v in np.round(g))
        assert np.abs(g - np.round(g)).max() < 1e-6 and gr in edges, g
        seen.add(gr)
    assert len(seen) >= 8


def test_simplex_noise_is_the_sum_over_the_kuhn_tetrahedron_holding_the_point():
    """Brute force: find, among the six tetrahedra of the skewed unit cube
    {0, e_a, e_a + e_b, 1}, the one whose corners hold the point (barycentric
    coordinates >= 0); take each corner's gradient from the field itself (as
    measured at the corner) and add 32 max(0, 0.6 - |d|^2)^4 g.d over the four
    corners, d the unskewed offset.  Equals the field to 1e-12 on random
    points (a wrong corner order, unskew of the inner corners or corner hash
    fails)."""
    from itertools import permutations
    rng = np.random.default_rng(51)
    perm = rng.permutation(256)
    for p in rng.uniform(-40, 40, (300, 3)):
        u = p + p.sum() / 3.0                        # skewed coordinates
        base = np.floor(u)
        found = None
        for order in permutations(range(3)):
            ks = [base.copy()]
            for ax in order:
                nxt = ks[-1].copy()
                nxt[ax] += 1
                ks.append(nxt)
            C = np.array([_corner(*kk) for kk in ks])
            M = np.vstack([(C[1:] - C[0]).T])
            lam = np.linalg.solve(M, p - C[0])
            if lam.min() >= -1e-12 and lam.sum() <= 1 + 1e-12:
                found = C
                break
        assert found is not None
        ref = 0.0
        for c in found:
            d = p - c
            w = 0.6 - d @ d
            if w > 0:
                ref += 32.0 * w ** 4 * (np.round(_simplex_grad_at(perm, c) / (32.0 * 0.6 ** 4)) @ d)
        assert abs(B.simplex_noise3d(perm, *p) - ref) < 1e-12, (p, ref)


def test_simplex_noise_periodicity_range_and_permutation_dependence():
    """Shifting the skewed lattice by 256 cells along any axis leaves the
    field unchanged (indices mod 256); values stay within [-1, 1] with mean
    about 0; another permutation gives another field."""
    rng = np.random.default_rng(52)
    perm = rng.permutation(256)
    pts = rng.uniform(-30, 30, (3, 2000))
    v = B.simplex_noise3d(perm, *pts)
    for ax in range(3):
        sh = np.array([256.0 * (a == ax) for a in range(3)]) - 256.0 / 6.0
        w = B.simplex_noise3d(perm, *(pts + sh[:, None]))
        assert np.abs(w - v).max() < 1e-9
    big = B.simplex_noise3d(perm, *rng.uniform(-100, 100, (3, 200000)))
    assert np.abs(big).max() <= 1.0 and abs(big.mean()) < 0.01 and 0.3 < big.std() < 0.5
    assert np.abs(B.simplex_noise3d(rng.permutation(256), *pts) - v).max() > 0.3


def test_deposit_simplex_equals_the_boundary_path_with_plane_samples():
    """deposit_simplex is Alg. 1's boundary path with eta_b the 3D simplex
    field sampled on each boundary's own depth plane: with the texture off
    it equals `deposit` given those plane samples; with both amplitudes 0
    it is the plain bed model."""
    rng = np.random.default_rng(53)
    t, ny, nx, dz, dy, dx = 70, 5, 6, 4.0, 12.0, 9.0
    thick = np.array([8.0, 11.0, 7.0, 12.0, 9.5, 10.0, 12.5])
    vbed = rng.normal(2600, 150, 7)
    pb, pt = rng.permutation(256), rng.permutation(256)
    lam_b, lam_t = (60.0, 250.0, 180.0), (20.0, 90.0, 70.0)
    H = np.cumsum(thick)[:-1]
    Z = np.broadcast_to((H * dz / lam_b[0])[:, None, None], (6, ny, nx))
    Y = np.broadcast_to((np.arange(ny) * dy / lam_b[1])[None, :, None], (6, ny, nx))
    X = np.broadcast_to((np.arange(nx) * dx / lam_b[2])[None, None, :], (6, ny, nx))
    eta_b = B.simplex_noise3d(pb, Z, Y, X)
    off = rng.uniform(0, 500, 7)
    a = B.deposit_simplex(t, ny, nx, dz, dy, dx, thick, vbed, 0.4, pb, lam_b, 3.0, pt, lam_t, off, 0.0, 0.2, 0.2)
    b = B.deposit(t, ny, nx, dz, dy, dx, thick, vbed, 0.4, eta_b, 3.0, np.zeros((2, 2, 2)), lam_t, off, 0.0,
                  0.2, 0.2)
    assert np.abs(a - b).max() < 1e-9
    c = B.deposit_simplex(t, ny, nx, dz, dy, dx, thick, vbed, 0.4, pb, lam_b, 0.0, pt, lam_t, off, 0.0, 0.2, 0.2)
    d = B.deposit(t, ny, nx, dz, dy, dx, thick, vbed, 0.4, np.zeros((6, ny, nx)), 0.0, np.zeros((2, 2, 2)),
                  lam_t, off, 0.0, 0.2, 0.2)
    assert np.abs(c - d).max() < 1e-9


def test_deposit_simplex_texture_restarts_at_each_bed_start():
    """With flat contacts (a_B = 0) and two beds given the same offset, the
    texture at k cells below the first bed's start equals the texture k
    cells below the second's (sampling at absolute depth fails), and at a
    bed start it is the field at (offset / lam_z, y dy / lam_y, x dx / lam_x)."""
    rng = np.random.default_rng(54)
    t, ny, nx, dz, dy, dx = 60, 4, 5, 5.0, 10.0, 10.0
    thick = np.array([10.0, 20.0, 20.0, 10.0])
    vbed = np.array([2500.0, 2500.0, 2500.0, 2500.0])
    pt = rng.permutation(256)
    lam_t = (35.0, 80.0, 60.0)
    off = np.array([0.0, 123.0, 123.0, 40.0])
    V = B.deposit_simplex(t, ny, nx, dz, dy, dx, thick, vbed, 0.0, pt, (1.0, 1.0, 1.0), 0.0, pt, lam_t, off, 50.0,
                          1e-9, 1e-9)
    tex = V - 2500.0                     # taper 1 below row 0, no trend, equal beds
    assert np.abs(tex[10:30] - tex[30:50]).max() < 1e-9
    assert np.abs(tex[10] - tex[25]).max() > 1.0
    Y = np.broadcast_to((np.arange(ny) * dy / lam_t[1])[:, None], (ny, nx))
    X = np.broadcast_to((np.arange(nx) * dx / lam_t[2])[None, :], (ny, nx))
    ref = 50.0 * B.simplex_noise3d(pt, np.full((ny, nx), 123.0 / lam_t[0]), Y, X)
    assert np.abs(tex[10] - ref).max() < 1e-9


def test_warped_axis_sums_the_gaussian_smoothed_frequency():
    """W[z] = sum of the smoothed frequency above z: sigma 0 gives the plain
    prefix sum (a linear ramp gives the quadratic closed form); a constant
    frequency is kept by the smoothing; a unit spike becomes the sampled
    Gaussian exp(-m^2 / 2 sigma^2), normalised over |m| <= 4 sigma."""
    t = 40
    f = 0.05 + 0.002 * np.arange(t)
    W = B.warped_axis(f, 0.0)
    z = np.arange(t)
    assert np.abs(W - (0.05 * z + 0.002 * z * (z - 1) / 2)).max() < 1e-12
    assert np.abs(B.warped_axis(np.full(t, 0.1), 2.5) - 0.1 * z).max() < 1e-12
    spike = np.zeros(t)
    spike[20] = 1.0
    sm = np.diff(B.warped_axis(spike, 2.0))          # smoothed values f[0..t-2]
    m = np.arange(-8, 9)
    g = np.exp(-m ** 2 / 8.0)
    assert np.abs(sm[12:29] - g / g.sum()).max() < 1e-12


def test_deposit_sinusoidal_closed_forms():
    """Constant frequency f, no smoothing effect, no texture, taper 1: V is
    v0 + beta z dz + amp1 sin(2 pi f z) + amp2 sin(4 pi f z + phase2); a
    constant roughness c shifts the phase by 2 pi a_r c; the texture term
    is a_eta times the simplex field at (z dz, y dy, x dx) / lam."""
    rng = np.random.default_rng(55)
    t, ny, nx, dz = 50, 3, 4, 2.0
    f = 0.07
    args = dict(v0=3000.0, beta=0.2, sigma=1.5, amp1=120.0, amp2=45.0, phase2=0.7)
    pt = rng.permutation(256)
    lam = (30.0, 70.0, 50.0)

    def run(rug, a_r, a_eta):
        return B.deposit_sinusoidal(t, ny, nx, dz, 10.0, 10.0, args["v0"], args["beta"], np.full(t, f),
                                    args["sigma"], args["amp1"], args["amp2"], args["phase2"], rug, a_r, pt, lam,
                                    a_eta, 1e-9, 1e-9)
    z = np.arange(t)[:, None, None] * 1.0
    V = run(np.zeros((ny, nx)), 0.0, 0.0)
    ref = 3000.0 + 0.2 * z * dz + 120.0 * np.sin(2 * np.pi * f * z) + 45.0 * np.sin(4 * np.pi * f * z + 0.7)
    assert np.abs(V[1:] - ref[1:]).max() < 1e-9
    c = 0.3
    V2 = run(np.full((ny, nx), c), 0.5, 0.0)
    ph = 2 * np.pi * (f * z + 0.5 * c)
    ref2 = 3000.0 + 0.2 * z * dz + 120.0 * np.sin(ph) + 45.0 * np.sin(2 * ph + 0.7)
    assert np.abs(V2[1:] - ref2[1:]).max() < 1e-9
    V3 = run(np.zeros((ny, nx)), 0.0, 25.0)
    Z, Y, X = np.meshgrid(np.arange(t) * dz / lam[0], np.arange(ny) * 10.0 / lam[1], np.arange(nx) * 10.0 / lam[2],
                          indexing="ij")
    assert np.abs((V3 - V)[1:] - 25.0 * B.simplex_noise3d(pt, Z, Y, X)[1:]).max() < 1e-9


# -- subsidiary faults (Riedel-shear geometry) --------------------------------

PRIMARY = dict(cz=1200.0, cy=2500.0, cx=3000.0, azimuth_deg=25.0, dip_deg=60.0, radius=3000.0, slip=120.0,
               direction=1, die_r=400.0, die_strike=2000.0, die_theta_deg=30.0)
RIEDEL = dict(B.RIEDEL_DEFAULTS, along_strike=1500.0, across_min=100.0, across_max=700.0, size_scale=0.3,
              slip_min=0.2, slip_max=0.5, min_distance=0.0)


def _strike(az_deg):
    a = math.radians(az_deg)
    return np.array([math.cos(a), -math.sin(a)])


def test_riedel_orientations_sides_and_draw_fractions():
    """20000 candidates without the distance filter: every subsidiary's
    strike makes 15 deg (synthetic) or 165 deg (antithetic) with the
    primary's; the synthetic share is 0.85 and the hanging-wall share 0.75
    (+-0.01); hanging-wall centres lie on the concave side of the primary's
    listric surface (inside its cylinder, r < R, measured from the axis the
    primary's dip and radius put at c - (R cos dip) n - (R sin dip) z), the
    footwall ones outside, all across-strike distances in [100, 700] m and
    along-strike offsets within +-1500 m; sizes and slips scaled as drawn."""
    rng = np.random.default_rng(60)
    u = rng.random((20000, 5))
    subs = B.riedel_subsidiaries(PRIMARY, RIEDEL, u)
    assert len(subs) == 20000
    s0 = _strike(PRIMARY["azimuth_deg"])
    n0 = np.array([s0[1] * -1.0, s0[0]])            # rotate strike by +90 deg: (sin a, cos a)
    ang = np.array([math.degrees(math.acos(np.clip(_strike(q["azimuth_deg"]) @ s0, -1, 1))) for q in subs])
    assert np.all((np.abs(ang - 15.0) < 1e-9) | (np.abs(ang - 165.0) < 1e-9))
    assert abs(np.mean(ang < 90) - 0.85) < 0.01
    a, dip, R = math.radians(PRIMARY["azimuth_deg"]), math.radians(PRIMARY["dip_deg"]), PRIMARY["radius"]
    axis_yx = np.array([PRIMARY["cy"], PRIMARY["cx"]]) - R * math.cos(dip) * n0
    axis_z = PRIMARY["cz"] - R * math.sin(dip)
    hang = []
    for q in subs:
        d = np.array([q["cy"], q["cx"]]) - np.array([PRIMARY["cy"], PRIMARY["cx"]])
        across, along = d @ n0, d @ s0
        assert 100.0 - 1e-9 <= abs(across) <= 700.0 + 1e-9 and abs(along) <= 1500.0 + 1e-9
        assert q["cz"] == PRIMARY["cz"]
        r = math.hypot((np.array([q["cy"], q["cx"]]) - axis_yx) @ n0, q["cz"] - axis_z)
        hang.append(r < R)
        assert (r < R) == (across < 0)
        assert q["radius"] == pytest.approx(0.3 * R) and q["die_r"] == pytest.approx(120.0)
        assert 0.2 * 120.0 - 1e-9 <= q["slip"] <= 0.5 * 120.0 + 1e-9
        assert q["dip_deg"] == 60.0 and q["direction"] == 1 and q["rough_lattice"] is None
    assert abs(np.mean(hang) - 0.75) < 0.01


def test_riedel_distance_filter_is_greedy_and_keeps_spacing():
    """With min_distance 250 m: accepted centres are pairwise >= 250 m apart
    (horizontally), every rejected candidate lies within 250 m of one
    accepted before it, and the accepted ones are the unfiltered run's in
    order (the filter drops, never alters)."""
    rng = np.random.default_rng(61)
    u = rng.random((60, 5))
    cfg = dict(RIEDEL, min_distance=250.0)
    kept = B.riedel_subsidiaries(PRIMARY, cfg, u)
    allc = B.riedel_subsidiaries(PRIMARY, RIEDEL, u)
    assert 5 < len(kept) < 60
    xy = lambda q: np.array([q["cy"], q["cx"]])
    for i in range(len(kept)):
        for j in range(i):
            assert np.linalg.norm(xy(kept[i]) - xy(kept[j])) >= 250.0
    it = iter(kept)
    nxt = next(it)
    accepted = []
    for q in allc:
        if nxt is not None and q == nxt:
            accepted.append(q)
            nxt = next(it, None)
        else:
            assert min(np.linalg.norm(xy(q) - xy(p)) for p in accepted) < 250.0
    assert nxt is None


def test_fault_sequence_applies_the_faults_in_order():
    """The sequence equals the faults applied one by one; a fault of zero
    slip leaves the model, and the order matters for overlapping faults."""
    rng = np.random.default_rng(62)
    V = 2000.0 + 30.0 * np.arange(24)[:, None, None] + rng.normal(0, 5, (24, 10, 12))
    p1 = dict(PRIMARY, cz=100.0, cy=50.0, cx=60.0, radius=300.0, slip=30.0, die_r=60.0, die_strike=200.0)
    p2 = dict(p1, azimuth_deg=40.0, cx=70.0, slip=25.0)
    seq = B.fault_sequence(V, 10.0, 10.0, 10.0, [p1, p2], 1500.0)
    one = B.fault(B.fault(V, 10.0, 10.0, 10.0, p1, 1500.0), 10.0, 10.0, 10.0, p2, 1500.0)
    assert np.abs(seq - one).max() == 0.0
    rev = B.fault_sequence(V, 10.0, 10.0, 10.0, [p2, p1], 1500.0)
    assert np.abs(seq - rev).max() > 1.0
    still = B.fault_sequence(V, 10.0, 10.0, 10.0, [dict(p1, slip=0.0)], 1500.0)
    assert np.abs(still - V).max() < 1e-9
