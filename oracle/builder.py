"""FP64 reference of the velocity-model builder modules of SubsurfaceGen
(arXiv 2605.30541, App. B): Deposit (Alg. 1, interbedded band; its simplex
noise fields and sinusoidal bedform mode from the module's prose), Squish
(Alg. 2, vertical warping by a fractal-noise displacement), Fault (Alg. 3, one
listric normal fault as a tapered rotation about a horizontal cylinder; sinc
pull for velocities, nearest-neighbour pull for labels; subsidiary faults in
Riedel-shear geometry) and SaltSDT (Alg. 4,
salt bodies from perturbed signed distances).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it; it shares no code with the HIP library.

Volumes are [nz][ny][nx] (x fastest), z is depth (down), positions in metres
are (z*dz, y*dy, x*dx).  Readings where the paper leaves the details open:

* sinc: 8-point Kaiser-windowed sinc, w(t) = sinc(t) I0(6 sqrt(1 - (t/4)^2)) /
  I0(6) on the taps floor(s)-3 .. floor(s)+4, weights divided by their sum;
  tap indices outside the axis are clamped to it (edge replication).  At
  integer s the weights are a unit impulse, so the sample is exact.  A 3D
  sample is the separable product of the three axes' weights.  (Among the
  usual 8-point windows this one keeps the error on band-limited signals
  below 1e-3 from 4 to 64 samples per period.)
* fractal noise (Alg. 2): smooth value noise on a periodic lattice per octave
  (values given, e.g. uniform in [-1, 1]), quintic fade between lattice
  nodes; horizontal coordinates rotated by the azimuth and scaled by the
  wavelengths; octave o has frequency 2^o and weight 2^-o; the sum is divided
  by sum_o 2^-o and scaled by the maximum shift, so |dz| <= dz_max.
* fault frame (Alg. 3): the horizontal unit vector n = (sin a, cos a) in
  (y, x) is the offset direction of the cylinder axis from the centre (the
  dip direction), s = (cos a, -sin a) the strike along the axis; in the plane
  across strike h = (p - c~).n and v = depth - c~_z give r = |(h, v)| and
  theta = atan2(v, h); the along-strike offset is (p - c~).s.  Angles in
  radians internally; the die-off angle is given in degrees.
"""
from __future__ import annotations

import math

import numpy as np

HALF = 4          # taps on each side of the sample position
BETA = 6.0        # Kaiser window shape


def _sinc(u):
    u = np.asarray(u, np.float64)
    out = np.ones_like(u)
    nz = u != 0.0
    out[nz] = np.sin(np.pi * u[nz]) / (np.pi * u[nz])
    return out


def sinc_taps(s, n: int):
    """Tap indices [..., 8] (clamped to 0..n-1) and normalised Kaiser-sinc
    weights [..., 8] for sample positions s (in cells) on an axis of n."""
    s = np.asarray(s, np.float64)
    base = np.floor(s)
    j = base[..., None] + np.arange(-HALF + 1, HALF + 1)
    t = s[..., None] - j
    w = _sinc(t) * np.i0(BETA * np.sqrt(np.clip(1.0 - (t / HALF) ** 2, 0.0, 1.0))) / np.i0(BETA)
    w = w / w.sum(axis=-1, keepdims=True)
    return np.clip(j, 0, n - 1).astype(np.int64), w


def sinc_sample_3d(V, sz, sy, sx):
    """V sampled at the positions (sz, sy, sx) (cells, arrays of one shape)."""
    V = np.asarray(V, np.float64)
    nz, ny, nx = V.shape
    jz, wz = sinc_taps(sz, nz)
    jy, wy = sinc_taps(sy, ny)
    jx, wx = sinc_taps(sx, nx)
    out = np.zeros(np.shape(sz))
    for a in range(2 * HALF):
        for b in range(2 * HALF):
            wab = wz[..., a] * wy[..., b]
            for c in range(2 * HALF):
                out += wab * wx[..., c] * V[jz[..., a], jy[..., b], jx[..., c]]
    return out


def fractal_noise2d(lattice, ny: int, nx: int, dy: float, dx: float, lam_y: float, lam_x: float,
                    azimuth_deg: float, amplitude: float):
    """Alg. 2, first step: the displacement field dz(y, x) [ny, nx] in metres
    from per-octave lattices [noct, gy, gx] (periodic)."""
    lattice = np.asarray(lattice, np.float64)
    noct, gy, gx = lattice.shape
    a = math.radians(azimuth_deg)
    Y = np.arange(ny)[:, None] * dy
    X = np.arange(nx)[None, :] * dx
    u = (X * math.cos(a) + Y * math.sin(a)) / lam_x      # along the azimuth
    w = (-X * math.sin(a) + Y * math.cos(a)) / lam_y     # across it
    return amplitude * fractal_value(lattice, u, w)


def fractal_value(lattice, u, w):
    """Normalised fractal value noise at lattice coordinates (u, w) (arrays of
    one shape; u runs along the lattice's columns): per octave o a periodic
    lattice [gy, gx] sampled with a quintic fade at (u, w) * 2^o, weight 2^-o;
    the sum divided by sum_o 2^-o, so the result lies within the lattice's range."""
    lattice = np.asarray(lattice, np.float64)
    noct, gy, gx = lattice.shape
    u, w = np.asarray(u, np.float64), np.asarray(w, np.float64)
    fade = lambda t: t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    total = np.zeros(np.broadcast(u, w).shape)
    norm = 0.0
    for o in range(noct):
        f = 2.0 ** o
        pu, pw = u * f, w * f
        iu, iw = np.floor(pu), np.floor(pw)
        tu, tw = fade(pu - iu), fade(pw - iw)
        iu, iw = iu.astype(np.int64), iw.astype(np.int64)
        L = lattice[o]
        v00 = L[iw % gy, iu % gx]
        v01 = L[iw % gy, (iu + 1) % gx]
        v10 = L[(iw + 1) % gy, iu % gx]
        v11 = L[(iw + 1) % gy, (iu + 1) % gx]
        n = (v00 * (1 - tu) + v01 * tu) * (1 - tw) + (v10 * (1 - tu) + v11 * tu) * tw
        total += n / f
        norm += 1.0 / f
    return total / norm


def squish(V, dz: float, shift):
    """Alg. 2, second step: V pulled from (z + shift(y, x), y, x); shift in
    metres, [ny, nx]."""
    V = np.asarray(V, np.float64)
    nz, ny, nx = V.shape
    sz = np.arange(nz)[:, None, None] + np.asarray(shift, np.float64)[None] / dz
    sy = np.broadcast_to(np.arange(ny)[None, :, None], sz.shape).astype(np.float64)
    sx = np.broadcast_to(np.arange(nx)[None, None, :], sz.shape).astype(np.float64)
    return sinc_sample_3d(V, sz, sy, sx)


def fault_source(shape, dz: float, dy: float, dx: float, p: dict):
    """Alg. 3: for every voxel, the pull source (metres, three arrays z, y, x)
    and the taper w.  p holds cz, cy, cx [m], azimuth_deg, dip_deg, radius,
    slip, direction (+1/-1), die_r, die_strike [m], die_theta_deg, and
    optionally a rough surface: rough_lattice [noct, gd, gs] (rows down dip,
    columns along strike; None = smooth),
    rough_amplitude, rough_lam_strike, rough_lam_dip [m].  A rough surface
    has radius R + rough_amplitude * N(u, w), N the normalised fractal value
    noise (fractal_value; it lies within the lattice's range) at
    u = along-strike offset / rough_lam_strike and
    w = R (theta - theta0) / rough_lam_dip (the down-dip arc length); it
    moves where the fault is (the side test and the across-fault taper) and
    leaves the rotation angle slip / R as it is."""
    nz, ny, nx = shape
    a, th, R = math.radians(p["azimuth_deg"]), math.radians(p["dip_deg"]), p["radius"]
    ny_, nx_ = math.sin(a), math.cos(a)            # n: offset direction of the axis
    sy_, sx_ = math.cos(a), -math.sin(a)           # s: strike
    dlt_z, dlt_az = R * math.sin(th), R * math.cos(th)
    cz = p["cz"] - dlt_z
    cy = p["cy"] - dlt_az * ny_
    cx = p["cx"] - dlt_az * nx_
    theta0 = math.atan2(dlt_z, dlt_az)
    shift = p["slip"] / (2.0 * math.pi * R) * 2.0 * math.pi  # 360 deg per circumference, in radians
    Z = np.arange(nz)[:, None, None] * dz
    Y = np.arange(ny)[None, :, None] * dy
    X = np.arange(nx)[None, None, :] * dx
    Z, Y, X = np.broadcast_arrays(Z, Y, X)
    qy, qx, v = Y - cy, X - cx, Z - cz
    h = qy * ny_ + qx * nx_
    az = qy * sy_ + qx * sx_
    r = np.hypot(h, v)
    t_old = np.arctan2(v, h)
    Rs = R
    if p.get("rough_lattice") is not None:
        N = fractal_value(p["rough_lattice"], az / p["rough_lam_strike"], R * (t_old - theta0) / p["rough_lam_dip"])
        Rs = R + p["rough_amplitude"] * N
    rho_r = np.abs(r - Rs) / p["die_r"]
    rho_t = np.abs(t_old - theta0) / math.radians(p["die_theta_deg"])
    rho_s = np.abs(az) / p["die_strike"]
    inside = (rho_r < 1) & (rho_t < 1) & (rho_s < 1)
    wt = np.where(inside, np.cos(0.5 * np.pi * rho_r) * np.cos(0.5 * np.pi * rho_t) * np.cos(0.5 * np.pi * rho_s), 0.0)
    chi = np.where(r >= Rs, 1.0, -1.0)
    dth = -chi * p["direction"] * wt * shift       # theta_new - theta_old
    # p_fwd - p = r (cos t_new - cos t_old, sin t_new - sin t_old) in the (h, v)
    # plane, the along-strike offset unchanged; written with half-angle
    # products it is exactly 0 where the rotation is 0 (src = 2p - p_fwd = p)
    mid, half = t_old + 0.5 * dth, np.sin(0.5 * dth)
    dh = -2.0 * r * np.sin(mid) * half
    dv = 2.0 * r * np.cos(mid) * half
    return (Z - dv, Y - dh * ny_, X - dh * nx_), wt


def fault(V, dz: float, dy: float, dx: float, p: dict, fill: float):
    """Alg. 3: V pulled from the sources of fault_source; voxels whose source
    depth falls outside [0, nz) cells get `fill`."""
    V = np.asarray(V, np.float64)
    (sz, sy, sx), _ = fault_source(V.shape, dz, dy, dx, p)
    sz, sy, sx = sz / dz, sy / dy, sx / dx
    out = sinc_sample_3d(V, sz, sy, sx)
    out[(sz < 0) | (sz >= V.shape[0])] = fill
    return out


def fault_labels(L, dz: float, dy: float, dx: float, p: dict, fill: int):
    """Alg. 3 for integer fields (layer labels), which the module resamples by
    nearest neighbour: the voxel nearest each pull source of fault_source
    (floor(s + 0.5) cells per axis, y and x clamped to the volume); `fill`
    where the source depth falls outside [0, nz) cells; voxels outside the
    taper keep their label."""
    L = np.asarray(L)
    nz, ny, nx = L.shape
    (sz, sy, sx), w = fault_source(L.shape, dz, dy, dx, p)
    sz, sy, sx = sz / dz, sy / dy, sx / dx
    iz = np.minimum(np.floor(np.where((sz >= 0) & (sz < nz), sz, 0.0) + 0.5), nz - 1).astype(np.int64)
    iy = np.clip(np.floor(sy + 0.5), 0, ny - 1).astype(np.int64)
    ix = np.clip(np.floor(sx + 0.5), 0, nx - 1).astype(np.int64)
    out = L[iz, iy, ix]
    out = np.where(w == 0, L, out)
    out[(w != 0) & ((sz < 0) | (sz >= nz))] = fill
    return out


RIEDEL_DEFAULTS = dict(synthetic_fraction=0.85, hangingwall_fraction=0.75, synthetic_offset_deg=15.0,
                       antithetic_offset_deg=165.0)


def riedel_subsidiaries(primary: dict, cfg: dict, uniforms):
    """Subsidiary faults of a primary in simplified Riedel-shear geometry (the
    Fault prose of App. B and the fault-array setting of App. C): candidate k
    draws five uniforms u in [0, 1) (the random draw, an input [n, 5]) and is

      * synthetic (an R-shear, strike turned by synthetic_offset_deg) when
        u0 < synthetic_fraction, else antithetic (R', antithetic_offset_deg);
      * in the hanging wall when u1 < hangingwall_fraction, else in the
        footwall: the hanging wall is the side of the primary's trace towards
        which it dips, -n with n = (sin a, cos a) in (y, x) the direction from
        the primary's cylinder axis to its centre;
      * centred at the primary's depth and at c_yx + along s + side across n
        with along = (2 u2 - 1) along_strike, across = across_min + u3
        (across_max - across_min), s = (cos a, -sin a) the primary's strike;
      * a copy of the primary scaled by size_scale in radius, die_r and
        die_strike, with slip = primary slip (slip_min + u4 (slip_max -
        slip_min)), a smooth surface, the same dip, die-off angle and direction.

    Candidates are taken in order; one whose centre lies closer than
    min_distance (horizontally) to an accepted subsidiary's is rejected.
    Returns the accepted subsidiaries (dicts like `primary`)."""
    u = np.asarray(uniforms, np.float64).reshape(-1, 5)
    a = math.radians(primary["azimuth_deg"])
    n_y, n_x = math.sin(a), math.cos(a)
    s_y, s_x = math.cos(a), -math.sin(a)
    out = []
    for k in range(u.shape[0]):
        u0, u1, u2, u3, u4 = u[k]
        synthetic = u0 < cfg["synthetic_fraction"]
        side = -1.0 if u1 < cfg["hangingwall_fraction"] else 1.0
        along = (2.0 * u2 - 1.0) * cfg["along_strike"]
        across = cfg["across_min"] + u3 * (cfg["across_max"] - cfg["across_min"])
        cy = primary["cy"] + along * s_y + side * across * n_y
        cx = primary["cx"] + along * s_x + side * across * n_x
        if cfg["min_distance"] > 0 and any(math.hypot(cy - q["cy"], cx - q["cx"]) < cfg["min_distance"]
                                           for q in out):
            continue
        sub = dict(primary)
        sub.update(cy=cy, cx=cx,
                   azimuth_deg=primary["azimuth_deg"] + (cfg["synthetic_offset_deg"] if synthetic
                                                         else cfg["antithetic_offset_deg"]),
                   radius=primary["radius"] * cfg["size_scale"], die_r=primary["die_r"] * cfg["size_scale"],
                   die_strike=primary["die_strike"] * cfg["size_scale"],
                   slip=primary["slip"] * (cfg["slip_min"] + u4 * (cfg["slip_max"] - cfg["slip_min"])),
                   rough_lattice=None)
        out.append(sub)
    return out


def fault_sequence(V, dz: float, dy: float, dx: float, faults, fill: float):
    """The faults applied one after another (a primary and its subsidiaries)."""
    V = np.asarray(V, np.float64)
    for p in faults:
        V = fault(V, dz, dy, dx, p, fill)
    return V


def fault_labels_sequence(L, dz: float, dy: float, dx: float, faults, fill: int):
    """Labels through the same faults one after another."""
    for p in faults:
        L = fault_labels(L, dz, dy, dx, p, fill)
    return L


def value_noise3d(lattice, z, y, x, lam_z: float, lam_y: float, lam_x: float):
    """Smooth value noise in [-1, 1] (lattice values in [-1, 1]) at points
    (z, y, x) in metres: periodic lattice [gz, gy, gx], node spacing
    (lam_z, lam_y, lam_x), quintic fade between nodes (the texture field of
    Alg. 1; one octave)."""
    lattice = np.asarray(lattice, np.float64)
    gz, gy, gx = lattice.shape
    fade = lambda t: t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    pz, py, px = np.asarray(z) / lam_z, np.asarray(y) / lam_y, np.asarray(x) / lam_x
    iz, iy, ix = np.floor(pz), np.floor(py), np.floor(px)
    tz, ty, tx = fade(pz - iz), fade(py - iy), fade(px - ix)
    iz, iy, ix = iz.astype(np.int64), iy.astype(np.int64), ix.astype(np.int64)
    out = 0.0
    for a in (0, 1):
        wz = tz if a else 1 - tz
        for b in (0, 1):
            wy = ty if b else 1 - ty
            for c in (0, 1):
                wx = tx if c else 1 - tx
                out = out + wz * wy * wx * lattice[(iz + a) % gz, (iy + b) % gy, (ix + c) % gx]
    return out


def deposit(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, thick, vbed, beta: float,
            eta_b, a_B: float, tex_lattice, lam, tex_off, a_eta: float, f_top: float, f_base: float):
    """Alg. 1 (interbedded package, boundary path) on a band of t cells:
    thick [n] bed thicknesses in cells (the drawn, clamped values), vbed [n]
    bed velocities, beta the velocity gradient [m/s per m], eta_b [n-1, ny, nx]
    boundary noise, a_B its amplitude [cells], tex_lattice / lam / tex_off [n]
    (metres) the texture noise and per-bed depth offsets, a_eta its amplitude
    [m/s], f_top / f_base the taper fractions.  Returns V [t, ny, nx].

    Readings: the internal boundaries are the cumulative thicknesses
    H_i = sum_{k < i} thick_k, i = 1..n-1; a voxel at depth z (cells) belongs
    to bed l = #{i : H_i(y, x) <= z}, whose start S_l is the largest perturbed
    boundary <= z (0 for bed 0); the texture is sampled at depth
    (z - S_l) dz + tex_off_l."""
    thick = np.asarray(thick, np.float64)
    vbed = np.asarray(vbed, np.float64)
    n = thick.size
    H = np.cumsum(thick)[:-1]                          # n - 1 internal boundaries
    vbar = vbed.mean()

    def tau(z):
        z = np.asarray(z, np.float64)
        return np.minimum(z / (f_top * t), 1.0) * np.minimum((t - z) / (f_base * t), 1.0)

    Hyx = np.clip(H[:, None, None] + tau(H)[:, None, None] * a_B * np.asarray(eta_b, np.float64), 0.0, t - 1.0)
    z = np.arange(t, dtype=np.float64)[:, None, None]
    le = Hyx[None, :, :, :] <= z[:, None, :, :]         # [t, n-1, ny, nx]
    bed = le.sum(axis=1)                               # [t, ny, nx]
    start = np.where(le, Hyx[None], 0.0).max(axis=1, initial=0.0)   # largest boundary <= z (0 if none)
    Y = (np.arange(ny) * dy)[None, :, None]
    X = (np.arange(nx) * dx)[None, None, :]
    zt = (z - start) * dz + np.asarray(tex_off, np.float64)[bed]
    eta = value_noise3d(tex_lattice, zt, np.broadcast_to(Y, zt.shape), np.broadcast_to(X, zt.shape), *lam)
    return (vbar + beta * z * dz) + tau(z) * ((vbed[bed] - vbar) + a_eta * eta)


# The twelve gradients of 3D simplex noise: the midpoints of the cube's edges.
SIMPLEX_GRADS = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1], [1, 0, -1],
                          [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], np.float64)


def simplex_noise3d(perm, a, b, c):
    """3D simplex noise (Perlin's simplex noise in the formulation published
    by Gustavson, "Simplex noise demystified", 2005) at lattice coordinates
    (a, b, c) (arrays of one shape; this library passes (z, y, x) divided by
    the wavelengths).  perm is a permutation of 0..255 (the random draw).

    The point is skewed by F3 = 1/3 onto the cubic lattice, whose cells split
    into six tetrahedra; the corners of the tetrahedron holding the point
    each add (0.6 - |d|^2)^4 (g . d) where positive, d the unskewed offset
    from the corner (G3 = 1/6) and g one of the twelve edge-midpoint
    gradients, chosen by the corner's hash perm[i + perm[j + perm[k]]] mod 12
    (indices mod 256); the sum is scaled by 32 (values in about [-1, 1]).
    The field is 0 at every lattice corner and periodic with 256 lattice
    cells on each skewed axis."""
    P = np.asarray(perm, np.int64)
    pts = [np.asarray(v, np.float64) for v in (a, b, c)]
    s = (pts[0] + pts[1] + pts[2]) / 3.0
    ijk = [np.floor(v + s) for v in pts]
    t = (ijk[0] + ijk[1] + ijk[2]) / 6.0
    d0 = [v - (i - t) for v, i in zip(pts, ijk)]
    # rank the offsets: the tetrahedron's corners step one axis at a time,
    # largest offset first (ties: the lower axis first)
    ge01, ge02, ge12 = d0[0] >= d0[1], d0[0] >= d0[2], d0[1] >= d0[2]
    first = [ge01 & ge02, ~ge01 & ge12, ~ge02 & ~ge12]
    second = [ge01 | ge02, ~ge01 | ge12, ~ge02 | ~ge12]
    second = [sec & ~fst for sec, fst in zip(second, first)]
    steps = [[np.zeros_like(s)] * 3,
             [f.astype(np.float64) for f in first],
             [(f | g).astype(np.float64) for f, g in zip(first, second)],
             [np.ones_like(s)] * 3]
    ii = [i.astype(np.int64) & 255 for i in ijk]
    total = np.zeros_like(s)
    for k, o in enumerate(steps):
        d = [d0[ax] - o[ax] + k / 6.0 for ax in range(3)]
        w = 0.6 - (d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        oi = [o[ax].astype(np.int64) for ax in range(3)]
        h = P[(ii[0] + oi[0] + P[(ii[1] + oi[1] + P[(ii[2] + oi[2]) & 255]) & 255]) & 255] % 12
        g = SIMPLEX_GRADS[h]
        dot = g[..., 0] * d[0] + g[..., 1] * d[1] + g[..., 2] * d[2]
        total += np.where(w > 0.0, np.maximum(w, 0.0) ** 4 * dot, 0.0)
    return 32.0 * total


def _deposit_taper(t, f_top, f_base):
    def tau(z):
        z = np.asarray(z, np.float64)
        return np.minimum(z / (f_top * t), 1.0) * np.minimum((t - z) / (f_base * t), 1.0)
    return tau


def deposit_simplex(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, thick, vbed, beta: float,
                    perm_b, lam_b, a_B: float, perm_t, lam_t, tex_off, a_eta: float, f_top: float,
                    f_base: float):
    """Alg. 1 (boundary path) with both noise fields from 3D simplex noise:
    boundary i (i = 1..n-1, mean depth H_i = thick_0 + .. + thick_{i-1}
    cells) moves by taper(H_i) a_B S_b(H_i dz / lam_b[0], y dy / lam_b[1],
    x dx / lam_b[2]) -- the 3D field perm_b sampled on the plane at the
    boundary's own depth, so close boundaries move together -- and is clamped
    to [0, t-1]; the texture is a_eta S_t(((z - S_l) dz + tex_off_l) /
    lam_t[0], y dy / lam_t[1], x dx / lam_t[2]) with the field perm_t.  The
    rest (bed lookup, depth trend, taper) is `deposit`'s; lengths in metres,
    a_B in cells, a_eta in m/s."""
    thick = np.asarray(thick, np.float64)
    vbed = np.asarray(vbed, np.float64)
    n = thick.size
    H = np.cumsum(thick)[:-1]
    vbar = vbed.mean()
    tau = _deposit_taper(t, f_top, f_base)
    Yb = (np.arange(ny) * dy / lam_b[1])[None, :, None]
    Xb = (np.arange(nx) * dx / lam_b[2])[None, None, :]
    Zb = (H * dz / lam_b[0])[:, None, None]
    shp = (n - 1, ny, nx)
    eta_b = simplex_noise3d(perm_b, np.broadcast_to(Zb, shp), np.broadcast_to(Yb, shp), np.broadcast_to(Xb, shp))
    Hyx = np.clip(H[:, None, None] + tau(H)[:, None, None] * a_B * eta_b, 0.0, t - 1.0)
    z = np.arange(t, dtype=np.float64)[:, None, None]
    le = Hyx[None, :, :, :] <= z[:, None, :, :]
    bed = le.sum(axis=1)
    start = np.where(le, Hyx[None], 0.0).max(axis=1, initial=0.0)
    zt = ((z - start) * dz + np.asarray(tex_off, np.float64)[bed]) / lam_t[0]
    Y = np.broadcast_to((np.arange(ny) * dy / lam_t[1])[None, :, None], zt.shape)
    X = np.broadcast_to((np.arange(nx) * dx / lam_t[2])[None, None, :], zt.shape)
    eta = simplex_noise3d(perm_t, zt, Y, X)
    return (vbar + beta * z * dz) + tau(z) * ((vbed[bed] - vbar) + a_eta * eta)


def warped_axis(freq_raw, sigma: float):
    """The z-warped axis of Deposit's sinusoidal mode: the instantaneous
    frequency freq_raw [t] (cycles per cell, the random draw) smoothed by a
    Gaussian of sigma cells (SciPy's gaussian_filter1d, reflecting ends,
    truncated at 4 sigma; sigma 0 leaves it), then summed: W[z] =
    f[0] + .. + f[z-1] cycles above depth z (W[0] = 0)."""
    from scipy import ndimage as nd
    f = np.asarray(freq_raw, np.float64)
    if sigma > 0:
        f = nd.gaussian_filter1d(f, sigma, mode="reflect", truncate=4.0)
    return np.concatenate([[0.0], np.cumsum(f)[:-1]])


def deposit_sinusoidal(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, v0: float, beta: float,
                       freq_raw, sigma: float, amp1: float, amp2: float, phase2: float, rug, a_r: float,
                       perm_t, lam_t, a_eta: float, f_top: float, f_base: float):
    """Deposit's sinusoidal bedform mode (the prose of App. B's Deposit):
    phi(z, y, x) = 2 pi (W[z] + a_r rug(y, x)), W the warped axis of
    `warped_axis(freq_raw, sigma)` and rug [ny, nx] a roughness field (e.g.
    fractal noise of amplitude 1; a_r in cycles); then
      V = (v0 + beta z dz) + taper(z) [amp1 sin(phi) + amp2 sin(2 phi + phase2)
                                       + a_eta S_t(z dz / lam_t[0], y dy / lam_t[1], x dx / lam_t[2])]
    with the taper of Alg. 1 and S_t the simplex field perm_t (the patchy
    texture).  amp1, amp2, a_eta in m/s, beta in m/s per m."""
    W = warped_axis(freq_raw, sigma)
    tau = _deposit_taper(t, f_top, f_base)
    z = np.arange(t, dtype=np.float64)[:, None, None]
    phi = 2.0 * np.pi * (W[:, None, None] + a_r * np.asarray(rug, np.float64)[None, :, :])
    shp = (t, ny, nx)
    Z = np.broadcast_to(z * dz / lam_t[0], shp)
    Y = np.broadcast_to((np.arange(ny) * dy / lam_t[1])[None, :, None], shp)
    X = np.broadcast_to((np.arange(nx) * dx / lam_t[2])[None, None, :], shp)
    eta = simplex_noise3d(perm_t, Z, Y, X)
    return (v0 + beta * z * dz) + tau(z) * (amp1 * np.sin(phi) + amp2 * np.sin(2.0 * phi + phase2) + a_eta * eta)


def salt_sdt(V, dz: float, dy: float, dx: float, centres, radii, rotations, grf, amplitude: float,
             v_salt: float, v_water: float, min_voxels: int = 1000):
    """Alg. 4 (SaltSDT).  Per body i: the rotated ellipsoid (centre [3] and
    radii [3] in metres as (z, y, x), rotation [3, 3] taking world offsets to
    the body frame) rasterised on the voxel centres, its signed distance phi
    (distance to the nearest voxel outside minus distance to the nearest voxel
    inside, in metres; SciPy's exact EDT), phi' = phi + amplitude * rbar * grf[i]
    (rbar = mean radius), K |= phi' > 0.  Then K is opened and closed with the
    6-neighbour cross (outside the volume counts as empty), components
    (6-connected) smaller than min_voxels are dropped, K is restricted to
    V >= v_water and V[K] = v_salt.  A body that covers no voxel adds nothing;
    one that covers every voxel adds them all.  Returns (V', K)."""
    from scipy import ndimage as nd
    V = np.asarray(V, np.float64)
    nz, ny, nx = V.shape
    Z, Y, X = np.meshgrid(np.arange(nz) * dz, np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    P = np.stack([Z, Y, X], axis=-1)
    K = np.zeros(V.shape, bool)
    samp = (dz, dy, dx)
    for i in range(len(centres)):
        c = np.asarray(centres[i], np.float64)
        r = np.asarray(radii[i], np.float64)
        Rm = np.asarray(rotations[i], np.float64)
        u = (P - c) @ Rm.T
        mask = np.sum((u / r) ** 2, axis=-1) <= 1.0
        if not mask.any():
            continue
        if mask.all():
            K[:] = True
            continue
        phi = nd.distance_transform_edt(mask, sampling=samp) - nd.distance_transform_edt(~mask, sampling=samp)
        K |= (phi + amplitude * r.mean() * np.asarray(grf[i], np.float64)) > 0
    cross = nd.generate_binary_structure(3, 1)
    K = nd.binary_opening(K, structure=cross)
    K = nd.binary_closing(K, structure=cross)
    lab, n = nd.label(K, structure=cross)
    if n:
        sizes = np.bincount(lab.ravel())
        K &= sizes[lab] >= min_voxels
        K &= lab > 0
    K &= V >= v_water
    out = V.copy()
    out[K] = v_salt
    return out, K


def grf_grid(nz: int, ny: int, nx: int):
    """The periodic grid the random field of Alg. 4 is sampled on: the
    smallest power of two >= each extent (reading: the field is sampled on a
    periodic grid containing the volume and cropped to it)."""
    return tuple(1 << max(0, int(n - 1).bit_length()) for n in (nz, ny, nx))


def grf(noise, shape, ell, p: float):
    """Alg. 4, the random field xi of one body: white noise (an input, [Pz, Py,
    Px] on grf_grid(*shape)) shaped in Fourier space by sqrt(P(k)),
    P(k) = (1 + sum_k (k_k ell_k)^2)^-p, k_k the angular wavenumber in radians
    per cell of the periodic grid along axis k and ell_k in cells; the real
    part of the inverse transform cropped to shape = (nz, ny, nx), then scaled
    to zero mean and unit variance over the volume (the paper fixes neither;
    the amplitude a of Alg. 4 multiplies this field)."""
    noise = np.asarray(noise, np.float64)
    nz, ny, nx = shape
    assert noise.shape == grf_grid(nz, ny, nx), noise.shape
    ks = [2.0 * np.pi * np.fft.fftfreq(n) for n in noise.shape]
    kz, ky, kx = np.meshgrid(*ks, indexing="ij")
    amp = (1.0 + (kz * ell[0]) ** 2 + (ky * ell[1]) ** 2 + (kx * ell[2]) ** 2) ** (-0.5 * p)
    xi = np.fft.ifftn(np.fft.fftn(noise) * amp).real[:nz, :ny, :nx]
    sd = xi.std()
    return (xi - xi.mean()) / sd if sd > 0 else np.zeros_like(xi)   # one cell: no variance to scale
