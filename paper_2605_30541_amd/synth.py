"""Seeded synthetic inputs: velocity slices and acquisition geometry.

These stand in for the paper's released dataset of 2D slices (10 km wide,
6.19 km deep at 10 m, velocities normalised into [1500, 5000] m/s; Sec. 4,
App. E.1).  No dataset item is reproduced.  This module holds no arithmetic
of the propagation method: it only draws models and positions, which both the
HIP path and the oracle then consume.

Recipes
  * flat_layers: piecewise-constant layers (the small parity case).
  * field_slice: 12 layers 1500-4500 m/s increasing with depth, one shared
    sinusoidal fold (amplitude 50-300 m, wavelength 1-5 km), one planar normal
    fault (dip 50-70 deg, throw 100-400 m), +-5 % multiplicative noise, an
    elliptical 4500 m/s salt body, clipped to [1500, 4500] m/s (the paper's
    normalisation step clips velocities into a fixed range, App. E.1).
  * uneven_slices: several field slices of random size from one seed.
"""
from __future__ import annotations

import numpy as np


def flat_layers(nz: int, nx: int, dz: float, tops_m, vels) -> np.ndarray:
    """v(z) = vels[i] for tops_m[i] <= z < tops_m[i+1]."""
    z = np.arange(nz) * dz
    v = np.empty((nz, nx), np.float32)
    for i, (top, vel) in enumerate(zip(tops_m, vels)):
        v[z >= top] = vel
    return v


def field_slice(seed: int, nz: int = 620, nx: int = 1001, dz: float = 10.0, dx: float = 10.0,
                n_layers: int = 12, vlo: float = 1500.0, vhi: float = 4500.0) -> np.ndarray:
    """Layered / folded / faulted / salt slice, float32 [nz, nx]."""
    rng = np.random.default_rng(seed)
    D, W = (nz - 1) * dz, (nx - 1) * dx
    # interface depths: sorted uniform draws with >= 60 m between neighbours
    # (less on models too shallow for that: half the mean layer thickness)
    min_gap = min(60.0, 0.5 * D / n_layers)
    for _ in range(10000):
        tops = np.sort(rng.uniform(0.0, D, n_layers - 1))
        if np.all(np.diff(np.concatenate([[0.0], tops, [D]])) >= min_gap):
            break
    else:
        tops = np.linspace(0.0, D, n_layers + 1)[1:-1]
    base = np.linspace(vlo, vhi, n_layers)
    amp = rng.uniform(50.0, 300.0)
    lam = rng.uniform(1000.0, 5000.0)
    phase = rng.uniform(0.0, 2 * np.pi)
    dip = np.deg2rad(rng.uniform(50.0, 70.0))
    x0 = rng.uniform(0.3, 0.7) * W
    throw = rng.uniform(100.0, 400.0)
    zc, xc = rng.uniform(0.45, 0.75) * D, rng.uniform(0.3, 0.7) * W
    ax, az = rng.uniform(500.0, 1500.0), rng.uniform(200.0, 500.0)

    z = (np.arange(nz) * dz)[:, None]
    x = (np.arange(nx) * dx)[None, :]
    fold = amp * np.sin(2 * np.pi * x / lam + phase)
    # hanging wall to the right of the fault plane x = x0 + z / tan(dip) moves down by `throw`
    hanging = x > x0 + z / np.tan(dip)
    zsrc = z - fold - np.where(hanging, throw, 0.0)
    layer = np.searchsorted(tops, zsrc, side="right")
    v = base[layer]
    v = v * (1.0 + 0.05 * np.clip(rng.standard_normal(v.shape), -1.0, 1.0))
    salt = ((x - xc) / ax) ** 2 + ((z - zc) / az) ** 2 <= 1.0
    v = np.where(salt, 4500.0, v)
    return np.clip(v, vlo, vhi).astype(np.float32)


def uneven_sizes(seed: int, n: int, nz_range=(400, 620), nx_range=(601, 1001)):
    """n (nz, nx) pairs drawn uniformly from the inclusive ranges."""
    rng = np.random.default_rng(seed)
    nzs = rng.integers(nz_range[0], nz_range[1] + 1, n)
    nxs = rng.integers(nx_range[0], nx_range[1] + 1, n)
    return [(int(a), int(b)) for a, b in zip(nzs, nxs)]


def uneven_slices(seed: int, n: int, nz_range=(400, 620), nx_range=(601, 1001), dz=10.0, dx=10.0):
    """Field slices of uneven size; slice i is drawn with seed + i."""
    return [field_slice(seed + i, nz, nx, dz, dx)
            for i, (nz, nx) in enumerate(uneven_sizes(seed, n, nz_range, nx_range))]


def surface_receivers(nx: int, dx: float, depth: float = 10.0) -> np.ndarray:
    """One receiver per grid column at `depth` m: [nx, 2] (z, x)."""
    return np.stack([np.full(nx, depth), np.arange(nx) * dx], 1)


def shot_line(n: int, x_lo: float, x_hi: float, depth: float = 10.0) -> np.ndarray:
    """n sources evenly spaced on [x_lo, x_hi] at `depth` m: [n, 2] (z, x)."""
    xs = np.linspace(x_lo, x_hi, n) if n > 1 else np.array([(x_lo + x_hi) / 2.0])
    return np.stack([np.full(n, depth), xs], 1)


def smoothed_1d(v: np.ndarray, sigma_m: float, dz: float) -> np.ndarray:
    """Starting model: lateral mean v(z), Gaussian-smoothed in depth (sigma in
    metres, edge padding), broadcast across x."""
    from scipy.ndimage import gaussian_filter1d
    vz = v.astype(np.float64).mean(axis=1)
    vz = gaussian_filter1d(vz, sigma_m / dz, mode="nearest")
    return np.repeat(vz[:, None], v.shape[1], axis=1).astype(np.float32)
