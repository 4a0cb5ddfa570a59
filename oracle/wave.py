"""ctypes marshalling for the FP64 oracle (``fdo.c``) and the paper's host-side
formulas, in double precision.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Citations name the sections, equations and tables of SubsurfaceGen
(arXiv 2605.30541).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdo.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libfdo.so")
_lib = None


def build(quiet: bool = True) -> str:
    """Compile ``fdo.c`` with gcc (-O2, OpenMP, strict IEEE double)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CGeom(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("dz", ctypes.c_double), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("nt", ctypes.c_int32),
                ("nbl", ctypes.c_int32), ("top_free", ctypes.c_int32),
                ("R", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    gp = ctypes.POINTER(_CGeom)
    i = ctypes.c_int
    lib.fdo_set_threads.argtypes = [i]
    lib.fdo_set_threads.restype = i
    lib.fdo_model_arrays.argtypes = [gp, dp, ctypes.POINTER(ctypes.c_int32), dp, dp, dp, dp, dp]
    lib.fdo_model_arrays.restype = i
    lib.fdo_apply_laplacian.argtypes = [gp, dp, dp, dp]
    lib.fdo_apply_laplacian.restype = i
    lib.fdo_forward.argtypes = [gp, dp, i, i, dp, dp, i, dp, i, dp, i, i, dp]
    lib.fdo_forward.restype = i
    lib.fdo_gradient.argtypes = [gp, dp, i, i, dp, dp, i, dp, i, dp, dp, dp, i]
    lib.fdo_gradient.restype = i
    _lib = lib
    return lib


@dataclass
class Geometry:
    """Grid and time axis of one simulation (App. E.3, Table "params").

    ``nt`` counts time levels t_n = n*dt, n = 0..nt-1 (so nt-1 updates); the
    paper's N = T/dt + 1 (5001 for 5 s at 1 ms) is this count.
    """
    nz: int
    nx: int
    dz: float
    dx: float
    dt: float
    nt: int
    nbl: int = 40
    top_free: bool = True
    R: float = 1e-3

    def _c(self) -> _CGeom:
        return _CGeom(int(self.nz), int(self.nx), float(self.dz), float(self.dx),
                      float(self.dt), int(self.nt), int(self.nbl),
                      1 if self.top_free else 0, float(self.R))

    @property
    def padded_shape(self):
        top = 0 if self.top_free else self.nbl
        return (self.nz + top + self.nbl, self.nx + 2 * self.nbl)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the oracle; returns the count in use."""
    return _load().fdo_set_threads(int(n))


def model_arrays(g: Geometry, v):
    """Padded (v, eta, a, b, W) arrays as the oracle builds them."""
    lib = _load()
    v = _f64(v)
    Nz, Nx = g.padded_shape
    out = [np.empty((Nz, Nx)) for _ in range(5)]
    nznx = (ctypes.c_int32 * 2)()
    rc = lib.fdo_model_arrays(ctypes.byref(g._c()), _dptr(v), nznx, *[_dptr(o) for o in out])
    if rc != 0:
        raise RuntimeError("fdo_model_arrays failed: %d" % rc)
    assert (nznx[0], nznx[1]) == (Nz, Nx)
    return dict(zip(("v", "eta", "a", "b", "W"), out))


def apply_laplacian(g: Geometry, v, p):
    """L p on the padded grid, with the oracle's boundary rules."""
    lib = _load()
    v, p = _f64(v), _f64(p)
    assert p.shape == g.padded_shape
    out = np.empty_like(p)
    rc = lib.fdo_apply_laplacian(ctypes.byref(g._c()), _dptr(v), _dptr(p), _dptr(out))
    if rc != 0:
        raise RuntimeError("fdo_apply_laplacian failed: %d" % rc)
    return out


def _shots(src_zx, wavelets, nt):
    src = _f64(src_zx)
    if src.ndim == 1:            # one shot, one point source
        src = src.reshape(1, 1, 2)
    elif src.ndim == 2:          # [nshot][2]: one point source per shot
        src = src.reshape(src.shape[0], 1, 2)
    nshot, nsrc = src.shape[0], src.shape[1]
    wl = _f64(wavelets)
    if wl.ndim == 1:
        wl = np.broadcast_to(wl, (nshot, nsrc, nt))
    elif wl.ndim == 2:
        wl = np.broadcast_to(wl.reshape(wl.shape[0], 1, nt), (nshot, nsrc, nt))
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    assert wl.shape == (nshot, nsrc, nt), wl.shape
    return np.ascontiguousarray(src), wl


def forward(g: Geometry, v, src_zx, wavelets, rec_zx, rec_every: int = 1,
            snap_every: int = 0, snap_count: int = 0):
    """Shot gathers (and optional snapshots) of every shot.

    src_zx: [2] | [nshot, 2] | [nshot, nsrc, 2] positions (z, x) in metres,
    wavelets: [nt] | [nshot, nt] | [nshot, nsrc, nt], rec_zx: [nrec, 2].
    Returns (gathers [nshot, ceil(nt/rec_every), nrec],
             snaps [nshot, snap_count, nz, nx] or None).
    """
    lib = _load()
    v = _f64(v)
    assert v.shape == (g.nz, g.nx)
    src, wl = _shots(src_zx, wavelets, g.nt)
    rec = _f64(rec_zx).reshape(-1, 2)
    nshot, nsrc = src.shape[:2]
    nrow = -(-g.nt // rec_every)
    gathers = np.zeros((nshot, nrow, rec.shape[0]))
    snaps = None
    if snap_count > 0:
        snaps = np.zeros((nshot, snap_count, g.nz, g.nx))
    rc = lib.fdo_forward(ctypes.byref(g._c()), _dptr(v), nshot, nsrc, _dptr(src), _dptr(wl),
                         rec.shape[0], _dptr(rec), int(rec_every), _dptr(gathers),
                         int(snap_every), int(snap_count),
                         _dptr(snaps) if snaps is not None else None)
    if rc != 0:
        raise ValueError("fdo_forward failed: %d" % rc)
    return gathers, snaps


def gradient(g: Geometry, v, src_zx, wavelets, rec_zx, resid, rec_every: int = 1,
             ckpt: int = 0, want_wavelet_grad: bool = False):
    """dJ/dv (physical [nz, nx], summed over shots) for J with dJ/dd = resid."""
    lib = _load()
    v = _f64(v)
    src, wl = _shots(src_zx, wavelets, g.nt)
    rec = _f64(rec_zx).reshape(-1, 2)
    nshot, nsrc = src.shape[:2]
    nrow = -(-g.nt // rec_every)
    resid = _f64(resid)
    assert resid.shape == (nshot, nrow, rec.shape[0]), resid.shape
    grad = np.zeros((g.nz, g.nx))
    wg = np.zeros((nshot, nsrc, g.nt)) if want_wavelet_grad else None
    rc = lib.fdo_gradient(ctypes.byref(g._c()), _dptr(v), nshot, nsrc, _dptr(src), _dptr(wl),
                          rec.shape[0], _dptr(rec), int(rec_every), _dptr(resid),
                          _dptr(grad), _dptr(wg) if wg is not None else None, int(ckpt))
    if rc != 0:
        raise ValueError("fdo_gradient failed: %d" % rc)
    return (grad, wg) if want_wavelet_grad else grad


def misfit(d, d_obs) -> float:
    """J = 1/2 sum (d - d_obs)^2 over shots, recorded samples and receivers."""
    r = np.asarray(d, np.float64) - np.asarray(d_obs, np.float64)
    return 0.5 * float(np.sum(r * r))


# --------------------------------------------------------------------------
# Host-side formulas of the paper
# --------------------------------------------------------------------------

def ricker(f0: float, dt: float, nt: int, t0: float | None = None) -> np.ndarray:
    """Ricker pulse of peak frequency f0 centred at t0 = 1/f0 (App. E.4):
    w(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def fd_coefficients(M: int = 4):
    """Central second-derivative weights c_0..c_M as exact fractions.

    They are the unique weights that make sum_m c_m (u_{j+m}+u_{j-m}) exact for
    even powers up to 2M (Fornberg 1988, cited in App. E.3.2); for M = 4 they
    are -205/72, 8/5, -1/5, 8/315, -1/560.
    """
    # closed form: c_m = 2 (-1)^{m+1} (M!)^2 / (m^2 (M-m)! (M+m)!), c_0 = -2 sum c_m
    fac = math.factorial
    c = [Fraction(0)] * (M + 1)
    for m in range(1, M + 1):
        c[m] = Fraction(2 * (-1) ** (m + 1) * fac(M) ** 2, m * m * fac(M - m) * fac(M + m))
    c[0] = -2 * sum(c[1:])
    return c


def wave_residual(frames, v, dz: float, dx: float, dt: float, top_free: bool = True):
    """Residual of the discretised acoustic operator on a stack of wavefield
    frames (App. F.5, the physics-residual ratio of the predicted wavefields):

        R_t = (u_{t+1} - 2 u_t + u_{t-1}) / dt^2 - v^2 L u_t,

    L the 8th-order Laplacian of App. E.3, dt the spacing of the frames.
    Evaluated where the frames alone define it: frames t = 1..T-2; columns
    4..nx-5; rows 4..nz-5, or rows 1..nz-5 under a free top (odd mirror
    u(-m) = -u(m) above the pinned row 0).

    Returns (res2, dtt2): per-frame sums over those cells of R_t^2 and of
    ((u_{t+1} - 2 u_t + u_{t-1}) / dt^2)^2 (zero for the first and last
    frames).  The ratio sqrt(sum res2 / sum dtt2) measures how far the
    frames are from satisfying the discrete wave equation.
    """
    u = np.asarray(frames, np.float64)
    v2 = np.asarray(v, np.float64) ** 2
    T, nz, nx = u.shape
    c = [float(x) for x in fd_coefficients()]
    z0 = 1 if top_free else 4
    res2, dtt2 = np.zeros(T), np.zeros(T)
    if T < 3 or nz - 4 <= z0 or nx <= 8:
        return res2, dtt2
    for t in range(1, T - 1):
        ut = u[t]
        if top_free:   # rows -4..-1 are the odd mirror of rows 4..1
            ut = np.concatenate([-ut[4:0:-1], ut], axis=0)
            off = 4
        else:
            off = 0
        zs = slice(z0 + off, nz - 4 + off)
        xs = slice(4, nx - 4)
        lap = (c[0] / dz ** 2 + c[0] / dx ** 2) * ut[zs, xs]
        for m in range(1, 5):
            lap = lap + c[m] / dz ** 2 * (ut[z0 + off + m:nz - 4 + off + m, xs] + ut[z0 + off - m:nz - 4 + off - m, xs])
            lap = lap + c[m] / dx ** 2 * (ut[zs, 4 + m:nx - 4 + m] + ut[zs, 4 - m:nx - 4 - m])
        dtt = (u[t + 1, z0:nz - 4, 4:nx - 4] - 2.0 * u[t, z0:nz - 4, 4:nx - 4] + u[t - 1, z0:nz - 4, 4:nx - 4]) / dt ** 2
        r = dtt - v2[z0:nz - 4, 4:nx - 4] * lap
        res2[t] = float(np.sum(r * r))
        dtt2[t] = float(np.sum(dtt * dtt))
    return res2, dtt2


def cfl_smax(M: int = 4, d: int = 2) -> float:
    """Paper's stability constant s_max = (sqrt(d sum_{m=1}^M |a_m|))^{-1}
    (App. E.3.2, "CFL Stability Condition")."""
    c = fd_coefficients(M)
    return 1.0 / math.sqrt(d * float(sum(abs(x) for x in c[1:])))


def von_neumann_courant(M: int = 4, d: int = 2) -> float:
    """Exact leapfrog stability limit on v dt / h for the same stencil:
    (v dt/h)^2 * d * max_k |symbol(k)| <= 4, the symbol's extreme at k h = pi."""
    c = fd_coefficients(M)
    sym = float(c[0] + 2 * sum(c[m] * (-1) ** m for m in range(1, M + 1)))
    return 2.0 / math.sqrt(d * abs(sym))


def cfl_dt_max(h: float, vmax: float, M: int = 4, d: int = 2) -> float:
    """dt <= s_max h / v_max (App. E.3.2)."""
    return cfl_smax(M, d) * h / vmax


def dispersion_h_max(vmin: float, fmax: float, G: float = 4.0) -> float:
    """h <= v_min / (G f_max), G = 4 for the 8th-order stencil (App. E.3.1)."""
    return vmin / (G * fmax)


def subsample_factor(N: int, fmax: float, T: float) -> int:
    """k = floor(N / (2 f_max T)) (App. E.3.3)."""
    return int(math.floor(N / (2.0 * fmax * T)))


def n_saved(N: int, k: int) -> int:
    """N_saved = ceil(N / k) (App. E.3.3)."""
    return -(-int(N) // int(k))


def nyquist_margin(fmax: float, dt_saved: float) -> float:
    """1 / (2 f_max dt_saved) (Table "bands")."""
    return 1.0 / (2.0 * fmax * dt_saved)


def c_damp(nbl: int, R: float = 1e-3) -> float:
    """c_damp = 1.5 ln(1/R) / n_bl (App. E.2, eq. "cerjan_damp")."""
    return 1.5 * math.log(1.0 / R) / nbl


def bandpass_ricker(f0: float, band: tuple[float, float], dt: float, nt: int,
                    bandwidth_ref: float = 24.0, t0: float | None = None) -> np.ndarray:
    """Band-limited source of App. E.4: Ricker(f0) centred at t0 (default
    1/f0), 4th-order zero-phase Butterworth band-pass (forward-backward
    second-order sections), divided by its l2 norm, then scaled by
    sqrt(B / 24 Hz), B = band width."""
    from scipy.signal import butter, sosfiltfilt
    w = ricker(f0, dt, nt, t0=t0)
    sos = butter(4, [band[0], band[1]], btype="bandpass", fs=1.0 / dt, output="sos")
    y = sosfiltfilt(sos, w)
    y = y / np.linalg.norm(y)
    return y * math.sqrt((band[1] - band[0]) / bandwidth_ref)
