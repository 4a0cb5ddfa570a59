"""Python binding of libsgwave (the C ABI of include/sgwave.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch supplies device memory and the stream; arrays cross the
boundary as raw pointers.  The ``sg_*`` functions mirror the C calls one for
one; ``Plan`` and the helpers below them only allocate the caller-owned
buffers the C calls expect.
"""
from __future__ import annotations

import ctypes
import math
import os
import re
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SGWAVE_LIBRARY selects another build of the same library (e.g. the host
# sanitizer build of build.py --sanitize); there is no fallback either way
LIB_PATH = os.environ.get("SGWAVE_LIBRARY") or os.path.join(_HERE, "_build", "libsgwave.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sgwave.h")

SG_OK, SG_EINVAL, SG_ECFL, SG_ENOSPACE, SG_EHIP, SG_EDIVERGED, SG_EUNSUPPORTED = range(7)
SG_TOP_FREE, SG_TOP_ABSORBING = 0, 1
SG_ALLOW_UNSTABLE = 1
SG_WARN_DISPERSION = 1


class SGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


_STATUS_NAMES = {0: "SG_OK", 1: "SG_EINVAL", 2: "SG_ECFL", 3: "SG_ENOSPACE", 4: "SG_EHIP",
                 5: "SG_EDIVERGED", 6: "SG_EUNSUPPORTED"}


class sg_geometry(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("dz", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("nbl", ctypes.c_int32), ("top", ctypes.c_int32),
                ("damp_R", ctypes.c_double), ("vmax_hint", ctypes.c_double),
                ("vmin_hint", ctypes.c_double), ("fmax_hint", ctypes.c_double),
                ("rec_every", ctypes.c_int32), ("snap_every", ctypes.c_int32),
                ("snap_count", ctypes.c_int32)]


class sg_shots(ctypes.Structure):
    _fields_ = [("nshot", ctypes.c_int32), ("src_zx", ctypes.POINTER(ctypes.c_double)),
                ("nrec", ctypes.c_int32), ("rec_zx", ctypes.POINTER(ctypes.c_double)),
                ("wavelet", ctypes.c_void_p), ("wavelet_per_shot", ctypes.c_int32)]


class sg_tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("time_block", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32)]


class sg_batch_item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("vp", ctypes.c_void_p),
                ("shots", ctypes.POINTER(sg_shots)), ("gathers", ctypes.c_void_p),
                ("snaps", ctypes.c_void_p)]


class sg_batch_grad_item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("vp", ctypes.c_void_p),
                ("shots", ctypes.POINTER(sg_shots)), ("resid", ctypes.c_void_p),
                ("grad", ctypes.c_void_p)]


_lib = None
class sg_fault_params(ctypes.Structure):
    _fields_ = [("cz", ctypes.c_double), ("cy", ctypes.c_double), ("cx", ctypes.c_double),
                ("azimuth_deg", ctypes.c_double), ("dip_deg", ctypes.c_double), ("radius", ctypes.c_double),
                ("slip", ctypes.c_double), ("direction", ctypes.c_int32), ("die_r", ctypes.c_double),
                ("die_strike", ctypes.c_double), ("die_theta_deg", ctypes.c_double),
                ("rough_lattice", ctypes.c_void_p), ("rough_noct", ctypes.c_int32), ("rough_gd", ctypes.c_int32),
                ("rough_gs", ctypes.c_int32), ("rough_amplitude", ctypes.c_double),
                ("rough_lam_strike", ctypes.c_double), ("rough_lam_dip", ctypes.c_double)]


class sg_riedel_config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("synthetic_fraction", "hangingwall_fraction", "synthetic_offset_deg",
                                               "antithetic_offset_deg", "along_strike", "across_min", "across_max",
                                               "size_scale", "slip_min", "slip_max", "min_distance")]


_FAULT_FIELDS = ("cz", "cy", "cx", "azimuth_deg", "dip_deg", "radius", "slip", "direction", "die_r", "die_strike",
                 "die_theta_deg")


def _fault_params(params: dict, device=None) -> sg_fault_params:
    """sg_fault_params from a dict of its fields; an optional rough surface is
    given by rough_lattice (a float32 device tensor [noct, gd, gs] on
    `device`), rough_amplitude, rough_lam_strike and rough_lam_dip."""
    p = sg_fault_params(**{k: params[k] for k in _FAULT_FIELDS})
    lat = params.get("rough_lattice")
    if lat is not None:
        _need(lat, "rough_lattice", "float32", (None, None, None), device)
        p.rough_lattice = lat.data_ptr()
        p.rough_noct, p.rough_gd, p.rough_gs = lat.shape
        p.rough_amplitude = params["rough_amplitude"]
        p.rough_lam_strike = params["rough_lam_strike"]
        p.rough_lam_dip = params["rough_lam_dip"]
    return p


_SIGS = {
    "sg_abi_version": (ctypes.c_int32, []),
    "sg_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "sg_last_error": (ctypes.c_char_p, []),
    "sg_plan_create": (ctypes.c_int32, [ctypes.POINTER(sg_geometry), ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "sg_plan_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "sg_plan_warnings": (ctypes.c_uint32, [ctypes.c_void_p]),
    "sg_plan_reserve": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "sg_grf_workspace_size": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t)]),
    "sg_grf": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_void_p]),
    "sg_plan_padded_shape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
    "sg_plan_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sg_tuning)]),
    "sg_plan_get_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(sg_tuning)]),
    "sg_plan_set_profiling": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "sg_plan_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "sg_ricker": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_float)]),
    "sg_cfl_dt_max": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "sg_forward_workspace_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "sg_forward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(sg_shots),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]),
    "sg_forward_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(sg_shots),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_grad_workspace_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sg_forward_ckpt": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(sg_shots),
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "sg_adjoint_gradient": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(sg_shots),
                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sg_batch_workspace_size": (ctypes.c_int32, [ctypes.POINTER(sg_batch_item), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "sg_batch_forward": (ctypes.c_int32, [ctypes.POINTER(sg_batch_item), ctypes.c_int32,
                                          ctypes.POINTER(sg_tuning), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "sg_check_finite": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "sg_set_graphs": (ctypes.c_int32, [ctypes.c_int32]),
    "sg_fractal_noise2d": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "sg_deposit": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "sg_simplex_noise3d": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
                           + [ctypes.c_double] * 7 + [ctypes.c_void_p, ctypes.c_void_p]),
    "sg_deposit_simplex": (ctypes.c_int32, [ctypes.c_int32] * 3 + [ctypes.c_double] * 3
                           + [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
                           + [ctypes.c_double] * 4 + [ctypes.c_void_p] + [ctypes.c_double] * 3
                           + [ctypes.c_void_p] + [ctypes.c_double] * 3 + [ctypes.c_void_p, ctypes.c_void_p]),
    "sg_deposit_sinusoidal": (ctypes.c_int32, [ctypes.c_int32] * 3 + [ctypes.c_double] * 5
                              + [ctypes.c_void_p] + [ctypes.c_double] * 4 + [ctypes.c_void_p, ctypes.c_double,
                                                                             ctypes.c_void_p]
                              + [ctypes.c_double] * 6 + [ctypes.c_void_p, ctypes.c_void_p]),
    "sg_squish": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_fault": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.POINTER(sg_fault_params), ctypes.c_float,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "sg_fault_sequence": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.POINTER(sg_fault_params), ctypes.c_int32, ctypes.c_float,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_fault_labels_sequence": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                  ctypes.POINTER(sg_fault_params), ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_riedel_subsidiaries": (ctypes.c_int32, [ctypes.POINTER(sg_fault_params), ctypes.POINTER(sg_riedel_config),
                                                ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(sg_fault_params), ctypes.POINTER(ctypes.c_int32)]),
    "sg_salt_workspace_size": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "sg_salt_sdt": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sg_fault_labels": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(sg_fault_params), ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "sg_wave_residual_workspace_size": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sg_wave_residual": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "sg_bandpass_ricker": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_float)]),
    "sg_batch_autotune": (ctypes.c_int32, [ctypes.POINTER(sg_batch_item), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                           ctypes.POINTER(sg_tuning)]),
    "sg_batch_grad_workspace_size": (ctypes.c_int32, [ctypes.POINTER(sg_batch_grad_item), ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    "sg_batch_adjoint_gradient": (ctypes.c_int32, [ctypes.POINTER(sg_batch_grad_item), ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(sg_tuning),
                                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sg_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(sg_shots), ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.POINTER(sg_tuning)]),
}


def lib():
    """The loaded libsgwave.  Raises if the library has not been built: there
    is no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsgwave.so is not built (%s); run python -m paper_2605_30541_amd.build" % LIB_PATH)
        # torch (which owns device memory and streams here) is loaded first:
        # loading this library before torch's HIP runtime has left the
        # library's later HIP calls without a device
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/sgwave.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", text)) - {"sg_shots"})


def _check(status: int):
    if status != SG_OK:
        raise SGError(status, lib().sg_last_error().decode())


# ------------------------------------------------------------------ C calls

def sg_abi_version() -> int:
    return lib().sg_abi_version()


def sg_status_string(s: int) -> str:
    return lib().sg_status_string(s).decode()


def sg_last_error() -> str:
    return lib().sg_last_error().decode()


def sg_ricker(f0: float, dt: float, nt: int, t0: float = 0.0) -> np.ndarray:
    out = np.empty(nt, np.float32)
    _check(lib().sg_ricker(f0, dt, nt, t0, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def sg_cfl_dt_max(dz: float, dx: float, vmax: float) -> float:
    return lib().sg_cfl_dt_max(dz, dx, vmax)


@dataclass
class Geometry:
    """Mirror of sg_geometry (include/sgwave.h)."""
    nz: int
    nx: int
    dz: float
    dx: float
    dt: float
    nt: int
    nbl: int = 40
    top: int = SG_TOP_FREE
    damp_R: float = 1e-3
    vmax_hint: float = 5000.0
    vmin_hint: float = 0.0
    fmax_hint: float = 0.0
    rec_every: int = 1
    snap_every: int = 0
    snap_count: int = 0

    def c(self) -> sg_geometry:
        return sg_geometry(self.nz, self.nx, self.dz, self.dx, self.dt, self.nt, self.nbl, self.top,
                           self.damp_R, self.vmax_hint, self.vmin_hint, self.fmax_hint,
                           self.rec_every, self.snap_every, self.snap_count)

    @property
    def nrow(self) -> int:
        return -(-self.nt // self.rec_every)


class Plan:
    """Owner of one sg_plan*."""

    def __init__(self, geom: Geometry, flags: int = 0):
        self.geom = geom
        self._g = geom.c()
        h = ctypes.c_void_p()
        _check(lib().sg_plan_create(ctypes.byref(self._g), flags, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sg_plan_destroy(self.handle)
            self.handle = None

    @property
    def warnings(self) -> int:
        return lib().sg_plan_warnings(self.handle)

    @property
    def padded_shape(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sg_plan_padded_shape(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_tuning(self, variant=0, tile_x=0, tile_z=0, time_block=0, rows_per_thread=0):
        t = sg_tuning(variant, tile_x, tile_z, time_block, rows_per_thread)
        _check(lib().sg_plan_set_tuning(self.handle, ctypes.byref(t)))

    def reserve(self, nshot: int, nrec: int, ckpt_every: int = 0):
        """Size the plan's pinned table staging (sg_plan_reserve)."""
        _check(lib().sg_plan_reserve(self.handle, nshot, nrec, ckpt_every))

    def clear_tuning(self):
        _check(lib().sg_plan_set_tuning(self.handle, None))

    def set_profiling(self, on: bool):
        _check(lib().sg_plan_set_profiling(self.handle, 1 if on else 0))

    def profile(self):
        """(summed kernel ms, launches) of the time-stepping kernels of the last call."""
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib().sg_plan_profile(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def get_tuning(self, nshot: int = 1):
        t = sg_tuning()
        _check(lib().sg_plan_get_tuning(self.handle, nshot, ctypes.byref(t)))
        return dict(variant=t.variant, tile_x=t.tile_x, tile_z=t.tile_z, time_block=t.time_block,
                    rows_per_thread=t.rows_per_thread)


@dataclass
class Shots:
    """Host side of sg_shots; `wavelet` is a float32 CUDA tensor [1 or nshot, nt]."""
    src_zx: np.ndarray
    rec_zx: np.ndarray
    wavelet: object
    _keep: list = field(default_factory=list, repr=False)

    def c(self, nt: int) -> sg_shots:
        """The C struct for a plan of `nt` levels; the wavelet must be a
        contiguous float32 CUDA tensor [nt], [1, >= nt] or [nshot, nt]."""
        src = np.ascontiguousarray(np.asarray(self.src_zx, np.float64).reshape(-1, 2))
        rec = np.ascontiguousarray(np.asarray(self.rec_zx, np.float64).reshape(-1, 2))
        self._keep = [src, rec]
        w = self.wavelet
        _need(w, "wavelet", "float32")
        if w.dim() not in (1, 2):
            raise ValueError("wavelet must be [nt], [1, nt] or [nshot, nt]")
        per_shot = 1 if (w.dim() == 2 and w.shape[0] > 1) else 0
        if per_shot and w.shape[0] != src.shape[0]:
            raise ValueError("wavelet rows must be 1 or nshot")
        if (per_shot and w.shape[-1] != nt) or w.shape[-1] < nt:
            raise ValueError("wavelet rows hold %d samples; the plan needs %d" % (w.shape[-1], nt))
        return sg_shots(src.shape[0], src.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        rec.shape[0], rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.c_void_p(w.data_ptr()), per_shot)

    @property
    def nshot(self) -> int:
        return int(np.asarray(self.src_zx).reshape(-1, 2).shape[0])

    @property
    def nrec(self) -> int:
        return int(np.asarray(self.rec_zx).reshape(-1, 2).shape[0])


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, dtype, shape=None, device=None, optional=False):
    """Raise ValueError unless `t` is a contiguous CUDA tensor of `dtype`
    ("float32", "float64", "int32" or "uint8") whose shape equals `shape`
    (None entries match any extent) and that lives on `device` when given.
    The library dereferences these pointers on the GPU: a host tensor, a
    wrong element type or a short buffer would be read out of bounds."""
    import torch
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP device) tensor" % name)
    if t.dtype != getattr(torch, dtype):
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and (t.dim() != len(shape) or
                              any(e is not None and a != e for a, e in zip(t.shape, shape))):
        want = "[" + ", ".join("*" if e is None else str(e) for e in shape) + "]"
        raise ValueError("%s has shape %s; expected %s" % (name, list(t.shape), want))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s; expected %s" % (name, t.device, device))


def _need_ws(ws, device):
    _need(ws, "workspace", "uint8", device=device)


def _check_slice_args(plan: "Plan", vp, shots: "Shots", gathers=None, snaps=None, resid=None, grad=None,
                      gathers_optional=True):
    """Validates the device tensors of a call on one slice against its plan."""
    g = plan.geom
    _need(vp, "vp", "float32", (g.nz, g.nx))
    dev = vp.device
    ns, nr = shots.nshot, shots.nrec
    _need(shots.wavelet, "wavelet", "float32", device=dev)
    _need(gathers, "gathers", "float32", (ns, g.nrow, nr), dev, optional=gathers_optional)
    _need(snaps, "snaps", "float32", (ns, g.snap_count, g.nz, g.nx), dev, optional=True)
    _need(resid, "resid", "float32", (ns, g.nrow, nr), dev, optional=resid is None)
    _need(grad, "grad", "float32", (g.nz, g.nx), dev, optional=grad is None)
    return dev


def sg_forward_workspace_size(plan: Plan, nshot: int, nrec: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().sg_forward_workspace_size(plan.handle, nshot, nrec, ctypes.byref(n)))
    return n.value


def sg_forward(plan: Plan, vp, shots: Shots, gathers, snaps, ws, stream=None):
    _need_ws(ws, _check_slice_args(plan, vp, shots, gathers, snaps))
    sh = shots.c(plan.geom.nt)
    _check(lib().sg_forward(plan.handle, _ptr(vp), ctypes.byref(sh), _ptr(gathers), _ptr(snaps),
                            _ptr(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)))


def sg_forward_noalloc(plan: Plan, vp, shots: Shots, gathers, snaps, stream=None):
    """sg_forward with the library's static device scratch as its workspace."""
    _check_slice_args(plan, vp, shots, gathers, snaps)
    sh = shots.c(plan.geom.nt)
    _check(lib().sg_forward_noalloc(plan.handle, _ptr(vp), ctypes.byref(sh), _ptr(gathers), _ptr(snaps),
                                    _stream_ptr(stream)))


def sg_grad_workspace_size(plan: Plan, nshot: int, nrec: int, ckpt_every: int = 0) -> int:
    n = ctypes.c_size_t()
    _check(lib().sg_grad_workspace_size(plan.handle, nshot, nrec, ckpt_every, ctypes.byref(n)))
    return n.value


def sg_forward_ckpt(plan: Plan, vp, shots: Shots, ckpt_every: int, gathers, ws, stream=None):
    _need_ws(ws, _check_slice_args(plan, vp, shots, gathers))
    sh = shots.c(plan.geom.nt)
    _check(lib().sg_forward_ckpt(plan.handle, _ptr(vp), ctypes.byref(sh), ckpt_every, _ptr(gathers),
                                 _ptr(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)))


def sg_adjoint_gradient(plan: Plan, vp, shots: Shots, ckpt_every: int, resid, grad, ws, stream=None):
    _need_ws(ws, _check_slice_args(plan, vp, shots, resid=resid, grad=grad))
    sh = shots.c(plan.geom.nt)
    _check(lib().sg_adjoint_gradient(plan.handle, _ptr(vp), ctypes.byref(sh), ckpt_every, _ptr(resid),
                                     _ptr(grad), _ptr(ws), ws.numel() * ws.element_size(),
                                     _stream_ptr(stream)))


def _batch_items(items):
    """items: list of (plan, vp, shots, gathers, snaps) -> ctypes array (and keep-alive list)."""
    keep = []
    arr = (sg_batch_item * len(items))()
    for i, (plan, vp, shots, gathers, snaps) in enumerate(items):
        _check_slice_args(plan, vp, shots, gathers, snaps)
        sh = shots.c(plan.geom.nt)
        keep.append(sh)
        arr[i] = sg_batch_item(plan.handle, vp.data_ptr(), ctypes.pointer(sh),
                               gathers.data_ptr() if gathers is not None else None,
                               snaps.data_ptr() if snaps is not None else None)
    return arr, keep


def sg_batch_workspace_size(items) -> int:
    arr, keep = _batch_items(items)
    n = ctypes.c_size_t()
    _check(lib().sg_batch_workspace_size(arr, len(items), ctypes.byref(n)))
    return n.value


def sg_batch_forward(items, ws, tuning=None, stream=None):
    arr, keep = _batch_items(items)
    _need_ws(ws, items[0][1].device if items else None)
    t = None
    if tuning is not None:
        t = ctypes.byref(sg_tuning(tuning.get("variant", 2), tuning.get("tile_x", 0), tuning.get("tile_z", 0),
                                   tuning.get("time_block", 0), tuning.get("rows_per_thread", 0)))
    _check(lib().sg_batch_forward(arr, len(items), t, _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream_ptr(stream)))


def sg_batch_autotune(items, ws, trial_levels: int = 64, stream=None) -> dict:
    """Fastest tuning for the whole batch (a dict for sg_batch_forward's `tuning`)."""
    arr, keep = _batch_items(items)
    _need_ws(ws, items[0][1].device if items else None)
    t = sg_tuning()
    _check(lib().sg_batch_autotune(arr, len(items), trial_levels, _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream_ptr(stream), ctypes.byref(t)))
    return dict(variant=t.variant, tile_x=t.tile_x, tile_z=t.tile_z, time_block=t.time_block,
                rows_per_thread=t.rows_per_thread)


def sg_autotune(plan: Plan, vp, shots: Shots, trial_levels: int, ws, stream=None) -> dict:
    _need_ws(ws, _check_slice_args(plan, vp, shots))
    sh = shots.c(plan.geom.nt)
    t = sg_tuning()
    _check(lib().sg_autotune(plan.handle, _ptr(vp), ctypes.byref(sh), trial_levels, _ptr(ws),
                             ws.numel() * ws.element_size(), _stream_ptr(stream), ctypes.byref(t)))
    return dict(variant=t.variant, tile_x=t.tile_x, tile_z=t.tile_z, time_block=t.time_block,
                rows_per_thread=t.rows_per_thread)


def _grad_items(items):
    """items: list of (plan, vp, shots, resid, grad) -> ctypes array (and keep-alive list)."""
    keep = []
    arr = (sg_batch_grad_item * len(items))()
    for i, (plan, vp, shots, resid, grad) in enumerate(items):
        _check_slice_args(plan, vp, shots, resid=resid, grad=grad)
        sh = shots.c(plan.geom.nt)
        keep.append(sh)
        arr[i] = sg_batch_grad_item(plan.handle, vp.data_ptr(), ctypes.pointer(sh), resid.data_ptr(),
                                    grad.data_ptr())
    return arr, keep


def sg_batch_grad_workspace_size(items, ckpt_every=0, shots_per_wave=0) -> int:
    arr, keep = _grad_items(items)
    n = ctypes.c_size_t()
    _check(lib().sg_batch_grad_workspace_size(arr, len(items), ckpt_every, shots_per_wave, ctypes.byref(n)))
    return n.value


def sg_batch_adjoint_gradient(items, ws, ckpt_every=0, shots_per_wave=0, tuning=None, stream=None):
    arr, keep = _grad_items(items)
    _need_ws(ws, items[0][1].device if items else None)
    t = None
    if tuning is not None:
        t = ctypes.byref(sg_tuning(tuning.get("variant", 2), tuning.get("tile_x", 0), tuning.get("tile_z", 0),
                                   tuning.get("time_block", 0), tuning.get("rows_per_thread", 0)))
    _check(lib().sg_batch_adjoint_gradient(arr, len(items), ckpt_every, shots_per_wave, t, _ptr(ws),
                                           ws.numel() * ws.element_size(), _stream_ptr(stream)))


def sg_wave_residual_workspace_size(nframes: int, nz: int, nx: int, top: int = SG_TOP_FREE) -> int:
    n = ctypes.c_size_t()
    _check(lib().sg_wave_residual_workspace_size(nframes, nz, nx, top, ctypes.byref(n)))
    return n.value


def fractal_noise2d(lattice, ny: int, nx: int, dy: float, dx: float, lam_y: float, lam_x: float,
                    azimuth_deg: float, amplitude: float, stream=None):
    """Displacement field [ny, nx] (float32 device tensor, metres) from the
    per-octave lattices [noct, gy, gx] (float32 device)."""
    import torch
    _need(lattice, "lattice", "float32", (None, None, None))
    noct, gy, gx = lattice.shape
    out = torch.empty((ny, nx), dtype=torch.float32, device=lattice.device)
    _check(lib().sg_fractal_noise2d(_ptr(lattice), noct, gy, gx, ny, nx, dy, dx, lam_y, lam_x, azimuth_deg,
                                    amplitude, _ptr(out), _stream_ptr(stream)))
    return out


def deposit(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, thick, vbed, beta: float, eta_b,
            a_B: float, tex_lattice, lam, tex_off, a_eta: float, f_top: float, f_base: float, stream=None):
    """Interbedded band [t, ny, nx] of Alg. 1 from device float32 tables:
    thick/vbed/tex_off [nbeds], eta_b [nbeds-1, ny, nx], tex_lattice
    [gz, gy, gx]; lam = (lam_z, lam_y, lam_x) in metres."""
    import torch
    _need(thick, "thick", "float32", (None,))
    nbeds = thick.numel()
    dev = thick.device
    _need(vbed, "vbed", "float32", (nbeds,), dev)
    _need(tex_off, "tex_off", "float32", (nbeds,), dev)
    _need(eta_b, "eta_b", "float32", (nbeds - 1, ny, nx), dev, optional=nbeds <= 1 or eta_b is None)
    _need(tex_lattice, "tex_lattice", "float32", (None, None, None), dev)
    gz, gy, gx = tex_lattice.shape
    out = torch.empty((t, ny, nx), dtype=torch.float32, device=thick.device)
    _check(lib().sg_deposit(t, ny, nx, dz, dy, dx, nbeds, _ptr(thick), _ptr(vbed), beta,
                            _ptr(eta_b) if eta_b is not None else None, a_B, _ptr(tex_lattice), gz, gy, gx,
                            lam[0], lam[1], lam[2], _ptr(tex_off), a_eta, f_top, f_base, _ptr(out),
                            _stream_ptr(stream)))
    return out


def simplex_noise3d(perm, shape, origin=(0.0, 0.0, 0.0), step=(1.0, 1.0, 1.0), amplitude: float = 1.0,
                    stream=None):
    """amplitude S(origin + index * step) on a [nz, ny, nx] grid (float32
    device tensor), S the 3D simplex noise of perm (int32 device [256])."""
    import torch
    _need(perm, "perm", "int32", (256,))
    nz, ny, nx = shape
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device=perm.device)
    _check(lib().sg_simplex_noise3d(_ptr(perm), nz, ny, nx, origin[0], origin[1], origin[2], step[0], step[1],
                                    step[2], amplitude, _ptr(out), _stream_ptr(stream)))
    return out


def deposit_simplex(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, thick, vbed, beta: float, perm_b,
                    lam_b, a_B: float, perm_t, lam_t, tex_off, a_eta: float, f_top: float, f_base: float,
                    stream=None):
    """Interbedded band [t, ny, nx] of Alg. 1 with simplex contact and
    texture noise: thick/vbed/tex_off float32 [nbeds], perm_b/perm_t int32
    [256] (device); lam_b, lam_t = (z, y, x) lengths in metres."""
    import torch
    _need(thick, "thick", "float32", (None,))
    nbeds = thick.numel()
    dev = thick.device
    _need(vbed, "vbed", "float32", (nbeds,), dev)
    _need(tex_off, "tex_off", "float32", (nbeds,), dev)
    _need(perm_b, "perm_b", "int32", (256,), dev)
    _need(perm_t, "perm_t", "int32", (256,), dev)
    out = torch.empty((t, ny, nx), dtype=torch.float32, device=dev)
    _check(lib().sg_deposit_simplex(t, ny, nx, dz, dy, dx, nbeds, _ptr(thick), _ptr(vbed), beta, _ptr(perm_b),
                                    lam_b[0], lam_b[1], lam_b[2], a_B, _ptr(perm_t), lam_t[0], lam_t[1], lam_t[2],
                                    _ptr(tex_off), a_eta, f_top, f_base, _ptr(out), _stream_ptr(stream)))
    return out


def deposit_sinusoidal(t: int, ny: int, nx: int, dz: float, dy: float, dx: float, v0: float, beta: float, freq,
                       sigma: float, amp1: float, amp2: float, phase2: float, rug, a_r: float, perm_t, lam_t,
                       a_eta: float, f_top: float, f_base: float, stream=None):
    """Deposit's sinusoidal bedform band [t, ny, nx]: freq float32 [t], rug
    float32 [ny, nx] (or None with a_r = 0), perm_t int32 [256], device."""
    import torch
    _need(freq, "freq", "float32", (t,))
    dev = freq.device
    _need(rug, "rug", "float32", (ny, nx), dev, optional=rug is None)
    _need(perm_t, "perm_t", "int32", (256,), dev)
    out = torch.empty((t, ny, nx), dtype=torch.float32, device=dev)
    _check(lib().sg_deposit_sinusoidal(t, ny, nx, dz, dy, dx, v0, beta, _ptr(freq), sigma, amp1, amp2, phase2,
                                       _ptr(rug) if rug is not None else None, a_r, _ptr(perm_t), lam_t[0], lam_t[1],
                                       lam_t[2], a_eta, f_top, f_base, _ptr(out), _stream_ptr(stream)))
    return out


def squish(v, dz: float, shift, stream=None):
    """v [nz, ny, nx] pulled from depth z + shift(y, x) (shift [ny, nx] in
    metres); float32 device tensors in, a new one out."""
    import torch
    _need(v, "v", "float32", (None, None, None))
    nz, ny, nx = v.shape
    _need(shift, "shift", "float32", (ny, nx), v.device)
    out = torch.empty_like(v)
    _check(lib().sg_squish(_ptr(v), nz, ny, nx, dz, _ptr(shift), _ptr(out), _stream_ptr(stream)))
    return out


def fault(v, dz: float, dy: float, dx: float, params: dict, fill: float, stream=None):
    """v [nz, ny, nx] through one listric normal fault; params holds the
    fields of sg_fault_params (see _fault_params for a rough surface)."""
    import torch
    _need(v, "v", "float32", (None, None, None))
    nz, ny, nx = v.shape
    p = _fault_params(params, v.device)
    out = torch.empty_like(v)
    _check(lib().sg_fault(_ptr(v), nz, ny, nx, dz, dy, dx, ctypes.byref(p), fill, _ptr(out), _stream_ptr(stream)))
    return out


def _fault_array(faults, device):
    arr = (sg_fault_params * max(len(faults), 1))()
    for k, f in enumerate(faults):
        arr[k] = _fault_params(f, device)
    return arr


def fault_sequence(v, dz: float, dy: float, dx: float, faults, fill: float, ws=None, stream=None):
    """v [nz, ny, nx] (float32 device) through the faults (a list of dicts as
    for `fault`) in order; ws: a second float32 volume of v's shape (made
    here when None and two or more faults are given)."""
    import torch
    _need(v, "v", "float32", (None, None, None))
    nz, ny, nx = v.shape
    if ws is None and len(faults) > 1:
        ws = torch.empty_like(v)
    _need(ws, "ws", "float32", tuple(v.shape), v.device, optional=ws is None)
    arr = _fault_array(faults, v.device)
    out = torch.empty_like(v)
    _check(lib().sg_fault_sequence(_ptr(v), nz, ny, nx, dz, dy, dx, arr, len(faults), fill, _ptr(out), _ptr(ws),
                                   _stream_ptr(stream)))
    return out


def fault_labels_sequence(labels, dz: float, dy: float, dx: float, faults, fill: int, ws=None, stream=None):
    """int32 device labels through the faults in order (nearest-neighbour pulls)."""
    import torch
    _need(labels, "labels", "int32", (None, None, None))
    nz, ny, nx = labels.shape
    if ws is None and len(faults) > 1:
        ws = torch.empty_like(labels)
    _need(ws, "ws", "int32", tuple(labels.shape), labels.device, optional=ws is None)
    arr = _fault_array(faults, labels.device)
    out = torch.empty_like(labels)
    _check(lib().sg_fault_labels_sequence(_ptr(labels), nz, ny, nx, dz, dy, dx, arr, len(faults), fill, _ptr(out),
                                          _ptr(ws), _stream_ptr(stream)))
    return out


def riedel_subsidiaries(primary: dict, cfg: dict, uniforms):
    """Subsidiary faults of `primary` (dict as for `fault`, smooth) from
    uniforms [n, 5] (host) and cfg (the fields of sg_riedel_config); returns a
    list of dicts."""
    u = np.ascontiguousarray(uniforms, np.float64).reshape(-1, 5)
    n = u.shape[0]
    out = (sg_fault_params * max(n, 1))()
    m = ctypes.c_int32(0)
    c = sg_riedel_config(**{k: float(cfg[k]) for k, _ in sg_riedel_config._fields_})
    _check(lib().sg_riedel_subsidiaries(ctypes.byref(_fault_params(primary)), ctypes.byref(c), n,
                                        u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out, ctypes.byref(m)))
    return [{k: getattr(out[i], k) for k in _FAULT_FIELDS} for i in range(m.value)]


def sg_salt_workspace_size(nz: int, ny: int, nx: int) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().sg_salt_workspace_size(nz, ny, nx, ctypes.byref(n)))
    return n.value


def salt_sdt(v, dz: float, dy: float, dx: float, centres, radii, rotations, grf, amplitude: float, v_salt: float,
             v_water: float, min_voxels: int = 1000, stream=None):
    """Alg. 4 on a float32 device volume v [nz, ny, nx]: centres, radii
    [nbodies, 3] and rotations [nbodies, 3, 3] (host, metres, (z, y, x)),
    grf [nbodies, nz, ny, nx] a float32 device tensor.  Returns (out, mask):
    the salted volume and K as uint8."""
    import torch
    _need(v, "v", "float32", (None, None, None))
    nz, ny, nx = v.shape
    c = np.ascontiguousarray(centres, np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, np.float64).reshape(-1, 3)
    R = np.ascontiguousarray(rotations, np.float64).reshape(-1, 9)
    nb = c.shape[0]
    if r.shape[0] != nb or R.shape[0] != nb:
        raise ValueError("centres, radii and rotations must describe the same number of bodies")
    if nb:
        _need(grf, "grf", "float32", (nb, nz, ny, nx), v.device)
    out = torch.empty_like(v)
    mask = torch.empty(v.shape, dtype=torch.uint8, device=v.device)
    ws = torch.empty(sg_salt_workspace_size(nz, ny, nx), dtype=torch.uint8, device=v.device)
    _check(lib().sg_salt_sdt(_ptr(v), nz, ny, nx, dz, dy, dx, nb, c.ctypes.data, r.ctypes.data, R.ctypes.data,
                             _ptr(grf) if nb else None, amplitude, v_salt, v_water, min_voxels, _ptr(out),
                             _ptr(mask), _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return out, mask


def fault_labels(labels, dz: float, dy: float, dx: float, params: dict, fill: int, stream=None):
    """int32 device labels [nz, ny, nx] through one listric normal fault,
    nearest-neighbour pull; params holds the fields of sg_fault_params."""
    import torch
    _need(labels, "labels", "int32", (None, None, None))
    nz, ny, nx = labels.shape
    p = _fault_params(params, labels.device)
    out = torch.empty_like(labels)
    _check(lib().sg_fault_labels(_ptr(labels), nz, ny, nx, dz, dy, dx, ctypes.byref(p), fill, _ptr(out),
                                 _stream_ptr(stream)))
    return out


def wave_residual(frames, vp, dz: float, dx: float, dt: float, top: int = SG_TOP_FREE, stream=None):
    """Per-frame sums (res2, dtt2) of the wave-equation residual of a device
    frame stack [T][nz][nx] (float32) on velocity vp [nz][nx]; returns two
    float64 device tensors of T entries."""
    import torch
    _need(frames, "frames", "float32", (None, None, None))
    T, nz, nx = frames.shape
    _need(vp, "vp", "float32", (nz, nx), frames.device)
    res2 = torch.empty(T, dtype=torch.float64, device=frames.device)
    dtt2 = torch.empty_like(res2)
    ws = torch.empty(sg_wave_residual_workspace_size(T, nz, nx, top), dtype=torch.uint8, device=frames.device)
    _check(lib().sg_wave_residual(_ptr(frames), T, nz, nx, _ptr(vp), dz, dx, dt, top, _ptr(res2), _ptr(dtt2),
                                  _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return res2, dtt2


def grf_grid(nz: int, ny: int, nx: int):
    """(periodic grid of the random field, workspace bytes) for a volume."""
    g = (ctypes.c_int32 * 3)()
    n = ctypes.c_size_t()
    _check(lib().sg_grf_workspace_size(nz, ny, nx, g, ctypes.byref(n)))
    return (g[0], g[1], g[2]), n.value


def grf(noise, shape, ell, p: float, ws=None, stream=None):
    """Alg. 4's random field [nz, ny, nx] (float32 device tensor) from white
    noise on grf_grid(*shape)[0] (float32 device), lengths ell = (lz, ly, lx)
    in cells and spectral exponent p."""
    import torch
    nz, ny, nx = shape
    grid, nbytes = grf_grid(nz, ny, nx)
    _need(noise, "noise", "float32", grid)
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device=noise.device)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=noise.device)
    _need_ws(ws, noise.device)
    _check(lib().sg_grf(_ptr(noise), nz, ny, nx, float(ell[0]), float(ell[1]), float(ell[2]), float(p), _ptr(out),
                        _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return out


def sg_set_graphs(on: bool):
    _check(lib().sg_set_graphs(1 if on else 0))


def sg_check_finite(x, ws, stream=None):
    _need(x, "x", "float32")
    _need_ws(ws, x.device)
    _check(lib().sg_check_finite(_ptr(x), x.numel(), _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream_ptr(stream)))


# ------------------------------------------------------------------ helpers

def sg_bandpass_ricker(f0: float, fmin: float, fmax: float, dt: float, nt: int,
                       bandwidth_ref: float = 24.0) -> np.ndarray:
    out = np.empty(nt, np.float32)
    _check(lib().sg_bandpass_ricker(f0, fmin, fmax, dt, nt, bandwidth_ref,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def ricker_tensor(f0: float, dt: float, nt: int, device="cuda"):
    """Ricker wavelet from sg_ricker as a [1, nt] float32 tensor."""
    import torch
    return torch.from_numpy(sg_ricker(f0, dt, nt)).reshape(1, nt).to(device)


def batch_forward(items, tuning=None, ws=None, stream=None):
    """items: list of (plan, vp, shots).  Allocates gathers (and snapshots
    when the plan asks for them) per item and runs sg_batch_forward; returns
    [(gathers, snaps), ...]."""
    import torch
    full = []
    for plan, vp, shots in items:
        g = plan.geom
        gathers = torch.empty((shots.nshot, g.nrow, shots.nrec), dtype=torch.float32, device=vp.device)
        snaps = torch.empty((shots.nshot, g.snap_count, g.nz, g.nx), dtype=torch.float32, device=vp.device) \
            if g.snap_count > 0 else None
        full.append((plan, vp, shots, gathers, snaps))
    if ws is None:
        ws = torch.empty(sg_batch_workspace_size(full), dtype=torch.uint8, device=full[0][1].device)
    sg_batch_forward(full, ws, tuning, stream)
    return [(f[3], f[4]) for f in full]


def forward(plan: Plan, vp, shots: Shots, want_gathers=True, want_snaps=None, ws=None, stream=None):
    """Allocate outputs (and the workspace unless given) with torch, run
    sg_forward, return (gathers, snaps)."""
    import torch
    g = plan.geom
    dev = vp.device
    gathers = torch.empty((shots.nshot, g.nrow, shots.nrec), dtype=torch.float32, device=dev) \
        if want_gathers and shots.nrec > 0 else None
    if want_snaps is None:
        want_snaps = g.snap_count > 0
    snaps = torch.empty((shots.nshot, g.snap_count, g.nz, g.nx), dtype=torch.float32, device=dev) \
        if want_snaps and g.snap_count > 0 else None
    if ws is None:
        ws = torch.empty(sg_forward_workspace_size(plan, shots.nshot, shots.nrec), dtype=torch.uint8,
                         device=dev)
    sg_forward(plan, vp, shots, gathers, snaps, ws, stream)
    return gathers, snaps


def _autograd():
    import torch

    class Propagate(torch.autograd.Function):
        """Shot gathers of every shot as a differentiable function of the
        velocity: forward = sg_forward_ckpt (checkpoints kept in a workspace on
        the autograd context), backward = sg_adjoint_gradient with the incoming
        gradient of the gathers as the residual."""

        @staticmethod
        def forward(ctx, vp, plan, shots, ckpt_every):
            g = plan.geom
            ws = torch.empty(sg_grad_workspace_size(plan, shots.nshot, shots.nrec, ckpt_every),
                             dtype=torch.uint8, device=vp.device)
            gathers = torch.empty((shots.nshot, g.nrow, shots.nrec), dtype=torch.float32, device=vp.device)
            sg_forward_ckpt(plan, vp, shots, ckpt_every, gathers, ws)
            ctx.save_for_backward(vp)
            ctx.plan, ctx.shots, ctx.ckpt_every, ctx.ws = plan, shots, ckpt_every, ws
            return gathers

        @staticmethod
        def backward(ctx, dgathers):
            (vp,) = ctx.saved_tensors
            grad = torch.empty_like(vp)
            sg_adjoint_gradient(ctx.plan, vp, ctx.shots, ctx.ckpt_every, dgathers.contiguous().float(),
                                grad, ctx.ws)
            ctx.ws = None
            return grad, None, None, None

    return Propagate


_PROPAGATE = None


def propagate(vp, plan: Plan, shots: Shots, ckpt_every: int = 0):
    """Differentiable forward modelling: gathers [nshot, nrow, nrec] of the
    float32 CUDA velocity `vp` [nz, nx]; vp.grad receives dJ/dv by the adjoint
    state method when a loss of the gathers is back-propagated."""
    global _PROPAGATE
    if _PROPAGATE is None:
        _PROPAGATE = _autograd()
    return _PROPAGATE.apply(vp, plan, shots, ckpt_every)
