"""FP64 CPU oracle for the 2D acoustic finite-difference path of SubsurfaceGen
(arXiv 2605.30541).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the HIP implementation is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product package never imports, links or calls anything here, and nothing here
imports the product package.

Contents
  * ``fdo.c`` (compiled to ``_build/libfdo.so``): the discrete scheme itself --
    padding, Cerjan sponge, 8th-order Laplacian, leapfrog, free surface, point
    sources, receivers, snapshots, and the exact adjoint and velocity gradient.
  * ``wave.py``: ctypes marshalling for ``fdo.c`` and the host-side formulas
    of the paper (Ricker pulse, CFL and dispersion limits, temporal
    subsampling, band-passed wavelets) and the residual of the discretised
    wave operator on a stack of frames.
  * ``builder.py``: the velocity-model builder modules Deposit (boundary
    path with value or simplex noise, sinusoidal mode), Squish, Fault (smooth
    and rough surfaces, labels) and SaltSDT with its random field, their
    windowed-sinc pull sampling and noise fields, in NumPy FP64.
"""
from .wave import (  # noqa: F401
    Geometry,
    build,
    forward,
    gradient,
    model_arrays,
    apply_laplacian,
    set_threads,
    ricker,
    fd_coefficients,
    cfl_smax,
    von_neumann_courant,
    cfl_dt_max,
    dispersion_h_max,
    subsample_factor,
    n_saved,
    nyquist_margin,
    c_damp,
    bandpass_ricker,
    misfit,
    wave_residual,
)
from . import builder  # noqa: F401,E402
