"""MI355X-native acoustic finite-difference propagator (the seismic-data path
of SubsurfaceGen, arXiv 2605.30541).

The compute lives in the HIP library ``_build/libsgwave.so`` behind the C ABI
of ``include/sgwave.h``; ``sgwave`` is its ctypes binding.
"""
from . import sgwave  # noqa: F401
from .sgwave import Geometry, Plan, Shots, SGError, forward  # noqa: F401
