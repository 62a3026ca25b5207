"""MI355X-native coupled Stokes-Darcy solver (block-preconditioned Krylov).

The compute path lives in the native library ``libsd.so`` (C ABI in
include/sd.h); :mod:`paper_2108_13229_amd.sd` is its ctypes binding.
"""
from . import sd  # noqa: F401
from .sd import Problem, SDError, Server, Solver, lib, solver_opts  # noqa: F401
