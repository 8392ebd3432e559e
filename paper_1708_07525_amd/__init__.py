"""MI355X (gfx950) implementation of the porous double-diffusive MRT lattice Boltzmann
time step of Liu & He (arXiv 1708.07525).

``lbm`` is the ctypes binding of the C ABI in ``include/lbm.h``; ``serving`` is the
continuous-batching solve loop built on it.
"""
from .lbm import Batch, LbmError, Solver, footprint_bytes, lib  # noqa: F401
