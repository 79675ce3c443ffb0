"""MI355X engine for the multiple-Arnoldi Green's-function method.

Column-parallel Krylov solution of (zS - H) x = b per basis column over local
clusters, the Fermi-Dirac density matrix, the chemical potential by bisection,
energies and Slater-Koster forces, all in FP64 HIP kernels behind the C ABI of
``libmag.so`` (include/mag.h).  This package holds the ctypes binding, the
autograd glue and the in-tree build.
"""
from . import model  # noqa: F401
from ._lib import LIB_PATH, load  # noqa: F401
from .mag import Context, MagError, make_opts  # noqa: F401

__all__ = ["Context", "MagError", "make_opts", "model", "load", "LIB_PATH"]
