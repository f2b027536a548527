"""MI355X (gfx950) mixed-precision Runge--Kutta time stepping for 3-D finite-difference PDEs.

The compute path is libmprk.so (hand-written HIP kernels behind the C ABI in include/mprk.h);
this package is its Python binding.  Importing it without the built library raises ImportError.
"""
from . import _abi  # noqa: F401  (raises ImportError when libmprk.so is missing)
from ._abi import *  # noqa: F401,F403
from .stepper import Batch, Stepper, from_problem, precisions, tableau  # noqa: F401
