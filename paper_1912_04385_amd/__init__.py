"""MI355X-native multi-stage (CPTR3 / CPR) preconditioned GMRES for the reduced
Jacobians of thermal-compositional-reactive porous-media flow.

The numerics live in the HIP library ``libcptr.so`` (C ABI in include/cptr.h);
``cptr`` is its thin ctypes binding."""
from . import cptr  # noqa: F401
from .cptr import Solver, decouple, bsr_spmv, default_options, solver_for, CptrError  # noqa: F401
