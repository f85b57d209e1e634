"""MI355X-native polarized lattice-Boltzmann radiative-transfer solver.

The solver is the HIP library librtlbm.so (C ABI in include/rt_lbm.h); this
package is its Python binding.  Importing it without the built library raises
ImportError: there is no CPU or Python fallback.

    from paper_2609_23057_amd import Solver, Batch, make_problem, RTSolve
"""
from . import _abi  # noqa: F401  (fails loudly if the library is missing)
from ._abi import *  # noqa: F401,F403
from .solver import Batch, RTSolve, Solver, make_problem, sqrt_checkpoint_interval  # noqa: F401
