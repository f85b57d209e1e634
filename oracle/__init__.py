"""FP64 CPU oracle for the polarized lattice-Boltzmann radiative-transfer step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the HIP path: the direction set, the phase matrix (built here by the
rotation-phase-rotation sequence of Eq. 13, the GPU host side builds it from a
Jones projection), the coefficients, streaming, readout and adjoint are all
written independently from the paper.

Every function is plain, slow and written to be checked against the paper by
eye: loops over directions and bilinear taps, a single matrix product for the
direction-pair sum, float64 throughout.

Modules
  directions  zenith x azimuth direction grid, quadrature weights, lattice
              displacements (Sec. 2.1.1, Eq. 33)
  phase       Rayleigh reduced Mueller matrix, Mueller rotation, RPR pair
              matrix, Eq. 17 weights, the full 4n x 4n collision matrix
              (Eq. 13-17, Eq. 21-22, Eq. 25/30)
  lbm         per-cell coefficients, emission/absorption/scattering/streaming
              step, boundaries, time loop, readout and diagnostics
              (Eq. 2, 6-12, 33-39, Sec. 2.1.7, Eq. "36" DOP)
  adjoint     full-storage reverse-mode gradient of an edge readout loss with
              respect to per-cell extinction, albedo and emission
  dense       brute-force dense one-step operator for tiny lattices
"""
from . import directions, phase, lbm, adjoint, dense  # noqa: F401
from .lbm import Problem, make_problem  # noqa: F401
