"""Brute-force dense one-step operator for tiny lattices (oracle).

TEST INFRASTRUCTURE ONLY.

The step S -> S' is affine: S' = A S + b, with b the image of the zero state
(emission and inflow ghosts).  A is assembled column by column by stepping
unit vectors, which is only feasible for a few hundred unknowns.
"""
import numpy as np

from . import lbm


def step_operator(prob):
    """(A, b) with step(S) = A @ S.ravel() + b, for 4 n nx ny <= 4096."""
    N = int(np.prod(prob.shape))
    if N > 4096:
        raise ValueError("dense operator only for tiny lattices")
    b = lbm.step(np.zeros(prob.shape), prob).ravel()
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = lbm.step(e.reshape(prob.shape), prob).ravel() - b
    return A, b
