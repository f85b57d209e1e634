"""Writes adjoint256_fd_T500.json: float64 central differences of the
top-edge (I + DoLP) loss of the differentiation workload (adjoint256
generator on a 32 x 32 lattice, 4 x 8 directions, 500 time steps from S = 0)
with respect to the per-cell optical depth, albedo and emission at 16 seeded
random cells.

Only the oracle computes these values (test infrastructure; workloads draws
the inputs).  Run from the repository root:

    python tests/golden/make_adjoint256_fd.py

It takes a few minutes (96 forward runs of 500 steps).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import adjoint as OA  # noqa: E402
from oracle import lbm as OL  # noqa: E402

NX = NY = 32
T = 500
EDGE = 3
SEED = 41
REL_H = 1e-6


def main():
    spec = W.spec("adjoint256", nx=NX, ny=NY)
    med = W.medium(spec)
    prob = OL.make_problem(spec, med)
    S0 = np.zeros(prob.shape)
    rng = np.random.default_rng(SEED)
    flat = rng.choice(NX * NY, size=16, replace=False)
    cells = [(int(c // NX), int(c % NX)) for c in flat]
    out = {"workload": "adjoint256", "nx": NX, "ny": NY, "steps": T, "edge": EDGE, "seed": SEED,
           "rel_h": REL_H, "loss": "sum over the top row and its outgoing directions of I + DoLP",
           "cells": cells, "fd": {}}
    t0 = time.time()
    for which in ("tau", "albedo", "emis"):
        vals = []
        for cell in cells:
            vals.append(OA.central_difference(prob, S0, T, EDGE, which, cell, rel_h=REL_H))
            print(which, cell, vals[-1], "%.0fs" % (time.time() - t0), flush=True)
        out["fd"][which] = vals
    with open(os.path.join(HERE, "adjoint256_fd_T500.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
