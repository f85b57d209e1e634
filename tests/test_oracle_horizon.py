"""The oracle's adjoint at the differentiation workload's horizon (500 steps)
against float64 central differences of its own forward loss, stored in
tests/golden/adjoint256_fd_T500.json by tests/golden/make_adjoint256_fd.py
(CPU; the same reference the GPU gradients meet)."""
import json
import os

import numpy as np

import workloads as W
from oracle import adjoint as OA
from oracle import lbm as OL

GOLD = os.path.join(os.path.dirname(__file__), "golden", "adjoint256_fd_T500.json")


def test_adjoint_matches_central_differences_after_500_steps():
    with open(GOLD) as f:
        gold = json.load(f)
    spec = W.spec("adjoint256", nx=gold["nx"], ny=gold["ny"])
    prob = OL.make_problem(spec, W.medium(spec))
    T = gold["steps"]
    S0 = np.zeros(prob.shape)
    ST = OL.run(S0, prob, T)
    _, g = OL.edge_loss(ST, prob, gold["edge"])
    ref = OA.adjoint(S0, prob, T, OL.readout_transpose(g, prob, gold["edge"]))
    for which in ("tau", "albedo", "emis"):
        field = ref["g_" + which]
        scale = np.abs(field).max()
        at = np.array([field[y, x] for y, x in gold["cells"]])
        fd = np.array(gold["fd"][which])
        # central differences with h = 1e-6 |p| carry O(h^2) truncation and
        # a rounding error of about 1e-16 |L| / h: with |L| ~ 500 and the
        # per-step optical depth p ~ 4e-3 that is 1e-5 absolute, 1e-6 of the
        # largest gradient (13.7); the bound leaves a factor of 3
        assert np.abs(at - fd).max() <= 5e-6 * scale, (which, np.abs(at - fd).max() / scale)
        # the sampled cells are not all negligible
        assert np.abs(fd).max() > 1e-3 * scale
