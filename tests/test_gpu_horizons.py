"""Parity at the horizons of the measured workloads, from S = 0, on reduced
lattices the float64 oracle follows in seconds (every cell compared):

  * the precision workload's generator (n = 128, 8 x 16 directions, 4n = 512
    contraction rows) for its 200 steps, every contraction precision;
  * the throughput workload's generator (n = 32) for its 2000 steps;
  * the differentiation workload's generator (n = 32, emission everywhere)
    for its 500 steps with sqrt(T) = 23-step checkpoints: the gradients of the
    top-edge (I + DoLP) loss against the oracle's adjoint everywhere and
    against float64 central differences at 16 seeded random cells
    (tests/golden/adjoint256_fd_T500.json, written by the oracle alone).

Each case prints its measured errors.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import GTOL, assert_close, build, stokes_errors, to_dev, to_np, tolerance
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECISIONS = ["fp32", "plain", "bf16x3", "bf16", "fp16"]
GOLD = os.path.join(os.path.dirname(__file__), "golden", "adjoint256_fd_T500.json")

_cache = {}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_run(name, over, steps):
    key = (name, tuple(sorted(over.items())), steps)
    if key not in _cache:
        spec = W.spec(name, **over)
        oprob = OL.make_problem(spec, W.medium(spec))
        _cache[key] = OL.run(np.zeros(oprob.shape), oprob, steps)
    return _cache[key]


HORIZONS = [
    ("prec1024", dict(nx=96, ny=96), 200),
    ("beam512", dict(nx=64, ny=64), 2000),
]


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("case", HORIZONS, ids=lambda c: "%s-%dx%d-T%d" % (c[0], c[1]["nx"], c[1]["ny"], c[2]))
def test_forward_at_the_workload_horizon(case, precision):
    name, over, steps = case
    spec = W.spec(name, **over)
    solver, oprob, _ = build(spec, precision)
    S = solver.empty_state()
    solver.run(S, steps)
    got = to_np(S)
    ref = _oracle_run(name, over, steps)
    # the polarisation the method computes is there: Q and U carry 0.1-1 %
    # of the intensity norm (single scattering of the unpolarised beam)
    nI = np.linalg.norm(ref[:, 0])
    assert 1e-3 < np.linalg.norm(ref[:, 1]) / nI < 1e-1
    e = stokes_errors(got, ref)
    print("horizon", name, over, steps, precision, {k: "%.2e" % v for k, v in e.items()})
    assert_close(got, ref, tolerance(precision, oprob, steps), (name, precision))


def _adjoint_reference():
    if "adj" not in _cache:
        with open(GOLD) as f:
            gold = json.load(f)
        spec = W.spec("adjoint256", nx=gold["nx"], ny=gold["ny"])
        oprob = OL.make_problem(spec, W.medium(spec))
        T = gold["steps"]
        S0 = np.zeros(oprob.shape)
        ST = OL.run(S0, oprob, T)
        _, g = OL.edge_loss(ST, oprob, gold["edge"])
        ref = OA.adjoint(S0, oprob, T, OL.readout_transpose(g, oprob, gold["edge"]))
        _cache["adj"] = (gold, spec, g, ref)
    return _cache["adj"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_gradients_at_the_differentiation_horizon(precision):
    gold, spec, g, ref = _adjoint_reference()
    T = gold["steps"]
    K = int(np.ceil(np.sqrt(T)))
    assert K == 23
    solver, _, _ = build(spec, precision)
    S = solver.empty_state()
    ck = solver.checkpoint_buffer(T, K)
    solver.run(S, T, ck, K)
    lam = solver.readout_adjoint(gold["edge"], to_dev(g, solver))
    grads = dict(zip(("tau", "albedo", "emis"), solver.adjoint(T, ck, K, lam)))
    torch.cuda.synchronize()
    tol = GTOL[precision]
    errs = {}
    for which, arr in grads.items():
        got = to_np(arr)
        r = ref["g_" + which]
        scale = np.abs(r).max()
        errs[which] = float(np.abs(got - r).max() / scale)
        fd = np.array(gold["fd"][which])
        at = np.array([got[y, x] for y, x in gold["cells"]])
        errs[which + "_fd"] = float(np.abs(at - fd).max() / scale)
    print("gradients T=%d" % T, precision, {k: "%.2e" % v for k, v in errs.items()})
    assert max(errs.values()) < tol, (precision, errs)
