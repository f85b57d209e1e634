"""GPU parity of tabulated scattering matrices (RT_PHASE_TABLE: a general
Mueller matrix with P12 and P34 != 0, so U and V couple) against the FP64
oracle, through the C ABI: forward in every precision, the adjoint, the full
beam512 lattice, and a batch channel against its own context.

The collision matrix is dense in the Stokes index (the V rows no longer
decouple), which every kernel handles as it handles any matrix: the tests
check that the whole path follows it.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import assert_close, build, GTOL, gtolerance, to_dev, to_np, tolerance
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

TABLE = {"kind": "table", "table": W.scattering_table()}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    ("beam512", dict(nx=40, ny=33), 30),                       # n = 32
    ("beam512", dict(nx=33, ny=29, n_zen=2, n_az=8), 40),      # n = 16
    ("beam512", dict(nx=21, ny=26, n_zen=4, n_az=16), 25),     # n = 64
    ("prec1024", dict(nx=19, ny=22), 15),                      # n = 128
    ("plain32", dict(nx=30, ny=21), 40),                       # n = 8, scattering-dominated
]


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-n%d" % (
    c[0], c[1]["nx"], c[1]["ny"], W.ndir(W.spec(c[0], **c[1]))))
def test_table_forward_parity(case, precision):
    """Against the unmodified oracle in every precision.  The n = 8 medium is
    scattering-dominated (beta 0.81 per step), where the tolerance is the
    accumulation bound of the operand rounding (gpu_common.tolerance)."""
    name, over, steps = case
    spec = W.spec(name, phase=TABLE, **over)
    solver, oprob, _ = build(spec, precision)
    S0 = W.initial_state(spec, "random")
    S = to_dev(S0, solver)
    solver.run(S, steps)
    # U -> V coupling is present in the operator the oracle runs
    assert np.abs(oprob.M[3::4, 2::4]).max() > 1e-3
    ref = OL.run(S0, oprob, steps)
    e = assert_close(to_np(S), ref, tolerance(precision, oprob, steps), (name, precision))
    print(name, precision, e)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "plain"])
def test_table_adjoint_parity(precision):
    spec = W.spec("adjoint256", nx=36, ny=33, phase=TABLE)
    T, K = 20, 5
    solver, oprob, _ = build(spec, precision)
    S0 = np.zeros(oprob.shape)
    ck = solver.checkpoint_buffer(T, K)
    S = to_dev(S0, solver)
    solver.run(S, T, ck, K)
    ST = OL.run(S0, oprob, T)
    _, g = OL.edge_loss(ST, oprob, 3)
    lamT = OL.readout_transpose(g, oprob, 3)
    ref = OA.adjoint(S0, oprob, T, lamT)
    got = solver.adjoint(T, ck, K, to_dev(lamT, solver), want_lambda0=True)
    for key, arr in zip(("g_tau", "g_albedo", "g_emis", "lambda0"), got):
        assert _rel(to_np(arr), ref[key]) < gtolerance(precision, oprob, T), (key, _rel(to_np(arr), ref[key]))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_table_full_size_beam512(precision):
    """The full 512 x 512, n = 32 lattice in the checkpointed launch: every
    cell for three steps against the oracle."""
    spec = W.spec("beam512", phase=TABLE)
    solver, oprob, _ = build(spec, precision)
    rng = np.random.default_rng(41)
    S0 = np.abs(rng.standard_normal(solver.shape)) * 0.1
    S0[:, 1:] *= 0.2 * np.sign(rng.standard_normal(S0[:, 1:].shape))
    T, K = 3, 2
    S = to_dev(S0, solver)
    ck = solver.checkpoint_buffer(T, K)
    solver.run(S, T, ck, K)
    torch.cuda.synchronize()
    hist = OL.run(S0, oprob, T, keep=True)[1]
    tol = tolerance(precision, oprob)
    assert_close(to_np(S), hist[T], tol, ("S_T", precision))
    assert_close(to_np(ck[1]), hist[2], tol, ("checkpoint 1", precision))


def test_table_batch_channel_matches_its_context_bitwise():
    """A batch of a tabulated-matrix channel and an HG channel: each channel
    reproduces its own context bit for bit."""
    import paper_2609_23057_amd as P
    specs = [W.spec("beam512", nx=40, ny=36, phase=TABLE),
             W.spec("beam512", nx=33, ny=30, n_zen=2, n_az=8)]
    probs = [P.make_problem(**dict(s, precision="bf16")) for s in specs]
    batch = P.Batch(probs)
    meds = []
    for ch, s in zip(batch.channels, specs):
        med = W.medium(s)
        t = [to_dev(med[k], ch) for k in ("tau", "albedo", "emis")]
        ch.set_medium(*t, med["jprof"], med["inflow"])
        ch._tensors = t
        meds.append(med)
    S0 = [to_dev(W.initial_state(s, "random"), ch) for s, ch in zip(specs, batch.channels)]
    states = [s.clone() for s in S0]
    batch.run(states, 9)
    for i, s in enumerate(specs):
        single, _, _ = build(s, "bf16", meds[i])
        S = S0[i].clone()
        single.run(S, 9)
        torch.cuda.synchronize()
        assert torch.equal(S, states[i]), i
