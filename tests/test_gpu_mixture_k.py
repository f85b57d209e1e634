"""GPU parity of per-cell mixtures of K phase functions against the FP64
oracle, through rt_set_phase_mixture_k.

The scattered part of the collision is beta ((1 - sum_j f_j) M X + sum_j
f_j M_j X) with per-cell fractions f_j >= 0, sum_j f_j <= 1 (the aerosol and
cloud mixtures the conclusion, Sec. 4, names as the next step, with more than
two components).  Each further matrix M_j is built as M is (Eq. 17 weights
times the rotated Rayleigh Mueller matrices, Sec. 2.1.5) and contracted on
the matrix cores in the context's precision (the plain path: on the vector
ALUs); the products are summed per cell at their fractions.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import assert_close, build, gtolerance, to_dev, to_np, tolerance
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

MIX3 = [{"kind": "rayleigh"}, {"kind": "hg", "g": -0.3}]
MIX4 = [{"kind": "rayleigh"}, {"kind": "hg", "g": -0.3}, {"kind": "mix", "g": 0.5, "mix_ray": 0.4}]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_mixture(spec, precision, medium=None):
    solver, oprob, med = build(spec, precision, medium)
    frac = to_dev(med["frac"], solver)
    solver.set_phase_mixture(spec["mixture"], frac)
    solver._frac = frac
    return solver, oprob, med


CASES = [
    # workload, overrides (further phase functions in "mixture"), steps, init
    ("beam512", dict(nx=70, ny=37, mixture=MIX3), 40, "zero"),                               # n = 32
    ("beam512", dict(nx=33, ny=29, n_zen=2, n_az=8, mixture=MIX4), 40, "random"),           # n = 16
    ("beam512", dict(nx=21, ny=26, n_zen=4, n_az=16, mixture=MIX4), 25, "random"),          # n = 64
    ("prec1024", dict(nx=19, ny=22, mixture=MIX3), 15, "random"),                           # n = 128
    ("plain32", dict(nx=45, ny=23, mixture=MIX4), 40, "random"),                            # n = 8
]


@pytest.mark.parametrize("precision", ["fp32", "bf16", "plain", "bf16x3", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-n%d-K%d" % (
    c[0], c[1]["nx"], c[1]["ny"], W.ndir(W.spec(c[0], **c[1])), len(c[1]["mixture"]) + 1))
def test_k_mixture_forward_parity(case, precision):
    """Against the unmodified oracle in every precision, at the tolerance of
    the two-phase mixture (the operand rounding of each product is weighted
    by its fraction, so the bound does not grow with K)."""
    name, over, steps, init = case
    spec = W.spec(name, **over)
    solver, oprob, _ = _with_mixture(spec, precision)
    assert len(oprob.mix_M) == len(over["mixture"])
    S0 = W.initial_state(spec, init)
    S = to_dev(S0, solver)
    solver.run(S, steps)
    ref = OL.run(S0, oprob, steps)
    e = assert_close(to_np(S), ref, tolerance(precision, oprob, steps), (name, precision))
    print(name, precision, e)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp16"])
def test_k_mixture_step_and_checkpoints(precision):
    """rt_step with four phase functions equals one oracle step; rt_run's
    checkpoints hold S_{kK} of the mixed medium."""
    spec = W.spec("beam512", nx=50, ny=44, mixture=MIX4)
    solver, oprob, _ = _with_mixture(spec, precision)
    tol = tolerance(precision, oprob)
    S0 = W.initial_state(spec, "random")
    a = to_dev(S0, solver)
    b = solver.empty_state()
    solver.step(a, b)
    assert_close(to_np(b), OL.step(S0, oprob), tol, "step")
    T, K = 17, 4
    ck = solver.checkpoint_buffer(T, K)
    S = to_dev(S0, solver)
    solver.run(S, T, ck, K)
    _, hist = OL.run(S0, oprob, T, keep=True)
    for k in range(ck.shape[0]):
        assert_close(to_np(ck[k]), hist[k * K], tol, ("ckpt", k))
    assert_close(to_np(S), hist[T], tol, "final")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "plain"])
@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_one_hot_fractions_equal_that_phase_function_alone(precision, j):
    """Every cell follows component j alone (j = 0: all fractions zero): the
    blend returns that product itself, so the run equals a context built with
    that phase function as its own, value for value (both pack the matrix the
    same way at n = 32)."""
    spec = W.spec("beam512", nx=37, ny=30, mixture=MIX4)
    med = W.medium(spec)
    solver, _, _ = build(spec, precision, med)
    f = torch.zeros((3, spec["ny"], spec["nx"]), dtype=torch.float32, device=solver.device)
    if j > 0:
        f[j - 1] = 1.0
    solver.set_phase_mixture(spec["mixture"], f)
    own = spec["phase"] if j == 0 else spec["mixture"][j - 1]
    other, oprob2, _ = build(dict(spec, phase=own, mixture=None), precision, med)
    S0 = W.initial_state(spec, "random")
    a, b = to_dev(S0, solver), to_dev(S0, other)
    solver.run(a, 12)
    other.run(b, 12)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert_close(to_np(a), OL.run(S0, oprob2, 12), tolerance(precision, oprob2, 12), "one-hot vs oracle")


def test_two_phase_call_after_a_k_mixture():
    """rt_set_phase_mixture after a four-phase mixture leaves a two-phase
    mixture that matches a fresh two-phase context bit for bit; removing it
    returns to the single-phase run."""
    spec = W.spec("beam512", nx=40, ny=33, mixture=MIX4)
    med = W.medium(spec)
    solver, _, _ = _with_mixture(spec, "fp32", med)
    spec2 = dict(spec, mixture={"kind": "hg", "g": -0.3})
    med2 = dict(med, frac=med["frac"][1].copy())
    fresh, _, _ = _with_mixture(spec2, "fp32", med2)
    f2 = to_dev(med2["frac"], solver)
    solver.set_phase_mixture(spec2["mixture"], f2)
    S0 = W.initial_state(spec, "random")
    a, b = to_dev(S0, solver), to_dev(S0, fresh)
    solver.run(a, 10)
    fresh.run(b, 10)
    single, _, _ = build(dict(spec, mixture=None), "fp32", med)
    c = to_dev(S0, single)
    single.run(c, 10)
    solver.set_phase_mixture(None, None)
    d = to_dev(S0, solver)
    solver.run(d, 10)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(c, d)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("over, T, K", [(dict(nx=36, ny=33), 30, 6),                   # n = 8
                                        (dict(nx=30, ny=27, n_zen=4, n_az=16), 20, 5)],  # n = 64
                         ids=lambda v: str(v))
def test_k_mixture_adjoint_parity(precision, over, T, K):
    """The checkpointed adjoint of a three-phase medium (the adjoint step
    contracts M^T and each M_j^T against the same mu tile) against the oracle
    adjoint for the top-edge (I + DoLP) loss; dropping the last component
    moves the oracle gradient far outside the bound."""
    spec = W.spec("adjoint256", mixture=[{"kind": "hg", "g": -0.4}, {"kind": "rayleigh"}], **over)
    solver, oprob, med = _with_mixture(spec, precision)
    S0 = np.zeros(oprob.shape)
    ck = solver.checkpoint_buffer(T, K)
    S = to_dev(S0, solver)
    solver.run(S, T, ck, K)
    ST = OL.run(S0, oprob, T)
    _, g = OL.edge_loss(ST, oprob, 3)
    lamT = OL.readout_transpose(g, oprob, 3)
    ref = OA.adjoint(S0, oprob, T, lamT)
    got = solver.adjoint(T, ck, K, to_dev(lamT, solver), want_lambda0=True)
    tol = gtolerance(precision, oprob, T)
    for key, arr in zip(("g_tau", "g_albedo", "g_emis", "lambda0"), got):
        assert _rel(to_np(arr), ref[key]) < tol, (key, _rel(to_np(arr), ref[key]))
    two = OL.make_problem(dict(spec, mixture=spec["mixture"][0]), dict(med, frac=med["frac"][0]))
    far = OA.adjoint(S0, two, T, lamT)
    assert _rel(far["g_tau"], ref["g_tau"]) > 10 * tol


def test_k_mixture_refusals():
    import paper_2609_23057_amd as P
    spec = W.spec("beam512", nx=20, ny=18, mixture=MIX3)
    med = W.medium(spec)
    solver, _, _ = build(spec, "fp32", med)     # holds two further phase functions
    S0 = to_dev(W.initial_state(spec, "random"), solver)
    ref = S0.clone()
    solver.run(ref, 5)
    ok = torch.full((2, 18, 20), 0.4, dtype=torch.float32, device=solver.device)
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(MIX4, torch.full((3, 18, 20), 0.2, device=solver.device))
    assert ei.value.status == P.RT_EINVAL        # more than mix_max
    bad = ok.clone()
    bad[1, 3, 4] = 0.7                           # 0.4 + 0.7 > 1
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(MIX3, bad)
    assert ei.value.status == P.RT_ERANGE
    bad = ok.clone()
    bad[0, 5, 6] = -1e-3
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(MIX3, bad)
    assert ei.value.status == P.RT_ERANGE
    bad[0, 5, 6] = float("inf")
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(MIX3, bad)
    assert ei.value.status == P.RT_ERANGE
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture([{"kind": "rayleigh"}, {"kind": "hg", "g": 1.2}], ok)
    assert ei.value.status == P.RT_EINVAL
    with pytest.raises(ValueError):
        solver.set_phase_mixture(MIX3, ok[0])    # one plane for two components
    S = S0.clone()
    solver.run(S, 5)      # a refused mixture leaves the context single-phase
    torch.cuda.synchronize()
    assert torch.equal(S, ref)
    # a mixture and dichroic absorption exclude each other
    solver.set_dichroism(to_dev(np.full((18, 20), 0.3), solver))
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(MIX3, ok)
    assert ei.value.status == P.RT_EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_k_mixture_full_size_beam512(precision):
    """The full 512 x 512, n = 32 lattice with four phase functions, in the
    checkpointed launch of the bench: every cell for three steps against the
    oracle."""
    spec = W.spec("beam512", mixture=MIX4)
    solver, oprob, _ = _with_mixture(spec, precision)
    rng = np.random.default_rng(37)
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


MIX8 = [{"kind": "rayleigh"}, {"kind": "hg", "g": -0.3}, {"kind": "mix", "g": 0.5, "mix_ray": 0.4},
        {"kind": "hg", "g": 0.2}, {"kind": "hg", "g": -0.6}, {"kind": "mix", "g": -0.2, "mix_ray": 0.7},
        {"kind": "hg", "g": 0.4}]


@pytest.mark.parametrize("precision", ["fp32", "bf16", "plain"])
def test_largest_mixture_eight_phase_functions(precision):
    """K = 8 (RT_MIX_MAX = 7 further phase functions), n = 16 and n = 64,
    against the oracle; the workspace holds exactly seven components."""
    import paper_2609_23057_amd._abi as A
    assert A.RT_MIX_MAX == len(MIX8)
    for over in (dict(nx=29, ny=23, n_zen=2, n_az=8), dict(nx=21, ny=17, n_zen=4, n_az=16)):
        spec = W.spec("beam512", mixture=MIX8, **over)
        solver, oprob, _ = _with_mixture(spec, precision)
        assert len(oprob.mix_M) == 7
        S0 = W.initial_state(spec, "random")
        S = to_dev(S0, solver)
        solver.run(S, 12)
        assert_close(to_np(S), OL.run(S0, oprob, 12), tolerance(precision, oprob, 12), (precision, over))


def test_fp16_range_refusal_of_one_component():
    """fp16 packs every further matrix at the first one's scale: one strongly
    forward-peaked component among acceptable ones is refused (RT_ERANGE) and
    leaves the context without a mixture."""
    import paper_2609_23057_amd as P
    mix = [{"kind": "rayleigh"}, {"kind": "hg", "g": 0.95}]
    spec = W.spec("prec1024", nx=20, ny=18, phase={"kind": "hg", "g": 0.0}, mixture=mix)
    solver, _, med = build(spec, "fp16")
    S0 = to_dev(W.initial_state(spec, "random"), solver)
    ref = S0.clone()
    solver.run(ref, 3)
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(mix, to_dev(med["frac"], solver))
    assert ei.value.status == P.RT_ERANGE
    S = S0.clone()
    solver.run(S, 3)
    torch.cuda.synchronize()
    assert torch.equal(S, ref)
    solver.set_phase_mixture(mix[:1], to_dev(med["frac"][:1], solver))   # the acceptable one alone
