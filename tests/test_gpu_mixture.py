"""GPU parity of the per-cell phase-function mixture against the FP64 oracle.

A per-cell fraction f of the scattering follows a second phase function:
Y = alpha X + beta ((1 - f) M X + f M2 X), with M and M2 each built as the
Eq. 17 weights times the rotated Rayleigh Mueller matrices (Sec. 2.1.5).
The fused steps (fp32, bf16, bf16x3 with the high and low parts of both
matrices, fp16 with the second matrix at the first one's power-of-two
scale) contract both matrices on the matrix cores and blend the two
products per cell; the plain float32 path does the same on the vector
ALUs.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import assert_close, build, GTOL, gtolerance, to_dev, to_np, tolerance
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_mixture(spec, precision, medium=None):
    solver, oprob, med = build(spec, precision, medium)
    frac = torch.tensor(np.ascontiguousarray(med["frac"]), dtype=torch.float32, device=solver.device)
    solver.set_phase_mixture(spec["mixture"], frac)
    return solver, oprob, med


CASES = [
    # workload, overrides (second phase function in "mixture"), steps, init
    ("beam512", dict(nx=70, ny=37, mixture={"kind": "rayleigh"}), 40, "zero"),              # n = 32
    ("beam512", dict(nx=33, ny=29, n_zen=2, n_az=8, mixture={"kind": "hg", "g": -0.3}), 40, "random"),
    ("beam512", dict(nx=21, ny=26, n_zen=4, n_az=16,
                     mixture={"kind": "mix", "g": 0.5, "mix_ray": 0.4}), 25, "random"),       # n = 64
    ("prec1024", dict(nx=19, ny=22, mixture={"kind": "hg", "g": 0.2}), 15, "random"),       # n = 128
    ("plain32", dict(nx=45, ny=23, mixture={"kind": "hg", "g": 0.6}), 40, "random"),         # n = 8
]
# (A strongly forward-peaked phase function in this scattering-dominated
# medium, HG g = 0.8 at n = 8, takes bf16 past its 1e-2 bound: the oracle run
# with M rounded to bf16 alone is 2-3% off after 40 steps, so the error is the
# bf16 representation of M, not the kernel; bf16x3 serves such media.)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "plain", "bf16x3", "fp16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-n%d" % (
    c[0], c[1]["nx"], c[1]["ny"], W.ndir(W.spec(c[0], **c[1]))))
def test_mixture_forward_parity(case, precision):
    """Against the unmodified oracle in every precision (the n = 8 medium is
    scattering-dominated: the tolerance there is the accumulation bound of
    the operand rounding, gpu_common.tolerance)."""
    name, over, steps, init = case
    spec = W.spec(name, **over)
    solver, oprob, _ = _with_mixture(spec, precision)
    assert oprob.M2 is not None
    S0 = W.initial_state(spec, init)
    S = to_dev(S0, solver)
    solver.run(S, steps)
    ref = OL.run(S0, oprob, steps)
    e = assert_close(to_np(S), ref, tolerance(precision, oprob, steps), (name, precision))
    print(name, precision, e)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp16"])
def test_mixture_step_and_checkpoints(precision):
    """rt_step with a mixture equals one oracle step; rt_run's checkpoints
    hold S_{kK} of the mixed medium."""
    spec = W.spec("beam512", nx=50, ny=44, mixture={"kind": "hg", "g": -0.5})
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


@pytest.mark.parametrize("precision", ["fp32", "bf16", "plain", "bf16x3", "fp16"])
@pytest.mark.parametrize("n_zen, n_az", [(4, 8), (8, 16)])
def test_zero_fraction_equals_single_phase(precision, n_zen, n_az):
    """f = 0 everywhere: the blend returns the first product unchanged, so
    the run equals the single-phase run value for value; removing the
    mixture returns to the single-phase kernels.  (bf16 at n = 128 is the
    exception: its single-phase kernel keeps X as bf16 high + low parts,
    exact to 2^-18, where the mixture kernel keeps X in float32.)"""
    spec = W.spec("beam512", nx=40, ny=33, n_zen=n_zen, n_az=n_az, mixture={"kind": "rayleigh"})
    solver, _, med = build(spec, precision)
    S0 = to_dev(W.initial_state(spec, "random"), solver)
    ref = S0.clone()
    solver.run(ref, 12)
    zero = torch.zeros((spec["ny"], spec["nx"]), dtype=torch.float32, device=solver.device)
    solver.set_phase_mixture(spec["mixture"], zero)
    S = S0.clone()
    solver.run(S, 12)
    torch.cuda.synchronize()
    if precision == "bf16" and n_zen * n_az > 64:
        # X as high + low bf16 parts is exact to 2^-18; the alpha X term passes
        # that on at every one of the 12 steps (alpha ~ 1), and DoLP takes the
        # errors of two components
        assert_close(to_np(S), to_np(ref), 2 * 12 * 2.0 ** -18, "f = 0, split X")
    else:
        assert torch.equal(S, ref)
    one = torch.ones_like(zero)
    solver.set_phase_mixture(spec["mixture"], one)
    S = S0.clone()
    solver.run(S, 12)
    torch.cuda.synchronize()
    assert not torch.equal(S, ref)
    solver.set_phase_mixture(None, None)
    S = S0.clone()
    solver.run(S, 12)
    torch.cuda.synchronize()
    assert torch.equal(S, ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
def test_unit_fraction_equals_second_phase(precision):
    """f = 1 everywhere: the mixed run equals a context built with the second
    phase function alone (the blend 0 p0 + 1 p1 returns p1 itself; the
    three-phase tests also check it value for value)."""
    spec = W.spec("beam512", nx=37, ny=30, mixture={"kind": "hg", "g": 0.3})
    med = W.medium(spec)
    solver, oprob, _ = build(spec, precision, med)
    solver.set_phase_mixture(spec["mixture"], torch.ones((spec["ny"], spec["nx"]), dtype=torch.float32,
                                                         device=solver.device))
    spec2 = dict(spec, phase=spec["mixture"], mixture=None)
    other, oprob2, _ = build(spec2, precision, med)
    S0 = W.initial_state(spec, "random")
    a, b = to_dev(S0, solver), to_dev(S0, other)
    solver.run(a, 20)
    other.run(b, 20)
    ref = OL.run(S0, oprob2, 20)
    tol = tolerance(precision, oprob2)
    assert_close(to_np(a), ref, tol, "mixture f=1 vs oracle of the second phase")
    assert_close(to_np(a), to_np(b), tol, "mixture f=1 vs single second phase")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixture_full_size_beam512(precision):
    """The full 512 x 512, n = 32 lattice in the checkpointed launch: every
    cell for three steps against the oracle."""
    spec = W.spec("beam512", mixture={"kind": "rayleigh"})
    solver, oprob, _ = _with_mixture(spec, precision)
    rng = np.random.default_rng(31)
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


def test_mixture_refusals():
    import paper_2609_23057_amd as P
    spec = W.spec("beam512", nx=20, ny=18, mixture={"kind": "rayleigh"})
    med = W.medium(spec)
    solver, _, _ = build(spec, "fp32", med)
    S0 = to_dev(W.initial_state(spec, "random"), solver)
    ref = S0.clone()
    solver.run(ref, 5)
    bad = torch.full((18, 20), 0.5, dtype=torch.float32, device=solver.device)
    bad[3, 4] = 1.5
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(spec["mixture"], bad)
    assert ei.value.status == P.RT_ERANGE
    bad[3, 4] = float("nan")
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(spec["mixture"], bad)
    assert ei.value.status == P.RT_ERANGE
    S = S0.clone()
    solver.run(S, 5)      # a refused mixture leaves the context single-phase
    torch.cuda.synchronize()
    assert torch.equal(S, ref)
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture({"kind": "hg", "g": 1.5}, torch.zeros_like(bad))
    assert ei.value.status == P.RT_EINVAL



def test_fp16_mixture_range_refusal():
    """fp16 packs the second matrix at the first one's power-of-two scale
    (max |M| scaled into [2^12, 2^13)); a second matrix more than 8 times
    larger would leave the fp16 range, and the call refuses it.  Isotropic
    first phase at n = 128 against a strongly forward-peaked second one."""
    import paper_2609_23057_amd as P
    spec = W.spec("prec1024", nx=20, ny=18, phase={"kind": "hg", "g": 0.0},
                  mixture={"kind": "hg", "g": 0.95})
    solver, oprob, med = build(spec, "fp16")
    ratio = np.abs(oprob.M2).max() / np.abs(oprob.M).max()
    assert ratio > 16.0, ratio
    S0 = to_dev(W.initial_state(spec, "random"), solver)
    ref = S0.clone()
    solver.run(ref, 4)
    with pytest.raises(P.RTError) as ei:
        solver.set_phase_mixture(spec["mixture"], to_dev(med["frac"], solver))
    assert ei.value.status == P.RT_ERANGE
    S = S0.clone()
    solver.run(S, 4)
    torch.cuda.synchronize()
    assert torch.equal(S, ref)
    # the same pair on fp32 and bf16x3 is accepted
    for precision in ("fp32", "bf16x3"):
        other, _, _ = build(spec, precision, med)
        other.set_phase_mixture(spec["mixture"], to_dev(med["frac"], other))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("over, T, K", [(dict(nx=36, ny=33), 30, 6),                   # n = 8
                                        (dict(nx=30, ny=27, n_zen=4, n_az=16), 20, 5),  # n = 64
                                        (dict(nx=20, ny=17, n_zen=8, n_az=16), 9, 9)],  # n = 128
                         ids=lambda v: str(v))
def test_mixture_adjoint_parity(precision, over, T, K):
    """The checkpointed adjoint of a mixed medium (the adjoint step contracts
    M^T and M2^T against the same mu tile and blends them per cell) against
    the oracle adjoint, for the top-edge (I + DoLP) readout loss: tau, albedo
    and emission gradients and lambda_0 to the gradient bound."""
    spec = W.spec("adjoint256", mixture={"kind": "hg", "g": -0.4}, **over)
    solver, oprob, _ = _with_mixture(spec, precision)
    assert oprob.M2 is not None
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
    # the second phase function matters at this bound: the single-phase
    # oracle gradient is far off
    oprob.M2 = None
    far = OA.adjoint(S0, oprob, T, lamT)
    assert _rel(far["g_tau"], ref["g_tau"]) > 10 * gtolerance(precision, oprob, T)


def test_mixture_adjoint_zero_fraction_equals_single_phase():
    """f = 0: the adjoint equals the single-phase adjoint bit for bit."""
    spec = W.spec("adjoint256", nx=30, ny=27, mixture={"kind": "rayleigh"})
    solver, oprob, _ = build(spec, "fp32")
    T, K = 12, 4
    rng = np.random.default_rng(4)
    lamT = to_dev(rng.standard_normal(oprob.shape), solver)
    out = []
    for f in (None, 0.0):
        if f is not None:
            solver.set_phase_mixture(spec["mixture"], torch.zeros((spec["ny"], spec["nx"]),
                                                                  dtype=torch.float32, device=solver.device))
        ck = solver.checkpoint_buffer(T, K)
        S = to_dev(np.zeros(oprob.shape), solver)
        solver.run(S, T, ck, K)
        out.append([t.clone() for t in solver.adjoint(T, ck, K, lamT, want_lambda0=True)])
    torch.cuda.synchronize()
    for a, b in zip(*out):
        assert torch.equal(a, b)
