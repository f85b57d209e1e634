"""Parity at the full sizes of the measured workloads, in the launch
configuration bench.py times (fused step with checkpoints, adjoint with
square-root checkpointing).

Where the float64 oracle cannot follow a whole run at full size it is used
on what it can compute: every cell for a few steps, sampled cells through
their dependence cone (a window of half-width 2T + 2 around the cell, since
a pull reaches at most two cells per step), and identities that hold at any
horizon (Stokes physicality, checkpoint replay, linearity in the emission).
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import GTOL, assert_close, build, tolerance, to_dev, to_np
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu


def random_state(shape, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    S = np.abs(rng.standard_normal(shape)) * scale
    S[:, 1:] = S[:, 1:] * 0.2 * np.sign(rng.standard_normal(S[:, 1:].shape))
    return S


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_beam512_full_lattice_few_steps(precision):
    spec = W.spec("beam512")
    solver, oprob, med = build(spec, precision)
    S0 = random_state(solver.shape, 21)
    T, K = 3, 2
    S = to_dev(S0, solver)
    ck = solver.checkpoint_buffer(T, K)
    solver.run(S, T, ck, K)
    torch.cuda.synchronize()
    hist = OL.run(S0, oprob, T, keep=True)[1]
    tol = tolerance(precision, oprob)
    assert_close(to_np(S), hist[T], tol, ("S_T", precision))
    assert_close(to_np(ck[1]), hist[2], tol, ("checkpoint 1", precision))
    assert torch.equal(ck[0], to_dev(S0, solver))


def test_beam512_full_horizon_invariants_and_checkpoint_replay():
    spec = W.spec("beam512")
    solver, oprob, med = build(spec, "fp32")
    T = spec["steps"]
    K = 45
    S = solver.empty_state()
    ck = solver.checkpoint_buffer(T, K)
    solver.run(S, T, ck, K)
    torch.cuda.synchronize()
    for field in (S, ck[-1]):
        assert bool(torch.isfinite(field).all())
        I, pol = field[:, 0], field[:, 1:].pow(2).sum(1).sqrt()
        assert float(I.min()) >= 0.0
        assert bool((pol <= I * (1 + 1e-5) + 1e-12).all())
    assert float(S[:, 0].sum()) > 0.0
    # re-running one segment from a checkpoint reproduces the next checkpoint
    for k in (3, 20):
        R = ck[k].clone()
        solver.run(R, K)
        torch.cuda.synchronize()
        assert torch.equal(R, ck[k + 1]), k


def window_oracle(spec, med, S0, cy, cx, T):
    """The oracle on the window of half-width 2T + 2 around (cy, cx): the
    value at the centre after T steps equals the full lattice's."""
    r = 2 * T + 2
    ys, xs = slice(cy - r, cy + r + 1), slice(cx - r, cx + r + 1)
    w = dict(spec)
    w.update(nx=2 * r + 1, ny=2 * r + 1, bc=(1, 1, 1, 1))
    wmed = dict(med)
    for k in ("tau", "albedo", "emis"):
        wmed[k] = med[k][ys, xs]
    wmed["inflow"] = None
    p = OL.make_problem(w, wmed)
    return OL.run(S0[:, :, ys, xs], p, T)[:, :, r, r]


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp16"])
def test_prec1024_sampled_cells_through_their_cone(precision):
    spec = W.spec("prec1024")
    solver, oprob, med = build(spec, precision)
    S0 = random_state(solver.shape, 33)
    T = 3
    S = to_dev(S0, solver)
    solver.run(S, T)
    torch.cuda.synchronize()
    got = to_np(S)
    rng = np.random.default_rng(5)
    r = 2 * T + 2
    cells = [(int(rng.integers(r, spec["ny"] - r)), int(rng.integers(r, spec["nx"] - r))) for _ in range(8)]
    ref = np.stack([window_oracle(spec, med, S0, cy, cx, T) for cy, cx in cells], axis=-1)
    out = np.stack([got[:, :, cy, cx] for cy, cx in cells], axis=-1)
    assert_close(out, ref, tolerance(precision, oprob), ("prec1024", precision, cells))


def test_adjoint256_full_lattice_gradients():
    spec = W.spec("adjoint256")
    solver, oprob, med = build(spec, "fp32")
    T, K = 6, 3
    S0 = np.zeros(solver.shape)
    S = solver.empty_state()
    ck = solver.checkpoint_buffer(T, K)
    solver.run(S, T, ck, K)
    ST = OL.run(S0, oprob, T)
    _, g = OL.edge_loss(ST, oprob, 3)
    lam = solver.readout_adjoint(3, to_dev(g, solver))
    g_tau, g_alb, g_em = solver.adjoint(T, ck, K, lam)
    torch.cuda.synchronize()
    ref = OA.adjoint(S0, oprob, T, OL.readout_transpose(g, oprob, 3))
    for got, key in ((g_tau, "g_tau"), (g_alb, "g_albedo"), (g_em, "g_emis")):
        err = np.abs(to_np(got) - ref[key]).max() / max(np.abs(ref[key]).max(), 1e-300)
        assert err < GTOL["fp32"], (key, err)
    # float64 central differences of the oracle's loss at a few cells near the top edge
    ny = spec["ny"]
    # (the error is normalised by the field's largest gradient, as above)
    for which, got, cell in (("tau", g_tau, (ny - 2, 100)), ("albedo", g_alb, (ny - 3, 31)),
                             ("emis", g_em, (ny - 2, 200)), ("tau", g_tau, (ny - 4, 7))):
        fd = OA.central_difference(oprob, S0, T, 3, which, cell)
        v = float(to_np(got)[cell])
        scale = np.abs(ref["g_" + which]).max()
        assert abs(v - fd) <= GTOL["fp32"] * scale, (which, cell, v, fd)


def test_adjoint256_full_horizon_emission_gradient_is_exact_for_a_linear_loss():
    """S_T is affine in the emission amplitude and the loss sum_top-row I is
    linear, so dL = <dL/d eps, d eps> exactly for any perturbation."""
    spec = W.spec("adjoint256")
    solver, oprob, med = build(spec, "fp32")
    T = spec["steps"]
    K = int(np.ceil(np.sqrt(T)))
    outd = OL.outgoing_directions(oprob, 3)

    def loss(emis):
        solver.set_medium(solver._tensors[0], solver._tensors[1], emis, med["jprof"], med["inflow"])
        S = solver.empty_state()
        ck = solver.checkpoint_buffer(T, K)
        solver.run(S, T, ck, K)
        out = solver.readout(S, 3)
        return float(to_np(out)[..., 0].sum()), ck

    em0 = solver._tensors[2]
    L0, ck = loss(em0)
    gout = torch.zeros((solver.nx, len(outd), 4), device=solver.device)
    gout[..., 0] = 1.0
    lam = solver.readout_adjoint(3, gout)
    _, _, g_em = solver.adjoint(T, ck, K, lam)
    delta = to_dev(np.random.default_rng(9).uniform(0.0, 0.05, (spec["ny"], spec["nx"])), solver)
    L1, _ = loss(em0 + delta)
    pred = float((g_em.double() * delta.double()).sum())
    assert abs((L1 - L0) - pred) <= 1e-4 * abs(L1 - L0), (L1 - L0, pred)
