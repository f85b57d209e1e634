"""CPU pins of the statevector emulation of the paper's circuit (oracle side).

The emulation must reproduce the classical step (Sec. 3.2.3: the quantum and
classical solvers agree to double-precision round-off, Tables 1-2), every
stage must be unitary on the whole register (ancillas included), and the
post-selected block of each stage must be the classical operator it dilates:
O_emis / 2 (Eq. 7-8), the absorption amplitude (Eq. 9-10), the survival +
redistribution combination (Eq. 12, 30-31) and the bilinear pull (Eq. 37-38).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lbm as OL
from oracle import statevector as SV


def _setup(**over):
    spec = W.spec("qlbm16", **over)
    med = W.medium(spec)
    return spec, med, OL.make_problem(spec, med)


SMALL = [
    dict(nx=4, ny=4, n_zen=2, n_az=2, plane="xy"),                              # fractional shifts, absorbing
    dict(nx=4, ny=2, n_zen=1, n_az=4, zen_rule="explicit", zen_explicit_deg=[75.0],
         plane="xy", bc=(0, 0, 0, 0)),                                         # periodic
    dict(nx=2, ny=4, n_zen=2, n_az=2, plane="xy_d2q9", az_offset_deg=45.0),    # D2Q9 diagonals
    dict(nx=4, ny=4, n_zen=1, n_az=3, zen_rule="explicit", zen_explicit_deg=[60.0],
         plane="xy", bc=(0, 0, 1, 1)),                                         # n = 3 padded to 4
]


@pytest.mark.parametrize("over", SMALL, ids=["xy-abs", "periodic", "d2q9-diag", "n3-mixed"])
def test_emulated_step_equals_classical_step(over):
    spec, med, prob = _setup(**over)
    S0 = W.initial_state(spec, "random")
    em = SV.Emulator(prob)
    S1, p = em.step(S0)
    ref = OL.step(S0, prob)
    assert np.abs(S1 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert 0.0 < p < 1.0


def test_paper_source_four_steps_natural_and_linear_light():
    """The paper's experiment (box source, J = 1, k_ext = 2.5, k_scat = 0.5,
    dt = 1/16, absorbing edges, D2Q9) on a 4 x 2 lattice with 2 x 4
    directions, 4 steps (natural light; 1 step linear) from S = 0 with
    re-encoding: I and the DOP map agree
    with the classical solver to round-off (Tables 1-2 report 1e-13 .. 1e-15)."""
    for pol, steps in (("natural", 4), ("linear", 1)):
        spec, med, prob = _setup(nx=4, ny=2, source_pol=pol)
        S0 = W.initial_state(spec, "zero")
        S, probs = SV.run(S0, prob, steps)
        ref = OL.run(S0, prob, steps)
        assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max()
        Iq, Dq = OL.maps(S)
        Ic, Dc = OL.maps(ref)
        assert np.abs(Iq - Ic).max() <= 1e-13 * np.abs(Ic).max()
        assert np.abs(Dq - Dc).max() <= 1e-12
        assert len(probs) == steps and all(0.0 < p < 1.0 for p in probs)


def _random_state(em, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal((2,) * em.L.nq)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("stage", ["emission", "absorption", "scattering", "streaming"])
def test_every_stage_is_unitary_on_the_whole_register(stage):
    """Norms and inner products of random states over all qubits (ancillas
    included, not only the |0> sector) are preserved."""
    _, _, prob = _setup(nx=4, ny=2, n_zen=1, n_az=4, zen_rule="explicit", zen_explicit_deg=[75.0],
                        plane="xy")
    em = SV.Emulator(prob)
    a, b = _random_state(em, 1), _random_state(em, 2)
    ip = float(np.sum(a * b))
    fa, fb = a.copy(), b.copy()
    getattr(em, stage)(fa)
    getattr(em, stage)(fb)
    assert abs(np.linalg.norm(fa) - 1.0) < 1e-13
    assert abs(np.linalg.norm(fb) - 1.0) < 1e-13
    assert abs(float(np.sum(fa * fb)) - ip) < 1e-13


def _block(em, stage, data):
    """Post-selected image of a data-register vector through one stage."""
    psi = np.zeros((2,) * em.L.nq)
    psi.reshape(-1)[:data.size] = data.reshape(-1)
    getattr(em, stage)(psi)
    return psi.reshape(-1)[:data.size].reshape(data.shape)


def test_stage_blocks_are_the_classical_operators():
    _, _, prob = _setup(nx=4, ny=2, n_zen=1, n_az=4, zen_rule="explicit", zen_explicit_deg=[75.0],
                        plane="xy")
    em = SV.Emulator(prob)
    L = em.L
    rng = np.random.default_rng(3)
    n, nd, ny, nx = prob.n, L.nd, prob.ny, prob.nx
    data = np.zeros((4, 2, nd, nd, ny, nx))
    dd = np.arange(n)
    S = rng.standard_normal((4, n, ny, nx))
    J = rng.standard_normal((4, n, ny, nx))
    data[:, 0, dd, dd] = S
    data[:, 1, dd, dd] = J
    # emission: [[1, 1], [0, 1]] / 2 on (live, source) (Eq. 6-8)
    out = _block(em, "emission", data)
    assert np.allclose(out[:, 0, dd, dd], (S + J) / 2.0, atol=1e-15)
    assert np.allclose(out[:, 1, dd, dd], J / 2.0, atol=1e-15)
    # absorption: a(c) on the live sector only (Eq. 9-10)
    out = _block(em, "absorption", data)
    assert np.allclose(out[:, 0, dd, dd], em.a_abs[None, None] * S, atol=1e-15)
    assert np.allclose(out[:, 1], data[:, 1], atol=1e-15)
    # scattering: (s I + (1 - s) M) / (2 - s), summed over d_in per d_out
    out = _block(em, "scattering", data)
    got = out[:, 0].sum(axis=1)[:, :n]                                   # [st, k, y, x]
    X = np.transpose(S, (1, 0, 2, 3)).reshape(4 * n, ny * nx)
    s = em.s_surv.reshape(1, -1)
    want = ((s * X + (1.0 - s) * (prob.M @ X)) / (2.0 - s)).reshape(n, 4, ny, nx)
    assert np.allclose(np.transpose(got, (1, 0, 2, 3)), want, atol=1e-14)
    assert np.allclose(out[:, 1], data[:, 1], atol=1e-15)
    # streaming: the bilinear pull with the lattice's edges (Eq. 34, 37-38)
    data2 = np.zeros_like(data)
    data2[:, 0, 0, dd] = S                                               # live field at d_out
    out = _block(em, "streaming", data2)
    got = np.transpose(out[:, 0, 0, :n], (1, 0, 2, 3))
    assert np.allclose(got, OL.stream(np.transpose(S, (1, 0, 2, 3)), prob), atol=1e-14)


def test_plausible_mistakes_fail():
    """On a grid whose scattering planes are not meridian planes (2 zeniths x
    3 azimuths), each of these mistakes moves the result far beyond
    round-off: the frame rotations' sign, sigma_in and sigma_out exchanged,
    the weights transposed (w(d_in <- k) for w(k <- d_in)), and the
    eigenvalues of the I +- Q modes exchanged."""
    spec, med, prob = _setup(nx=4, ny=2, n_zen=2, n_az=3, zen_rule="explicit", zen_explicit_deg=[50.0, 110.0],
                             plane="xy")
    S0 = W.initial_state(spec, "random")
    ref = OL.step(S0, prob)

    def neg(e):
        e.sig_in, e.sig_out = -e.sig_in, -e.sig_out

    def swap(e):
        e.sig_in, e.sig_out = e.sig_out.copy(), e.sig_in.copy()

    def transpose(e):
        e.w = e.w.T.copy()

    def modes(e):
        e.lam[..., 0], e.lam[..., 1] = e.lam[..., 1].copy(), e.lam[..., 0].copy()
    for mistake in (neg, swap, transpose, modes):
        em = SV.Emulator(prob)
        mistake(em)
        bad, _ = em.step(S0)
        assert np.abs(bad - ref).max() > 1e-4 * np.abs(ref).max(), mistake.__name__


def test_layout_counts_29_qubits_for_the_paper_lattice():
    """16 x 16 lattice, n = 8: 17 data qubits (st 2, sl 1, d_in 3, d_out 3,
    y 4, x 4) and 12 ancillas, the 29 qubits the paper reports."""
    L = SV.Layout(16, 16, 8)
    assert L.ndata == 17 and L.nq == 29


def test_refusals():
    with pytest.raises(ValueError):
        SV.Layout(6, 4, 8)
    spec, med, prob = _setup(nx=4, ny=4, bc=(1, 1, 1, 2))
    with pytest.raises(ValueError):
        SV.Emulator(prob)
    spec = W.spec("qlbm16", nx=4, ny=4, phase={"kind": "table", "table": W.scattering_table()})
    prob = OL.make_problem(spec, W.medium(spec))
    with pytest.raises(ValueError):
        SV.Emulator(prob)


def test_success_probability_is_the_post_selected_norm():
    spec, med, prob = _setup(nx=4, ny=2, n_zen=1, n_az=4, zen_rule="explicit", zen_explicit_deg=[75.0],
                             plane="xy")
    S0 = W.initial_state(spec, "random")
    em = SV.Emulator(prob)
    S1, p = em.step(S0)
    psi, norm = em.encode(S0)
    for st in ("emission", "absorption", "scattering", "streaming"):
        getattr(em, st)(psi)
    block, p2 = em.post_select(psi)
    assert p == p2 and math.isclose(float(np.sum(block ** 2)), p, rel_tol=1e-14)
