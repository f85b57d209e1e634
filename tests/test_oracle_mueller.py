"""Pins of the oracle's tabulated scattering matrices (general Mueller
matrices with P12, P34 != 0, the full-Mueller representation named as future
work in the paper's conclusions), against what does not depend on it:

  * Jones calculus: for a particle with amplitude functions S1, S2 the pair
    matrix of Eq. 13 (rotation, scattering-plane matrix, rotation) must equal
    the Mueller matrix of the Jones matrix obtained by projecting the field
    onto the scattering-plane axes and back onto the meridian axes;
  * a table of Rayleigh values reproduces the Rayleigh collision matrix (whose
    own pins are the printed DOP values) to the interpolation error bound;
  * piecewise-linear tables are interpolated exactly;
  * reciprocity Z(-k_in <- -k_out) = D Z(k_out <- k_in)^T D, D = diag(1,1,-1,1);
  * Stokes physicality of a run and intensity conservation.
"""
import numpy as np
import pytest

import workloads as W
from oracle import directions as OD
from oracle import lbm as OL
from oracle import phase as OP

# Stokes vector from the coherency vector (E1 E1*, E1 E2*, E2 E1*, E2 E2*):
# I = |E1|^2 + |E2|^2, Q = |E1|^2 - |E2|^2, U = 2 Re(E1 E2*), V = 2 Im(E1 E2*)
A_STOKES = np.array([[1, 0, 0, 1], [1, 0, 0, -1], [0, 1, 1, 0], [0, -1j, 1j, 0]], dtype=complex)


def jones_to_mueller(J):
    M = A_STOKES @ np.kron(J, J.conj()) @ np.linalg.inv(A_STOKES)
    assert np.abs(M.imag).max() < 1e-12
    return M.real


def amplitudes(cos_t):
    """A synthetic particle: S2 = S1 forward, S2 = -S1 backward."""
    t = np.arccos(np.clip(cos_t, -1.0, 1.0))
    e = 1.0 + 0.8 * np.cos(t) + 0.3 * np.cos(t) ** 2
    S1 = np.sqrt(e) * np.exp(0.7j * np.sin(t))
    S2 = np.sqrt(e) * (0.2 + 0.8 * np.cos(t) ** 2) * np.exp(1j * (0.4 * np.sin(t) + np.pi * np.sin(t / 2) ** 2))
    return S1, S2


def reduced_from_amplitudes(cos_t):
    S1, S2 = amplitudes(cos_t)
    a1 = 0.5 * (abs(S1) ** 2 + abs(S2) ** 2)
    b1 = 0.5 * (abs(S2) ** 2 - abs(S1) ** 2)
    z = S2 * np.conj(S1)
    return np.array([[a1, b1, 0, 0], [b1, a1, 0, 0], [0, 0, z.real, -z.imag], [0, 0, z.imag, z.real]])


def test_table_pair_matrix_equals_jones_calculus():
    dirs = OD.make_directions(3, 5, az_offset_deg=10.0)
    worst = 0.0
    for do in range(dirs.n):
        for di in range(dirs.n):
            ki, ko = dirs.k[di], dirs.k[do]
            nrm = np.cross(ki, ko)
            if np.linalg.norm(nrm) < 1e-9:
                continue
            nrm /= np.linalg.norm(nrm)
            epi, epo = np.cross(nrm, ki), np.cross(nrm, ko)
            # meridian components -> scattering-plane (par, perp) components, and back
            Bin = np.array([[epi @ dirs.e_theta[di], epi @ dirs.e_phi[di]],
                            [nrm @ dirs.e_theta[di], nrm @ dirs.e_phi[di]]])
            Bout = np.array([[dirs.e_theta[do] @ epo, dirs.e_theta[do] @ nrm],
                             [dirs.e_phi[do] @ epo, dirs.e_phi[do] @ nrm]])
            c = float(ko @ ki)
            S1, S2 = amplitudes(c)
            Zj = jones_to_mueller(Bout @ np.diag([S2, S1]) @ Bin)
            Z = OP.pair_matrix(dirs, do, di, reduced_from_amplitudes)
            worst = max(worst, np.abs(Z - Zj).max())
            # Rayleigh: the same projections give the dipole field projection
            Jr = Bout @ np.diag([c, 1.0]) @ Bin
            dip = np.array([[dirs.e_theta[do] @ dirs.e_theta[di], dirs.e_theta[do] @ dirs.e_phi[di]],
                            [dirs.e_phi[do] @ dirs.e_theta[di], dirs.e_phi[do] @ dirs.e_phi[di]]])
            assert np.abs(Jr - dip).max() < 1e-12
    assert worst < 1e-12, worst


def rayleigh_table(step_deg):
    th = np.arange(0.0, 180.0 + 1e-9, step_deg)
    c = np.cos(np.radians(th))
    a = 0.5 * (1 + c * c)
    return np.stack([th, a, a, c, c, -0.5 * (1 - c * c), 0 * c], axis=1)


@pytest.mark.parametrize("grid", [(2, 4, 0.0), (4, 8, 0.0), (3, 5, 22.5)])
def test_table_of_rayleigh_values_reproduces_rayleigh_matrix(grid):
    dirs = OD.make_directions(grid[0], grid[1], az_offset_deg=grid[2])
    M = OP.collision_matrix(dirs, "rayleigh")
    Mt = OP.collision_matrix(dirs, "table", table=rayleigh_table(0.25))
    # linear interpolation error <= h^2/8 max|f''| with h = 0.25 deg
    assert np.abs(Mt - M).max() < 1e-5
    Mc = OP.collision_matrix(dirs, "table", table=rayleigh_table(15.0))
    assert np.abs(Mc - M).max() > 1e-4   # a coarse table is visibly off: the table is used


def test_piecewise_linear_table_is_interpolated_exactly():
    def rows(step):
        th = np.arange(0.0, 180.0 + 1e-9, step)
        a1 = 2.0 - th / 180.0
        a2 = np.ones_like(th)
        a3 = 1.0 - 2.0 * th / 180.0
        a4 = 0.5 + 0.2 * th / 180.0
        b1 = np.interp(th, [0, 90, 180], [0.0, -0.3, 0.0])
        b2 = np.interp(th, [0, 60, 120, 180], [0.0, 0.2, 0.1, 0.0])
        return np.stack([th, a1, a2, a3, a4, b1, b2], axis=1)
    dirs = OD.make_directions(3, 6, az_offset_deg=7.0)
    M15 = OP.collision_matrix(dirs, "table", table=rows(15.0))
    M1 = OP.collision_matrix(dirs, "table", table=rows(1.0))
    assert np.abs(M15 - M1).max() < 1e-13
    F = OP.table_reduced(np.cos(np.radians(75.0)), rows(15.0))
    assert F[0, 0] == pytest.approx(2.0 - 75.0 / 180.0, abs=1e-14)
    assert F[2, 3] == pytest.approx(0.2 - 0.1 * 15.0 / 60.0, abs=1e-14)
    assert F[3, 2] == pytest.approx(-F[2, 3], abs=0)
    assert F[0, 1] == F[1, 0] == pytest.approx(-0.3 * 75.0 / 90.0, abs=1e-14)


@pytest.mark.parametrize("kind", ["rayleigh", "table"])
def test_reciprocity(kind):
    dirs = OD.make_directions(4, 8)
    red = None
    if kind == "table":
        tab = OP.check_table(W.scattering_table())
        red = lambda c: OP.table_reduced(c, tab)  # noqa: E731

    def rev(d):
        return int(np.argmin(np.linalg.norm(dirs.k + dirs.k[d], axis=1)))
    D = np.diag([1.0, 1.0, -1.0, 1.0])
    for do in range(dirs.n):
        for di in range(dirs.n):
            Z = OP.pair_matrix(dirs, do, di, red)
            Zr = OP.pair_matrix(dirs, rev(di), rev(do), red)
            degenerate = abs(abs(dirs.k[do] @ dirs.k[di]) - 1.0) < 1e-12
            assert np.abs(Zr - D @ Z.T @ D).max() < (1e-6 if degenerate else 1e-12), (do, di)


def test_table_couples_u_and_v_only_through_b2():
    dirs = OD.make_directions(4, 8)
    tab = W.scattering_table()
    M = OP.collision_matrix(dirs, "table", table=tab)
    n = dirs.n
    V_from_U = M[3::4, 2::4]
    assert np.abs(V_from_U).max() > 1e-3
    tab0 = tab.copy()
    tab0[:, 6] = 0.0
    M0 = OP.collision_matrix(dirs, "table", table=tab0)
    for s in range(3):
        assert np.all(M0[3::4, s::4] == 0.0) and np.all(M0[s::4, 3::4] == 0.0)
    # Eq. 17 normalisation: sum over outgoing directions of the I->I elements is 1
    assert np.allclose(M[0::4, 0::4].sum(axis=0), 1.0, atol=1e-14)
    assert M.shape == (4 * n, 4 * n)


def test_table_run_stays_physical_and_conserves_intensity():
    tab = W.scattering_table()
    spec = W.spec("plain32", nx=12, ny=10, phase={"kind": "table", "table": tab}, n_zen=4, n_az=8,
                  plane="xy")
    med = W.medium(spec)
    med["tau"][:] = 0.3
    med["albedo"][:] = 1.0
    med["emis"][:] = 0.0
    prob = OL.make_problem(spec, med)
    rng = np.random.default_rng(3)
    S0 = np.zeros(prob.shape)
    I0 = rng.uniform(0.5, 1.0, size=S0[:, 0].shape)
    pol = rng.standard_normal(S0[:, 1:].shape)
    pol *= 0.9 * I0[:, None] / np.linalg.norm(pol, axis=1, keepdims=True)
    S0[:, 0], S0[:, 1:] = I0, pol
    S = OL.run(S0, prob, 25)
    I = S[:, 0]
    assert I.min() >= 0.0
    assert np.all(np.linalg.norm(S[:, 1:], axis=1) <= I * (1 + 1e-12) + 1e-15)
    # periodic, no absorption (albedo 1): the Q, U -> I leak of the table's b1
    # moves intensity only through polarised light; with unpolarised input the
    # first step conserves I exactly
    S1 = OL.step(np.stack([I0, 0 * I0, 0 * I0, 0 * I0], axis=1), prob)
    assert S1[:, 0].sum() == pytest.approx(I0.sum(), rel=1e-12)


@pytest.mark.parametrize("bad", ["short", "order", "ends", "a1", "plane0", "plane180", "nan"])
def test_check_table_refusals(bad):
    tab = W.scattering_table()
    if bad == "short":
        tab = tab[:1]
    elif bad == "order":
        tab[[3, 4]] = tab[[4, 3]]
    elif bad == "ends":
        tab = tab[:-1]
    elif bad == "a1":
        tab[50, 1] = 0.0
    elif bad == "plane0":
        tab[0, 6] = 0.01
    elif bad == "plane180":
        tab[-1, 3] = -0.5 * tab[-1, 2]
    else:
        tab[7, 4] = np.nan
    with pytest.raises(ValueError):
        OP.check_table(tab)


# ---- dichroic absorption (polarisation-dependent extinction) --------------

def _dich_problem(eta, albedo=0.0, tau=0.4, n_zen=4, n_az=8, nx=5, ny=4):
    spec = W.spec("plain32", nx=nx, ny=ny, n_zen=n_zen, n_az=n_az, plane="xy")
    med = W.medium(spec)
    med["tau"][:] = tau
    med["albedo"][:] = albedo
    med["emis"][:] = 0.0
    med["eta"] = np.full((ny, nx), eta) if np.isscalar(eta) else eta
    return OL.make_problem(spec, med)


def test_dichroism_closed_form_for_the_two_linear_polarisations():
    """A pure absorber: light polarised along e_theta (Q = I) decays as
    exp(-tau (1 + eta sin^2 theta)), along e_phi (Q = -I) as
    exp(-tau (1 - eta sin^2 theta)); U and V as exp(-tau); unpolarised light
    becomes polarised with DoLP tanh(tau eta sin^2 theta)."""
    tau, eta = 0.4, 0.6
    prob = _dich_problem(eta, tau=tau)
    th = prob.dirs.theta
    w = np.sin(th) ** 2
    for q, sign in ((1.0, 1.0), (-1.0, -1.0)):
        S = np.zeros(prob.shape)
        S[:, 0], S[:, 1] = 1.0, q
        Y = OL.collide(S, prob)
        expect = np.exp(-tau * (1 + sign * eta * w))
        assert np.allclose(Y[:, 0], expect[:, None, None], rtol=1e-14, atol=0)
        assert np.allclose(Y[:, 1], q * expect[:, None, None], rtol=1e-14, atol=0)
    S = np.zeros(prob.shape)
    S[:, 2], S[:, 3] = 0.5, -0.25
    Y = OL.collide(S, prob)
    assert np.allclose(Y[:, 2], 0.5 * np.exp(-tau)) and np.allclose(Y[:, 3], -0.25 * np.exp(-tau))
    assert np.all(Y[:, :2] == 0.0)
    S = np.zeros(prob.shape)
    S[:, 0] = 1.0
    Y = OL.collide(S, prob)
    dolp = np.abs(Y[:, 1]) / Y[:, 0]
    assert np.allclose(dolp, np.tanh(tau * eta * w)[:, None, None], rtol=1e-13, atol=1e-15)
    assert np.all(Y[:, 1] <= 0.0)     # e_theta light is absorbed more for eta > 0


def test_dichroism_equals_matrix_exponential_and_reduces_without_eta():
    """exp(-tau_abs K_d) by scipy's expm, with the scattering share and a
    random field; eta = 0 reproduces the non-dichroic collision (to the
    rounding of forming (I + Q) and (I - Q) and halving their sum)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(5)
    nx, ny = 4, 3
    eta = rng.uniform(-0.9, 0.9, size=(ny, nx))
    prob = _dich_problem(eta, albedo=0.3, tau=0.5, nx=nx, ny=ny)
    S = rng.standard_normal(prob.shape)
    Y = OL.collide(S, prob)
    plain = _dich_problem(0.0, albedo=0.3, tau=0.5, nx=nx, ny=ny)
    plain.eta = None
    X = S.reshape(4 * prob.n, -1)
    tabs = 0.7 * 0.5
    s = 1.0 - 0.3 * 0.5
    Xa = np.empty_like(X)
    for c in range(nx * ny):
        for d in range(prob.n):
            w = np.sin(prob.dirs.theta[d]) ** 2
            K = np.eye(4)
            K[0, 1] = K[1, 0] = eta.reshape(-1)[c] * w
            Xa[4 * d:4 * d + 4, c] = expm(-tabs * K) @ X[4 * d:4 * d + 4, c]
    Yref = s * Xa + (1.0 - s) * (prob.M @ Xa)
    assert np.abs(Y.reshape(Yref.shape) - Yref).max() < 1e-13
    zero = _dich_problem(0.0, albedo=0.3, tau=0.5, nx=nx, ny=ny)
    assert np.abs(OL.collide(S, zero) - OL.collide(S, plain)).max() < 1e-15 * np.abs(S).max() * 4


def test_dichroism_keeps_stokes_physical_and_refuses_bad_eta():
    rng = np.random.default_rng(9)
    prob = _dich_problem(rng.uniform(-0.95, 0.95, size=(6, 7)), albedo=0.5, tau=0.8, nx=7, ny=6)
    S0 = np.zeros(prob.shape)
    I0 = rng.uniform(0.5, 1.0, size=S0[:, 0].shape)
    pol = rng.standard_normal(S0[:, 1:].shape)
    pol *= 0.99 * I0[:, None] / np.linalg.norm(pol, axis=1, keepdims=True)
    S0[:, 0], S0[:, 1:] = I0, pol
    S = OL.run(S0, prob, 10)
    assert np.all(np.linalg.norm(S[:, 1:], axis=1) <= S[:, 0] * (1 + 1e-12))
    for bad in (1.0, -1.2, np.nan):
        with pytest.raises(ValueError):
            _dich_problem(bad)
