"""Pins of the FP64 oracle against the paper's printed values, closed forms,
invariants and independent constructions (CPU only).

Each test names the passage it pins and the mistakes it is meant to catch.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import dense as OD
from oracle import directions as ODir
from oracle import lbm as OL
from oracle import phase as OP

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _dop(v):
    """Degree of polarisation of one Stokes vector, by the oracle's dop()
    (so that the printed DOP values and closed forms below pin it too)."""
    a = [np.array([float(x)]) for x in v]
    return float(OL.dop(*a)[0])


def _problem(nx=8, ny=8, n_zen=2, n_az=4, plane="xy", bc=(0, 0, 0, 0), tau=0.3,
             albedo=0.7, emis=None, jprof=None, inflow=None, kind="rayleigh", g=0.0,
             mix=1.0, zen_rule="equal_area", az_offset=0.0, zen_explicit=None, dt=1.0,
             courant=1.0, renorm=False, scalar=False, abs_taylor=False, scat_exp=False,
             fused_taylor=False):
    dirs = ODir.make_directions(n_zen, n_az, zen_rule, az_offset, zen_explicit)
    sh = ODir.displacements(dirs, plane, courant)
    M = OP.collision_matrix(dirs, kind, g, mix, renorm, scalar)
    n = dirs.n
    tau = np.broadcast_to(np.asarray(tau, float), (ny, nx)).copy()
    alb = np.broadcast_to(np.asarray(albedo, float), (ny, nx)).copy()
    em = np.zeros((ny, nx)) if emis is None else np.asarray(emis, float)
    jp = np.zeros((n, 4)) if jprof is None else np.asarray(jprof, float)
    return OL.Problem(nx, ny, dirs, sh, M, dt, bc, tau, alb, em, jp, inflow,
                      abs_taylor, scat_exp, fused_taylor)


# ------------------------------------------------------------------ P1 --

def test_p1_dop_by_scattering_angle_matches_printed_values():
    """Sec. 3.2.2: DOP 0.6000 at 60/120 deg and 9/17 at 75.5/104.5 deg.

    Pins the equal-area zenith reading (60/120 deg) and the frame-rotation
    angles of the RPR sequence (Eq. 13); a wrong rotation angle or a missing
    rotation changes the 75.5/104.5 deg value.
    """
    g = _gold("dop_by_scattering_angle.json")
    dirs = ODir.make_directions(g["grid"]["n_zen"], g["grid"]["n_az"])
    assert np.allclose(np.degrees(np.unique(dirs.theta)), g["grid"]["zenith_deg"])
    M = OP.collision_matrix(dirs)
    d_out = 0
    assert abs(np.degrees(dirs.theta[d_out]) - 60.0) < 1e-12 and dirs.phi[d_out] == 0.0
    groups = {}
    for d_in in range(dirs.n):
        ang = math.degrees(math.acos(np.clip(dirs.k[d_in] @ dirs.k[d_out], -1, 1)))
        groups.setdefault(round(ang, 1), []).append(d_in)
    e_i = np.array([1.0, 0.0, 0.0, 0.0])
    for key, want in g["printed"].items():
        members = groups[float(key)]
        v = sum(M[0:4, 4 * k:4 * k + 4] @ e_i for k in members)
        want = 9.0 / 17.0 if want == "9/17" else want
        assert abs(_dop(v) - want) < 1e-12, (key, _dop(v), want)
    assert abs(9.0 / 17.0 - g["printed_decimals"]["9/17"]) < 5e-5


def test_p1_literal_azimuth_angles_would_fail_the_pin():
    """Eq. 15 as printed (psi = azimuth of each direction) gives 15/17 at 75.5 deg,
    not the printed 9/17: the pin above discriminates the two readings."""
    dirs = ODir.make_directions(2, 4)
    d_out = 0
    v = np.zeros(4)
    for d_in in (1, 3):
        ct = float(dirs.k[d_in] @ dirs.k[d_out])
        Z = (OP.mueller_rotation(dirs.phi[d_out]) @ OP.rayleigh_reduced(ct)
             @ OP.mueller_rotation(dirs.phi[d_in]))
        v += Z @ np.array([1.0, 0, 0, 0]) / Z[0, 0]
    assert abs(_dop(v) - 9.0 / 17.0) > 0.1


# ------------------------------------------------------------ P2 / P3 --

@pytest.mark.parametrize("c", [-1.0, -0.83, -0.25, 0.0, 0.31, 0.5, 0.97, 1.0])
def test_p2_reduced_rayleigh_eigenvalues(c):
    """Sec. 2.1.5: eigenvalues of P~(theta) are {1, cos^2, cos, cos}."""
    ev = np.sort(np.linalg.eigvalsh(OP.rayleigh_reduced(c)))
    assert np.allclose(ev, np.sort([1.0, c * c, c, c]), atol=1e-14)


@pytest.mark.parametrize("grid", [(2, 4, 0.0), (2, 3, 0.0), (2, 4, 22.5), (4, 8, 0.0)])
def test_p3_single_scatter_dop_closed_form(grid):
    """Sec. 3.2.1: single Rayleigh scattering of natural light has DOP
    sin^2/(1+cos^2) (0 forward/backward, 1 at 90 deg), in any frame."""
    dirs = ODir.make_directions(grid[0], grid[1], az_offset_deg=grid[2])
    for do in range(dirs.n):
        for di in range(dirs.n):
            Z = OP.pair_matrix(dirs, do, di)
            c = float(dirs.k[do] @ dirs.k[di])
            v = Z @ np.array([1.0, 0, 0, 0])
            assert abs(v[0] - 0.5 * (1 + c * c)) < 1e-13
            assert abs(_dop(v) - (1 - c * c) / (1 + c * c)) < 1e-12


# ------------------------------------------------------------------ P4 --

def _stokes(E):
    """Stokes of a complex 2-vector E = (E_1, E_2) in its frame."""
    e1, e2 = E
    return np.array([abs(e1) ** 2 + abs(e2) ** 2, abs(e1) ** 2 - abs(e2) ** 2,
                     2 * (e1 * np.conj(e2)).real, -2 * (e1 * np.conj(e2)).imag])


def test_p4_mueller_rotation_from_field_components():
    """Eq. 21-22: R(psi) equals the Stokes transformation obtained by writing a
    field in a frame rotated by psi (e1' = cos psi e1 + sin psi e2)."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        E = rng.normal(size=2) + 1j * rng.normal(size=2)
        psi = rng.uniform(-np.pi, np.pi)
        c, s = math.cos(psi), math.sin(psi)
        E2 = np.array([c * E[0] + s * E[1], -s * E[0] + c * E[1]])
        assert np.allclose(OP.mueller_rotation(psi) @ _stokes(E), _stokes(E2), atol=1e-12)
    assert np.allclose(OP.mueller_rotation(np.pi), np.eye(4), atol=1e-15)
    a, b = 0.3, -1.1
    assert np.allclose(OP.mueller_rotation(a) @ OP.mueller_rotation(b),
                       OP.mueller_rotation(a + b), atol=1e-14)


# ----------------------------------------------------------------- P14 --

GRIDS = [dict(n_zen=2, n_az=4), dict(n_zen=2, n_az=3), dict(n_zen=2, n_az=4, az_offset_deg=22.5),
         dict(n_zen=4, n_az=8), dict(n_zen=8, n_az=16),
         dict(n_zen=4, n_az=2, zen_rule="explicit", zen_explicit_deg=[30, 45, 60, 75])]


@pytest.mark.parametrize("g", GRIDS)
def test_p14_rpr_equals_dipole_field_projection(g):
    """Eq. 13 (RPR) against an independent construction from fields: the
    scattered field of a dipole is the projection (1 - k_out k_out^T) E_in; its
    Stokes vector in the outgoing meridian frame must equal Z @ S_in for every
    ordered pair, including theta = 0 and pi.  Catches wrong rotation angles,
    signs of U and V, and swapped in/out frames.  Tables 1-2 (Sec. 3.2.3) accept 1e-13."""
    dirs = ODir.make_directions(g["n_zen"], g["n_az"], g.get("zen_rule", "equal_area"),
                                g.get("az_offset_deg", 0.0), g.get("zen_explicit_deg"))
    rng = np.random.default_rng(1)
    for do in range(dirs.n):
        ko = dirs.k[do]
        P = np.eye(3) - np.outer(ko, ko)
        for di in range(dirs.n):
            E = rng.normal(size=2) + 1j * rng.normal(size=2)
            E3 = E[0] * dirs.e_theta[di] + E[1] * dirs.e_phi[di]
            Eo3 = P @ E3
            Eo = np.array([dirs.e_theta[do] @ Eo3, dirs.e_phi[do] @ Eo3])
            Z = OP.pair_matrix(dirs, do, di)
            assert np.allclose(Z @ _stokes(E), _stokes(Eo), atol=1e-13 * np.abs(E).sum() ** 2)


@pytest.mark.parametrize("kind,g,mix", [("rayleigh", 0, 1), ("hg", 0.7, 0), ("mix", 0.6, 0.4)])
def test_eq17_weights_column_normalised_and_blocks_reduced(kind, g, mix):
    """Eq. 17: sum over outgoing directions of the weights is 1 for every
    incoming direction; the I->I element of every block is its weight.  A
    transposed (row-normalised) weight matrix fails on non-uniform grids."""
    dirs = ODir.make_directions(4, 8)
    w = OP.weights(dirs, kind, g, mix)
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-14)
    M = OP.collision_matrix(dirs, kind, g, mix)
    assert np.allclose(M[0::4, 0::4], w, atol=1e-15)
    # HG forward peak: weight of the incoming direction itself is the largest
    if kind == "hg":
        assert np.all(np.argmax(w, axis=0) == np.arange(dirs.n))
    # Rayleigh/HG structure: IQU <-> V blocks are exactly zero
    for s_out in range(4):
        for s_in in range(4):
            if (s_out == 3) != (s_in == 3):
                assert np.all(M[s_out::4, s_in::4] == 0.0)


# ------------------------------------------------------------------ P5 --

def test_p5_energy_partition_97_3():
    """Sec. 3.2.1: with k_scat = 0.5 and dt = 1/16 about 97% stays unscattered
    and 3% is redistributed (pins tau_sca = k_scat dt per step and the survival
    factor 1 - tau_sca of Eq. 11)."""
    g = _gold("energy_partition.json")
    tau_sca = g["k_scat"] * g["dt"]
    prob = _problem(nx=4, ny=4, tau=tau_sca, albedo=1.0)
    alpha, beta = prob.alpha[0, 0], prob.beta[0, 0]
    res = g["printed_resolution_percent"]
    assert abs(100 * alpha - g["printed_percent"]["unscattered"]) <= res
    assert abs(100 * beta - g["printed_percent"]["redistributed"]) <= res
    # one collision of a unit pencil: the un-redistributed share is alpha
    S = np.zeros(prob.shape)
    S[0, 0, 1, 1] = 1.0
    Y = OL.collide(S, prob)
    assert abs(Y[:, 0].sum() - 1.0) < 1e-14            # scattering conserves I here
    assert abs(Y[0, 0, 1, 1] - (alpha + beta * prob.M[0, 0])) < 1e-15


# ------------------------------------------------------------------ P6 --

@pytest.mark.parametrize("taylor", [False, True])
@pytest.mark.parametrize("plane,courant", [("xy_d2q9", 1.0), ("xy", 1.0), ("xz", 0.7)])
def test_p6_beer_lambert_pure_absorber(taylor, plane, courant):
    """Sec. 2.1.4: pure absorption multiplies every beam by exp(-k_abs dt) per
    step (Taylor: 1 - k_abs dt); on a periodic lattice streaming only moves it,
    so the lattice total after t steps is I0 exp(-tau t) exactly, any shift."""
    tau = 0.137
    prob = _problem(nx=9, ny=7, n_zen=2, n_az=4, plane=plane, courant=courant, tau=tau,
                    albedo=0.0, abs_taylor=taylor, az_offset=22.5 if plane != "xy_d2q9" else 0.0)
    rng = np.random.default_rng(3)
    S = np.zeros(prob.shape)
    S[2, 0] = rng.uniform(size=(7, 9))
    tot0 = S[2, 0].sum()
    f = (1 - tau) if taylor else math.exp(-tau)
    for t in range(1, 13):
        S = OL.step(S, prob)
        assert abs(S[:, 0].sum() - tot0 * f ** t) < 1e-12 * tot0
        assert np.all(S[[0, 1, 3, 4, 5, 6, 7]] == 0.0)


# ------------------------------------------------------------------ P7 --

@pytest.mark.parametrize("mode", ["scalar", "renorm"])
def test_p7_total_intensity_conserved_without_absorption(mode):
    """Albedo 1, periodic, no source: scattering redistributes and streaming
    moves, so total I is constant (Sec. 2.1.1 normalisation).  Exact for the
    scalar matrix and for the I-row renormalised polarised matrix."""
    prob = _problem(nx=8, ny=6, n_zen=4, n_az=8, plane="xy", tau=0.4, albedo=1.0,
                    kind="hg", g=0.5, scalar=(mode == "scalar"), renorm=(mode == "renorm"))
    S = W.initial_state(dict(nx=8, ny=6, n_zen=4, n_az=8, seed=7), "random")
    tot0 = S[:, 0].sum()
    for _ in range(20):
        S = OL.step(S, prob)
    assert abs(S[:, 0].sum() - tot0) < 1e-12 * tot0


def test_p7_polarised_leak_without_renormalisation():
    """Without the renormalisation the discrete Q,U -> I elements do not sum to
    zero, so polarised light leaks intensity (documented reading, not a bug)."""
    dirs = ODir.make_directions(2, 4)
    M = OP.collision_matrix(dirs)
    leak = np.abs(M[0::4, 1::4].sum(axis=0)).max()
    assert leak > 1e-3
    Mr = OP.collision_matrix(dirs, renorm_irow=True)
    assert np.abs(Mr[0::4, 1::4].sum(axis=0)).max() < 1e-15
    assert np.abs(Mr[0::4, 2::4].sum(axis=0)).max() < 1e-15


# ------------------------------------------------------------------ P8 --

@pytest.mark.parametrize("tau", [0.05, 0.5, 2.0])
def test_p8_kirchhoff_equilibrium(tau):
    """Uniform periodic purely absorbing medium with isotropic unpolarised
    emission j: emission is added before absorption (Eq. 8 then Eq. 10), so
    S_t = dt j a (1 - a^t)/(1 - a) with a = exp(-tau), and the equilibrium is
    dt j / (exp(tau) - 1) = B tau/(exp(tau)-1) for j = B tau / dt (I = B as
    tau -> 0).  Emission added after absorption would give dt j (1-a^t)/(1-a)."""
    jv, dt = 0.8, 0.25
    n = 8
    prob = _problem(nx=5, ny=4, tau=tau, albedo=0.0, emis=np.ones((4, 5)),
                    jprof=np.tile([jv, 0, 0, 0], (n, 1)), dt=dt, plane="xy")
    a = math.exp(-tau)
    S = np.zeros(prob.shape)
    for t in range(1, 40):
        S = OL.step(S, prob)
        want = dt * jv * a * (1 - a ** t) / (1 - a)
        assert np.allclose(S[:, 0], want, rtol=1e-13, atol=0)
        assert np.all(S[:, 1:] == 0)
    S_inf = dt * jv / (math.exp(tau) - 1)
    assert abs(S[0, 0, 0, 0] - S_inf) < 1e-12 + 2 * a ** 39 * S_inf


# ------------------------------------------------------------------ P9 --

@pytest.mark.parametrize("name", ["plain32", "beam512"])
def test_p9_stokes_physicality(name):
    """I^2 >= Q^2 + U^2 + V^2 everywhere, every step: positive combinations of
    pure Rayleigh Mueller matrices, non-negative bilinear weights and s >= 0."""
    s = W.spec(name, nx=12, ny=10)
    med = W.medium(s)
    prob = OL.make_problem(s, med)
    S = W.initial_state(s, "random")
    for _ in range(15):
        S = OL.step(S, prob)
        I = S[:, 0]
        pol2 = S[:, 1] ** 2 + S[:, 2] ** 2 + S[:, 3] ** 2
        assert np.all(I >= 0)
        assert np.all(I * I - pol2 >= -1e-13 * I * I)


# ----------------------------------------------------------------- P10 --

def test_p10_mirror_symmetry():
    """Mirror y -> -y maps direction (theta, phi) to (theta, -phi) and Stokes
    (I,Q,U,V) to (I,Q,-U,-V).  A mirror-symmetric setup (source on row 0 of a
    periodic lattice) must give S(x,-y,phi->-phi) = F S(x,y,phi).  Catches sign
    errors in U/V, in the rotation angles and in the streaming direction."""
    nx = ny = 9
    n_zen, n_az = 2, 8
    emis = np.zeros((ny, nx))
    emis[0, 3] = 1.0
    emis[0, 5] = 0.5
    jp = np.zeros((n_zen * n_az, 4))
    jp[:, 0] = 1.0
    jp[:, 1] = 0.3
    rng = np.random.default_rng(5)
    tau = rng.uniform(0.1, 0.6, size=(ny, nx))
    tau = 0.5 * (tau + tau[(-np.arange(ny)) % ny])
    prob = _problem(nx=nx, ny=ny, n_zen=n_zen, n_az=n_az, plane="xy", courant=0.8,
                    tau=tau, albedo=0.8, emis=emis, jprof=jp)
    S = OL.run(np.zeros(prob.shape), prob, 12)
    phis = prob.dirs.phi
    mir = []
    for d in range(prob.n):
        target = (-phis[d]) % (2 * np.pi)
        cand = [e for e in range(prob.n) if prob.dirs.theta[e] == prob.dirs.theta[d]
                and abs(((phis[e] - target + np.pi) % (2 * np.pi)) - np.pi) < 1e-12]
        mir.append(cand[0])
    F = np.array([1.0, 1.0, -1.0, -1.0])
    ym = (-np.arange(ny)) % ny
    Sm = S[mir][:, :, ym, :] * F[None, :, None, None]
    assert np.abs(Sm - S).max() < 1e-13 * np.abs(S).max()
    assert np.abs(S[:, 2]).max() > 1e-4  # the test is not vacuous


# ----------------------------------------------------------------- P11 --

def test_p11_two_dimensional_lattice_reproduces_d1q2():
    """Sec. 3.1: the 2D solver with Ny = 1 and two horizontal directions equals
    an independent D1Q2 solver (here a plain loop: forward/backward Rayleigh
    weights are equal, 1/2 each) to round-off."""
    nx, T, tau, alb, dt = 32, 40, 0.4, 0.3, 0.5
    em = np.zeros((1, nx))
    em[0, 10:20] = 1.0
    jp = np.array([[0.5, 0, 0, 0], [0.5, 0, 0, 0]])
    prob = _problem(nx=nx, ny=1, n_zen=1, n_az=2, zen_rule="explicit", zen_explicit=[90.0],
                    plane="xy", tau=tau, albedo=alb, emis=em, jprof=jp, dt=dt, scalar=True)
    assert np.allclose(prob.shifts, [[1, 0], [-1, 0]], atol=1e-15)
    S = OL.run(np.zeros(prob.shape), prob, T)
    a = math.exp(-(1 - alb) * tau)
    s = 1 - alb * tau
    R = [0.0] * nx
    L = [0.0] * nx
    for _ in range(T):
        XR = [R[i] + dt * 0.5 * em[0, i] for i in range(nx)]
        XL = [L[i] + dt * 0.5 * em[0, i] for i in range(nx)]
        YR = [a * (s * XR[i] + (1 - s) * 0.5 * (XR[i] + XL[i])) for i in range(nx)]
        YL = [a * (s * XL[i] + (1 - s) * 0.5 * (XR[i] + XL[i])) for i in range(nx)]
        R = [YR[(i - 1) % nx] for i in range(nx)]
        L = [YL[(i + 1) % nx] for i in range(nx)]
    assert np.abs(S[0, 0, 0] - np.array(R)).max() < 1e-15
    assert np.abs(S[1, 0, 0] - np.array(L)).max() < 1e-15


# ------------------------------------------------------------ streaming --

@pytest.mark.parametrize("l", [(0.3, 0.0), (-0.3, 0.55), (1.0, -1.0), (-0.75, -0.2), (0.0, 0.0)])
def test_stream_moves_mass_by_displacement(l):
    """Eq. 34: the bilinear shift moves a blob's centre of mass by exactly l
    per step and keeps its mass (periodic lattice, blob away from the edges)."""
    prob = _problem(nx=20, ny=20, n_zen=1, n_az=1, zen_rule="explicit", zen_explicit=[90.0],
                    plane="xy", tau=0.0, albedo=0.0)
    prob.shifts = np.array([l], dtype=float)
    Y = np.zeros(prob.shape)
    Y[0, 0, 8:11, 7:10] = np.arange(1, 10).reshape(3, 3)
    yy, xx = np.meshgrid(np.arange(20), np.arange(20), indexing="ij")
    m0 = Y[0, 0].sum()
    cx0, cy0 = (Y[0, 0] * xx).sum() / m0, (Y[0, 0] * yy).sum() / m0
    S = OL.stream(Y, prob)
    m1 = S[0, 0].sum()
    assert abs(m1 - m0) < 1e-12
    assert abs((S[0, 0] * xx).sum() / m1 - cx0 - l[0]) < 1e-12
    assert abs((S[0, 0] * yy).sum() / m1 - cy0 - l[1]) < 1e-12
    assert np.all(S >= 0)


def test_absorbing_edge_removes_and_inflow_edge_injects():
    """Sec. 2.1.7: an absorbing edge discards what streams out; an inflow edge
    supplies the prescribed radiance to directions entering through it."""
    n = 8
    inflow = np.zeros((4, n, 4))
    inflow[3, 5, :] = [2.0, 0.5, 0.0, 0.0]
    prob = _problem(nx=6, ny=5, plane="xz", bc=(1, 1, 1, 2), tau=0.0, albedo=0.0,
                    inflow=inflow)
    down = np.nonzero(prob.shifts[:, 1] < 0)[0]
    assert 5 in down
    S = OL.stream(np.zeros(prob.shape), prob)
    ly = prob.shifts[5, 1]
    # top row of direction 5 pulls |ly| from above the lattice -> inflow value
    assert np.allclose(S[5, :, 4, 1:-1].T, -ly * inflow[3, 5], atol=1e-15) or \
        np.allclose(S[5, :, 4, 2:-2].T, -ly * inflow[3, 5], atol=1e-15)
    others = [d for d in range(n) if d != 5]
    assert np.all(S[others] == 0.0)
    # mass leaving through absorbing edges is lost
    Y = np.ones(prob.shape)
    S2 = OL.stream(Y, prob)
    assert S2[:, 0].sum() < Y[:, 0].sum() - 1.0


# ------------------------------------------------------- P14 brute force --

def test_p14_stream_transpose_is_transpose_of_stream():
    """The adjoint's scatter-add (stream_transpose) is the exact transpose of
    the gather (stream), on every edge kind, by building both as matrices."""
    for bc in [(0, 0, 0, 0), (1, 1, 1, 2), (0, 0, 1, 1)]:
        prob = _problem(nx=5, ny=4, n_zen=2, n_az=3, plane="xz", courant=0.9, bc=bc)
        N = int(np.prod(prob.shape))
        zero = OL.stream(np.zeros(prob.shape), prob).ravel()
        L = np.zeros((N, N))
        LT = np.zeros((N, N))
        for j in range(N):
            e = np.zeros(N)
            e[j] = 1.0
            L[:, j] = OL.stream(e.reshape(prob.shape), prob).ravel() - zero
            LT[:, j] = OL.stream_transpose(e.reshape(prob.shape), prob).ravel()
        assert np.abs(L.T - LT).max() < 1e-15


def test_p14_dense_operator_and_multi_step():
    """The T-step oracle equals the affine recursion of its dense one-step
    operator, and the operator is the product of a block-diagonal collision
    (alpha I + beta M per cell, built here independently) and the stream."""
    s = W.spec("beam512", nx=4, ny=3, n_zen=2, n_az=4)
    med = W.medium(s)
    med["emis"][:] = 0.02
    med["jprof"][:, 0] = 1.0
    prob = OL.make_problem(s, med)
    A, b = OD.step_operator(prob)
    S0 = W.initial_state(s, "random")
    x = S0.ravel()
    for _ in range(6):
        x = A @ x + b
    assert np.abs(x - OL.run(S0, prob, 6).ravel()).max() < 1e-13
    # independent block construction of the collision part
    n, C = prob.n, prob.nx * prob.ny
    N = 4 * n * C
    Cm = np.zeros((N, N))
    idx = lambda d, s_, c: (d * 4 + s_) * C + c  # noqa: E731
    for c in range(C):
        yy, xx = divmod(c, prob.nx)
        al, be = prob.alpha[yy, xx], prob.beta[yy, xx]
        for r in range(4 * n):
            for k in range(4 * n):
                Cm[idx(r // 4, r % 4, c), idx(k // 4, k % 4, c)] = \
                    (al if r == k else 0.0) + be * prob.M[r, k]
    zero = OL.stream(np.zeros(prob.shape), prob).ravel()
    L = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        L[:, j] = OL.stream(e.reshape(prob.shape), prob).ravel() - zero
    assert np.abs(A - L @ Cm).max() < 1e-14


# ----------------------------------------------------------------- P15 --

MIX3 = [{"kind": "hg", "g": -0.4}, {"kind": "mix", "g": 0.7, "mix_ray": 0.3}]


def _adj_problem(fused=False, scat_exp=False, abs_taylor=False, mixture=False, dichroism=False):
    """mixture: False, True (one further HG(-0.4) phase) or a list of phases."""
    mix = {"kind": "hg", "g": -0.4} if mixture is True else (mixture or None)
    s = W.spec("adjoint256", nx=10, ny=8, n_zen=2, n_az=4, mixture=mix, dichroism=0.8 if dichroism else None)
    med = W.medium(s)
    med["tau"] = med["tau"] * 10.0
    s["fused_taylor"] = fused
    s["scat_exp"] = scat_exp
    s["abs_taylor"] = abs_taylor
    return s, OL.make_problem(s, med)


@pytest.mark.parametrize("variant", ["split", "fused", "scat_exp", "abs_taylor", "mixture", "mixture3",
                                     "dichroism"])
def test_p15_adjoint_dot_product(variant):
    """<A x, y> = <x, A^T y> for the T-step linear part: the adjoint state
    lambda_0 from lambda_T = y must satisfy <S_T(x) - S_T(0), y> = <x, lambda_0>."""
    s, prob = _adj_problem(variant == "fused", variant == "scat_exp", variant == "abs_taylor",
                           MIX3 if variant == "mixture3" else variant == "mixture", variant == "dichroism")
    if variant == "mixture":
        assert prob.M2 is not None and 0.1 < prob.frac.mean() < 0.9
    if variant == "mixture3":
        assert len(prob.mix_M) == 2 and np.all(prob.mix_f.mean(axis=(1, 2)) > 0.2)
    T = 7
    rng = np.random.default_rng(11)
    x = rng.normal(size=prob.shape)
    y = rng.normal(size=prob.shape)
    z = np.zeros(prob.shape)
    Ax = OL.run(x, prob, T) - OL.run(z, prob, T)
    res = OA.adjoint(z, prob, T, y)
    lhs = float(np.sum(Ax * y))
    rhs = float(np.sum(x * res["lambda0"]))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("variant", ["split", "fused", "scat_exp", "mixture", "mixture3", "dichroism"])
def test_p15_adjoint_gradients_match_central_differences(variant):
    """Gradients of the top-edge (I + DoLP) loss wrt per-cell tau, albedo and
    emission against FP64 central differences on sampled cells (the mixture
    variant: a per-cell HG(-0.4) fraction of the scattering; mixture3: three
    phase functions with Dirichlet fractions)."""
    s, prob = _adj_problem(variant == "fused", variant == "scat_exp",
                           mixture=MIX3 if variant == "mixture3" else variant == "mixture",
                           dichroism=variant == "dichroism")
    if variant == "dichroism":
        assert prob.eta is not None and np.abs(prob.eta).max() > 0.5
    T = 12
    S0 = np.zeros(prob.shape)
    S_T = OL.run(S0, prob, T)
    _, g = OL.edge_loss(S_T, prob, 3)
    lam_T = OL.readout_transpose(g, prob, 3)
    res = OA.adjoint(S0, prob, T, lam_T)
    rng = np.random.default_rng(2)
    for _ in range(6):
        cell = (int(rng.integers(prob.ny)), int(rng.integers(prob.nx)))
        for which, key in (("tau", "g_tau"), ("albedo", "g_albedo"), ("emis", "g_emis")):
            # (the dichroic medium's smallest gradients sit at cells with
            # tau ~ 0.02, where a 1e-5 relative step leaves the difference to
            # the roundoff of the O(1) loss)
            fd = OA.central_difference(prob, S0, T, 3, which, cell, rel_h=1e-4 if variant == "dichroism" else 1e-5)
            ad = res[key][cell]
            assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * np.abs(res[key]).max()) + 1e-12, \
                (which, cell, fd, ad)


def test_edge_loss_gradient_matches_differences():
    """dLoss/dS of the (I + DoLP) readout loss, against central differences."""
    s, prob = _adj_problem()
    S = OL.run(np.zeros(prob.shape), prob, 9)
    _, g = OL.edge_loss(S, prob, 3)
    G = OL.readout_transpose(g, prob, 3)
    rng = np.random.default_rng(4)
    d_up = OL.outgoing_directions(prob, 3)
    for _ in range(10):
        d = int(rng.choice(d_up))
        st = int(rng.integers(3))
        x = int(rng.integers(prob.nx))
        h = 1e-7
        Sp, Sm = S.copy(), S.copy()
        Sp[d, st, prob.ny - 1, x] += h
        Sm[d, st, prob.ny - 1, x] -= h
        fd = (OL.edge_loss(Sp, prob, 3)[0] - OL.edge_loss(Sm, prob, 3)[0]) / (2 * h)
        assert abs(fd - G[d, st, prob.ny - 1, x]) < 1e-6 * max(1.0, abs(fd))


# ----------------------------------------------------------- Table grids --

@pytest.mark.parametrize("g", [dict(n_zen=2, n_az=4), dict(n_zen=2, n_az=4, az_offset_deg=22.5),
                               dict(n_zen=2, n_az=3),
                               dict(n_zen=4, n_az=2, zen_rule="explicit",
                                    zen_explicit_deg=[30, 45, 60, 75])])
@pytest.mark.parametrize("pol", ["natural", "linear"])
def test_table_grids_run_physically(g, pol):
    """Tables 1-2 direction grids (cardinal, 22.5 deg offset, 3 azimuths,
    explicit zeniths) with natural and linear sources: the step keeps Stokes
    vectors physical and conserves I with albedo 1 in scalar mode."""
    n = g["n_zen"] * g["n_az"]
    jp = np.zeros((n, 4))
    jp[:, 0] = 1.0 / n
    if pol == "linear":
        jp[:, 1] = 1.0 / n
    em = np.zeros((8, 8))
    em[3:5, 3:5] = 1.0
    prob = _problem(nx=8, ny=8, n_zen=g["n_zen"], n_az=g["n_az"], plane="xy",
                    zen_rule=g.get("zen_rule", "equal_area"), zen_explicit=g.get("zen_explicit_deg"),
                    az_offset=g.get("az_offset_deg", 0.0), tau=2.5 / 16, albedo=0.2,
                    emis=em, jprof=jp, dt=1 / 16)
    S = np.zeros(prob.shape)
    for _ in range(4):
        S = OL.step(S, prob)
        assert np.all(S[:, 0] ** 2 - (S[:, 1:] ** 2).sum(axis=1) >= -1e-15)
    I_map, dop_map = OL.maps(S)
    assert I_map.max() > 0 and np.all(dop_map <= 1 + 1e-12)


# ------------------------------------------------------------- phase mixture --
# Per-cell mixtures of two phase functions (the aerosol / cloud fractions the
# conclusion, Sec. 4, names as the next step): Y = alpha X + beta ((1 - f) M X
# + f M2 X).  Pinned against the single-phase problems it must reduce to, its
# affine dependence on f, and intensity conservation.

def _with_mixture(p, M2, frac):
    return OL.Problem(p.nx, p.ny, p.dirs, p.shifts, p.M, p.dt, p.bc, p.tau, p.albedo, p.emis, p.jprof,
                      p.inflow_cells, p.abs_taylor, p.scat_exp, p.fused_taylor, M2=M2, frac=frac)


def _mixture_setup(**kw):
    nx, ny = kw.get("nx", 7), kw.get("ny", 6)
    rng = np.random.default_rng(41)
    base = dict(nx=nx, ny=ny, n_zen=2, n_az=8, plane="xy", tau=0.35, albedo=0.8,
                emis=rng.uniform(0.0, 0.1, (ny, nx)), jprof=np.tile([1.0, 0.2, 0.0, 0.0], (16, 1)))
    base.update(kw)
    p_hg = _problem(kind="hg", g=0.6, **base)
    p_ray = _problem(kind="rayleigh", **base)
    S = W.initial_state(dict(nx=nx, ny=ny, n_zen=2, n_az=8, seed=9), "random")
    return p_hg, p_ray, S, rng


def test_mixture_fraction_zero_and_one_reduce_to_each_phase():
    """f = 0 is the main phase function's problem, f = 1 the second's, to the
    bit: catches swapped weights and a missing (1 - f) factor."""
    p_hg, p_ray, S, _ = _mixture_setup()
    zero = _with_mixture(p_hg, p_ray.M, np.zeros((p_hg.ny, p_hg.nx)))
    one = _with_mixture(p_hg, p_ray.M, np.ones((p_hg.ny, p_hg.nx)))
    assert np.array_equal(OL.step(S, zero), OL.step(S, p_hg))
    assert np.array_equal(OL.step(S, one), OL.step(S, p_ray))
    assert not np.allclose(OL.step(S, p_hg), OL.step(S, p_ray))   # the two phases differ


def test_mixture_collision_is_affine_in_the_fraction():
    """Per cell, the collision with fraction f equals (1 - f) times the f = 0
    collision plus f times the f = 1 collision."""
    p_hg, p_ray, S, rng = _mixture_setup()
    f = rng.uniform(0.0, 1.0, (p_hg.ny, p_hg.nx))
    Yf = OL.collide(S, _with_mixture(p_hg, p_ray.M, f))
    Y0 = OL.collide(S, _with_mixture(p_hg, p_ray.M, np.zeros_like(f)))
    Y1 = OL.collide(S, _with_mixture(p_hg, p_ray.M, np.ones_like(f)))
    ref = (1.0 - f) * Y0 + f * Y1
    assert np.abs(Yf - ref).max() < 1e-14 * np.abs(ref).max()


def test_mixture_conserves_total_intensity_without_absorption():
    """Albedo 1, periodic, no source, I-row renormalised matrices: any
    per-cell mixture of two conservative redistributions conserves total I
    (the weights of a cell sum to one)."""
    p_hg, p_ray, S, rng = _mixture_setup(albedo=1.0, renorm=True, emis=None, jprof=None)
    prob = _with_mixture(p_hg, p_ray.M, rng.uniform(0.0, 1.0, (p_hg.ny, p_hg.nx)))
    tot0 = S[:, 0].sum()
    for _ in range(20):
        S = OL.step(S, prob)
    assert abs(S[:, 0].sum() - tot0) < 1e-12 * tot0


def test_mixture_fraction_outside_unit_interval_is_refused():
    p_hg, p_ray, _, _ = _mixture_setup()
    with pytest.raises(ValueError):
        _with_mixture(p_hg, p_ray.M, np.full((p_hg.ny, p_hg.nx), 1.5))


# Mixtures of K phase functions: further matrices M_1 .. M_{K-1} and per-cell
# fractions f_k >= 0, sum_k f_k <= 1, the first matrix taking the rest.  Pinned
# against the single-phase problems (one-hot fractions), the two-phase form,
# convexity, the order and splitting of components, and conservation.

def _k_setup(**kw):
    """Four phase functions on one medium: HG(0.6) (the context's own),
    Rayleigh, HG(-0.5) and a Rayleigh / HG(0.3) mix."""
    p_hg, p_ray, S, rng = _mixture_setup(**kw)
    nx, ny = p_hg.nx, p_hg.ny
    p_back = _with_mixture(p_hg, None, None)
    p_back.M = OP.collision_matrix(p_hg.dirs, "hg", -0.5, 1.0, kw.get("renorm", False), False)
    p_mix = _with_mixture(p_hg, None, None)
    p_mix.M = OP.collision_matrix(p_hg.dirs, "mix", 0.3, 0.5, kw.get("renorm", False), False)
    return [p_hg, p_ray, p_back, p_mix], S, rng, (ny, nx)


def _dirichlet(rng, k, shape):
    e = -np.log1p(-rng.uniform(0.0, 1.0, (k + 1,) + shape))
    return (e / e.sum(axis=0))[1:]


def test_k_mixture_one_hot_cells_take_each_phase_function():
    """Each cell follows one of four phase functions (one-hot fractions): the
    collision there is that phase function's own, to the bit."""
    probs, S, rng, shp = _k_setup()
    pick = rng.integers(0, 4, shp)
    pick[0, :4] = [0, 1, 2, 3]
    f = np.stack([(pick == k).astype(float) for k in (1, 2, 3)])
    mixed = OL.collide(S, _with_mixture(probs[0], [p.M for p in probs[1:]], f))
    for k, p in enumerate(probs):
        own = OL.collide(S, p)
        assert np.array_equal(mixed[..., pick == k], own[..., pick == k]), k
    assert not np.allclose(OL.collide(S, probs[2]), OL.collide(S, probs[3]))


def test_k_mixture_with_one_further_phase_is_the_two_phase_form():
    probs, S, rng, shp = _k_setup()
    f = rng.uniform(0.0, 1.0, shp)
    two = _with_mixture(probs[0], probs[1].M, f)
    listed = _with_mixture(probs[0], [probs[1].M], f[None])
    assert np.array_equal(OL.run(S, two, 3), OL.run(S, listed, 3))


def test_k_mixture_collision_is_the_convex_combination_of_the_phases():
    """Per cell, (1 - sum f_k) times the first phase function's collision plus
    f_k times each further one's."""
    probs, S, rng, shp = _k_setup()
    f = _dirichlet(rng, 3, shp)
    Yf = OL.collide(S, _with_mixture(probs[0], [p.M for p in probs[1:]], f))
    Ys = [OL.collide(S, p) for p in probs]
    ref = (1.0 - f.sum(axis=0)) * Ys[0] + sum(f[k] * Ys[k + 1] for k in range(3))
    assert np.abs(Yf - ref).max() < 1e-14 * np.abs(ref).max()


def test_k_mixture_order_and_splitting_of_components_do_not_matter():
    """Listing the further components in another order (with their
    fractions), or splitting one component's fraction over two copies of it,
    leaves a 5-step run unchanged up to rounding."""
    probs, S, rng, shp = _k_setup()
    f = _dirichlet(rng, 3, shp)
    Ms = [p.M for p in probs[1:]]
    ref = OL.run(S, _with_mixture(probs[0], Ms, f), 5)
    perm = [2, 0, 1]
    got = OL.run(S, _with_mixture(probs[0], [Ms[k] for k in perm], f[perm]), 5)
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()
    split = rng.uniform(0.0, 1.0, shp)
    f4 = np.concatenate([f, (1.0 - split)[None] * f[1:2]])
    f4[1] = split * f[1]
    got = OL.run(S, _with_mixture(probs[0], Ms + [Ms[1]], f4), 5)
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


def test_k_mixture_conserves_total_intensity_without_absorption():
    probs, S, rng, shp = _k_setup(albedo=1.0, renorm=True, emis=None, jprof=None)
    prob = _with_mixture(probs[0], [p.M for p in probs[1:]], _dirichlet(rng, 3, shp))
    tot0 = S[:, 0].sum()
    for _ in range(20):
        S = OL.step(S, prob)
    assert abs(S[:, 0].sum() - tot0) < 1e-12 * tot0


def test_k_mixture_fractions_summing_past_one_are_refused():
    probs, _, _, shp = _k_setup()
    Ms = [p.M for p in probs[1:]]
    f = np.full((3,) + shp, 0.3)
    _with_mixture(probs[0], Ms, f)                        # sum 0.9: accepted
    f[2, 1, 2] = 0.45
    with pytest.raises(ValueError):
        _with_mixture(probs[0], Ms, f)                    # sum 1.05 in one cell
    f[2, 1, 2] = -0.01
    with pytest.raises(ValueError):
        _with_mixture(probs[0], Ms, f)
    with pytest.raises(ValueError):
        _with_mixture(probs[0], [], np.zeros((0,) + shp))
