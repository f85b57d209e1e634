"""Pins of the oracle's polarisation measures and readouts (CPU only).

The degree of polarisation (Sec. 3.2.1), the direction-mean maps shown in the
paper's figures, and the edge / face readouts that select the directions
leaving the lattice (Sec. 2.1.7) are checked against values fixed by the
field definition of the Stokes parameters and by pure transport, not by
retyping the oracle's formulas.  Each test names the plausible mistake it
catches:
  * DoLP in place of DOP (V dropped), or DOP of the direction-summed Stokes
    vector in place of the mean of per-direction DOP;
  * incoming instead of outgoing directions at an edge or face;
  * the wrong cell order along an edge.
"""
import math

import numpy as np
import pytest

from oracle import directions as ODir
from oracle import lbm as OL
from oracle import lbm3d as O3
from oracle import phase as OP


def _stokes(E):
    """Stokes vector of a complex field (E_theta, E_phi) from its definition:
    I = |E1|^2 + |E2|^2, Q = |E1|^2 - |E2|^2, U = 2 Re(E1 E2*),
    V = 2 Im(E1 E2*) (the sign of V does not enter any degree of polarisation)."""
    e1, e2 = complex(E[0]), complex(E[1])
    return np.array([abs(e1) ** 2 + abs(e2) ** 2, abs(e1) ** 2 - abs(e2) ** 2,
                     2.0 * (e1 * e2.conjugate()).real, 2.0 * (e1 * e2.conjugate()).imag])


def _dop_of(v):
    return float(OL.dop(np.array([v[0]]), np.array([v[1]]), np.array([v[2]]), np.array([v[3]]))[0])


def _dolp_of(v, eps=1e-6):
    return float(OL.dolp(np.array([v[0]]), np.array([v[1]]), np.array([v[2]]), eps)[0])


# ------------------------------------------------------------------- DOP --

@pytest.mark.parametrize("chi", [0.0, 0.2, math.pi / 8, 0.6, math.pi / 4])
@pytest.mark.parametrize("psi", [0.0, 0.7, 2.0])
def test_dop_of_a_pure_field_is_one_and_dolp_is_cos_2chi(chi, psi):
    """A single coherent field is fully polarised: DOP = 1 for any ellipticity
    chi and orientation psi; its linear part is |cos 2 chi| (circular light,
    chi = pi/4, has none).  Dropping V from DOP fails every chi > 0."""
    a = complex(math.cos(chi), 0.0)
    b = complex(0.0, math.sin(chi))
    # rotate the ellipse by psi in the (e_theta, e_phi) frame
    E = (math.cos(psi) * a - math.sin(psi) * b, math.sin(psi) * a + math.cos(psi) * b)
    v = 2.5 * _stokes(E)
    assert abs(_dop_of(v) - 1.0) < 1e-12
    want = math.sqrt(math.cos(2 * chi) ** 2 + 1e-12)
    assert abs(_dolp_of(v) - want) < 1e-12


@pytest.mark.parametrize("w", [0.0, 0.1, 0.35, 0.5, 0.8, 1.0])
def test_dop_of_incoherent_orthogonal_mixture(w):
    """Incoherent sum of an elliptical field (weight w) and its orthogonal
    partner (weight 1 - w): DOP = |2 w - 1| (Stokes vectors of incoherent
    beams add; orthogonal states have opposite polarised parts)."""
    chi, psi = 0.3, 0.4
    a, b = complex(math.cos(chi), 0.0), complex(0.0, math.sin(chi))
    E1 = (math.cos(psi) * a - math.sin(psi) * b, math.sin(psi) * a + math.cos(psi) * b)
    # the orthogonal state: (-E2*, E1*)
    E2 = (-E1[1].conjugate(), E1[0].conjugate())
    v = w * _stokes(E1) + (1.0 - w) * _stokes(E2)
    assert abs(v[0] - 1.0) < 1e-14
    assert abs(_dop_of(v) - abs(2 * w - 1)) < 1e-12


def test_dop_is_zero_where_there_is_no_light():
    assert OL.dop(np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3)).tolist() == [0.0, 0.0, 0.0]


@pytest.mark.parametrize("grid", [(2, 4, 0.0), (4, 8, 0.0), (2, 3, 22.5)])
def test_single_rayleigh_scatter_dop_through_the_oracle_dop(grid):
    """Sec. 3.2.1 closed form, computed by the oracle's own dop(): natural
    light singly Rayleigh-scattered through Theta has DOP
    sin^2 Theta / (1 + cos^2 Theta), in every pair of meridian frames."""
    dirs = ODir.make_directions(grid[0], grid[1], az_offset_deg=grid[2])
    for do in range(dirs.n):
        for di in range(dirs.n):
            v = OP.pair_matrix(dirs, do, di) @ np.array([1.0, 0.0, 0.0, 0.0])
            c = float(dirs.k[do] @ dirs.k[di])
            assert abs(_dop_of(v) - (1 - c * c) / (1 + c * c)) < 1e-12


def test_dop_of_rayleigh_scattered_circular_light_keeps_v():
    """Circular light scattered at 90 deg by the Rayleigh matrix is linearly
    polarised (V -> cos Theta V = 0), while forward (Theta = 0) it stays fully
    circular: DOP 1 with DoLP ~ 0.  A DOP that drops V gives 0 there."""
    circ = _stokes((1.0 / math.sqrt(2.0), 1j / math.sqrt(2.0)))
    v0 = OP.rayleigh_reduced(1.0) @ circ
    assert abs(_dop_of(v0) - 1.0) < 1e-12
    assert _dolp_of(v0) < 1e-5
    v90 = OP.rayleigh_reduced(0.0) @ circ
    # P~(90 deg) maps (1, 0, 0, 1) to (1/2, -1/2, 0, 0) up to its normalisation
    assert abs(_dop_of(v90) - 1.0) < 1e-12
    assert abs(v90[3]) < 1e-15


# ------------------------------------------------------------------ maps --

def test_maps_average_the_per_direction_dop():
    """Two cells, two directions, hand-computed.

    cell 0: direction 0 fully polarised along e_theta (I 1, Q 1), direction 1
    along e_phi (I 1, Q -1): the mean of the per-direction DOP is 1, while
    the summed Stokes vector (2, 0, 0, 0) would give 0.
    cell 1: direction 0 (I 2, V 1) has DOP 1/2 (DoLP 0), direction 1 is dark
    (DOP 0 by convention): the mean is 1/4; a DOP without V gives 0.
    Intensity means: 1 and 1.
    """
    S = np.zeros((2, 4, 1, 2))
    S[0, :, 0, 0] = (1.0, 1.0, 0.0, 0.0)
    S[1, :, 0, 0] = (1.0, -1.0, 0.0, 0.0)
    S[0, :, 0, 1] = (2.0, 0.0, 0.0, 1.0)
    I_mean, dop_mean = OL.maps(S)
    assert I_mean.shape == (1, 2) and dop_mean.shape == (1, 2)
    assert np.allclose(I_mean[0], [1.0, 1.0], atol=0, rtol=1e-15)
    assert np.allclose(dop_mean[0], [1.0, 0.25], atol=1e-15)


def test_totals_sum_every_cell_and_direction():
    S = np.arange(2 * 4 * 3 * 5, dtype=np.float64).reshape(2, 4, 3, 5)
    want = [sum(S[d, s, y, x] for d in range(2) for y in range(3) for x in range(5)) for s in range(4)]
    assert np.array_equal(OL.totals(S), np.array(want))


# ------------------------------------------------------ 2-D edge readout --

def _transport_problem(nx, ny, n_zen, n_az, plane, bc, inflow=None):
    """Pure transport (tau = 0: no absorption, no scattering)."""
    dirs = ODir.make_directions(n_zen, n_az)
    sh = ODir.displacements(dirs, plane)
    M = OP.collision_matrix(dirs)
    z = np.zeros((ny, nx))
    return OL.Problem(nx, ny, dirs, sh, M, 1.0, bc, z, z, z, np.zeros((dirs.n, 4)), inflow)


def test_edge_readout_of_pulses_on_the_d2q9_lattice():
    """Unit pulses in all 8 directions at (x, y) = (2, 5) and (4, 1) of an
    8 x 9 lattice with absorbing edges, 3 steps of pure transport on the
    D2Q9 velocities: the up-going pulses of (2, 5) sit on the top row at
    x = 2, the right-going pulses of (4, 1) on the right column at y = 1, and
    nothing else touches an edge.  The readout must show exactly these at
    edge position e = x (y edges) or e = y (x edges); selecting incoming
    directions, or indexing the edge the wrong way, fails."""
    prob = _transport_problem(8, 9, 2, 4, "xy_d2q9", (1, 1, 1, 1))
    S0 = np.zeros(prob.shape)
    for (x, y) in ((2, 5), (4, 1)):
        S0[:, 0, y, x] = 1.0
    S = OL.run(S0, prob, 3)
    phi = np.degrees(prob.dirs.phi)
    expect = {OL.EDGE_YP: (90.0, 2), OL.EDGE_XP: (0.0, 1), OL.EDGE_YM: (None, None), OL.EDGE_XM: (None, None)}
    for edge, (az, pos) in expect.items():
        out = OL.readout(S, prob, edge)
        dsel = OL.outgoing_directions(prob, edge)
        want = np.zeros_like(out)
        if az is not None:
            for k, d in enumerate(dsel):
                if abs(phi[d] - az) < 1e-9:
                    want[pos, k, 0] = 1.0
            assert want.sum() == 2.0    # both zenith rings of that azimuth
        assert np.array_equal(out, want), edge


def _binomial_tail(T, p, m):
    """P(Bin(T, p) >= m)."""
    return sum(math.comb(T, k) * p ** k * (1.0 - p) ** (T - k) for k in range(m, T + 1))


def test_beam_leaves_through_the_bottom_edge_not_the_top():
    """Vertical plane (lattice y = altitude): a unit beam enters the top edge
    in the downward direction nearest 150 deg zenith (l_y = cos 138.6 deg =
    -3/4) and crosses an empty periodic-in-x column with an absorbing floor.
    The pull of Eq. 34 reads the row above with weight 3/4 and the row itself
    with weight 1/4, so after T steps the bottom row holds the probability
    that T such draws climb ny rows: P(Bin(T, 3/4) >= ny), on every cell of
    the bottom edge and in that direction only.  The top-edge readout lists
    only up-going directions (zenith < 90 deg), all dark."""
    nx, ny = 6, 10
    n_zen, n_az = 4, 8
    d_b = 3 * n_az + 0    # zenith 138.6 deg, azimuth 0
    inflow = np.zeros((4, n_zen * n_az, 4))
    inflow[OL.EDGE_YP, d_b, 0] = 1.0
    prob = _transport_problem(nx, ny, n_zen, n_az, "xz", (0, 0, 1, 2), inflow)
    assert abs(prob.shifts[d_b, 1] + 0.75) < 1e-15
    T = 13
    S = OL.run(np.zeros(prob.shape), prob, T)
    theta = np.degrees(prob.dirs.theta)
    down = OL.outgoing_directions(prob, OL.EDGE_YM)
    up = OL.outgoing_directions(prob, OL.EDGE_YP)
    assert sorted(down.tolist()) == [d for d in range(prob.n) if theta[d] > 90.0]
    assert sorted(up.tolist()) == [d for d in range(prob.n) if theta[d] < 90.0]
    bottom = OL.readout(S, prob, OL.EDGE_YM)
    k_b = int(np.nonzero(down == d_b)[0][0])
    want = _binomial_tail(T, 0.75, ny)
    assert 0.3 < want < 0.9
    assert np.allclose(bottom[:, k_b, 0], want, rtol=0, atol=1e-13)
    rest = np.delete(bottom, k_b, axis=1)
    assert np.abs(rest).max() == 0.0 and np.abs(bottom[:, k_b, 1:]).max() == 0.0
    assert d_b not in up
    assert np.abs(OL.readout(S, prob, OL.EDGE_YP)).max() == 0.0


@pytest.mark.parametrize("edge", [0, 1, 2, 3])
def test_readout_transpose_is_the_transpose(edge):
    """<readout(S), G> = <S, readout_transpose(G)> (the readout adjoint)."""
    prob = _transport_problem(5, 4, 2, 4, "xz", (1, 1, 1, 1))
    rng = np.random.default_rng(edge)
    S = rng.standard_normal(prob.shape)
    G = rng.standard_normal(OL.readout(S, prob, edge).shape)
    lhs = float(np.sum(OL.readout(S, prob, edge) * G))
    rhs = float(np.sum(S * OL.readout_transpose(G, prob, edge)))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


# ------------------------------------------------------ 3-D face readout --

def _transport3d(nx, ny, nz, bc6, inflow6=None):
    dirs = ODir.make_directions(4, 8)
    M = OP.collision_matrix(dirs)
    z = np.zeros((nz, ny, nx))
    return O3.Problem3D(nx, ny, nz, dirs, 1.0, bc6, M, 1.0, z, z, z, np.zeros((dirs.n, 4)), inflow6)


def test_beam_leaves_through_the_bottom_face_not_the_top():
    """3-D: a unit beam enters the top face (z+) in the downward direction
    nearest 150 deg zenith; x and y are periodic, the floor absorbing.  After
    T steps the bottom layer holds P(Bin(T, 3/4) >= nz) in that direction on
    every face cell (the 1-D pull along z of the 2-D test; the x and y pulls
    of a uniform field change nothing), the top face lists only
    up-going directions (zenith < 90 deg), all dark; the x+ face lists the
    directions with k_x > 0 (azimuth within 90 deg of +x)."""
    nx, ny, nz = 4, 3, 6
    d_b = 3 * 8 + 0
    inflow = np.zeros((6, 32, 4))
    inflow[O3.FACE_ZP, d_b, 0] = 1.0
    prob = _transport3d(nx, ny, nz, (0, 0, 0, 0, 1, 2), inflow)
    T = 9
    S = O3.run(np.zeros(prob.shape), prob, T)
    theta = np.degrees(prob.dirs.theta)
    phi = np.degrees(prob.dirs.phi)
    down, up = O3.outgoing(prob, O3.FACE_ZM), O3.outgoing(prob, O3.FACE_ZP)
    assert down == [d for d in range(prob.n) if theta[d] > 90.0]
    assert up == [d for d in range(prob.n) if theta[d] < 90.0]
    east = O3.outgoing(prob, O3.FACE_XP)
    assert east == [d for d in range(prob.n) if math.cos(math.radians(phi[d])) > 1e-12]
    bottom = O3.readout(S, prob, O3.FACE_ZM)
    assert bottom.shape == (nx * ny, len(down), 4)
    k_b = down.index(d_b)
    want = _binomial_tail(T, 0.75, nz)
    assert 0.3 < want < 0.95
    assert np.allclose(bottom[:, k_b, 0], want, rtol=0, atol=1e-13)
    assert np.abs(np.delete(bottom, k_b, axis=1)).max() == 0.0
    assert d_b not in up
    assert np.abs(O3.readout(S, prob, O3.FACE_ZP)).max() == 0.0


def test_face_readout_cell_order():
    """Face cells run with the first index fastest: z faces (x, y), x faces
    (y, z), y faces (x, z).  A field whose I equals a unique cell code must
    come back in that order at every outgoing direction."""
    nx, ny, nz = 3, 4, 2
    prob = _transport3d(nx, ny, nz, (1, 1, 1, 1, 1, 1))
    S = np.zeros(prob.shape)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    S[:, 0] = (100 * zz + 10 * yy + xx)[None]
    cases = {O3.FACE_ZP: [100 * (nz - 1) + 10 * y + x for y in range(ny) for x in range(nx)],
             O3.FACE_XM: [100 * z + 10 * y + 0 for z in range(nz) for y in range(ny)],
             O3.FACE_YP: [100 * z + 10 * (ny - 1) + x for z in range(nz) for x in range(nx)]}
    for face, codes in cases.items():
        out = O3.readout(S, prob, face)
        for k in range(out.shape[1]):
            assert out[:, k, 0].tolist() == codes, face


@pytest.mark.parametrize("face", range(6))
def test_face_readout_transpose_is_the_transpose(face):
    prob = _transport3d(3, 2, 4, (1, 1, 1, 1, 1, 1))
    rng = np.random.default_rng(10 + face)
    S = rng.standard_normal(prob.shape)
    G = rng.standard_normal(O3.readout(S, prob, face).shape)
    lhs = float(np.sum(O3.readout(S, prob, face) * G))
    rhs = float(np.sum(S * O3.readout_transpose(G, prob, face)))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


# --------------------------------------------------- per-edge-cell inflow --

def test_per_cell_inflow_is_carried_along_integer_velocities():
    """Inflow radiance given per top-edge cell, p(x), on the D2Q9 lattice
    with pure transport: after T >= ny steps the straight-down directions
    (velocity (0, -1)) hold p(x) in every row, and the diagonal (-1, -1)
    directions hold p(x + ny - y) where the path back reaches the top edge
    first, zero where it reaches the absorbing right edge first, and at the
    corner (both at once) the top edge's last cell p(nx - 1): a ghost outside
    in y takes its y edge at the x clamped to the lattice (Sec. 2.1.7)."""
    nx, ny = 7, 5
    dirs = ODir.make_directions(2, 8)          # 8 azimuths: diagonals included
    sh = ODir.displacements(dirs, "xy_d2q9")
    n = dirs.n
    prof = 1.0 + np.arange(nx, dtype=np.float64) ** 2 / 7.0
    inflow = np.zeros((2 * (nx + ny), n, 4))
    top = 2 * ny + nx                          # first cell of the y+ edge
    for d in range(n):
        inflow[top:top + nx, d, 0] = prof
        inflow[top:top + nx, d, 1] = 0.25 * prof
    M = OP.collision_matrix(dirs)
    z = np.zeros((ny, nx))
    prob = OL.Problem(nx, ny, dirs, sh, M, 1.0, (1, 1, 1, 2), z, z, z, np.zeros((n, 4)), inflow)
    S = OL.run(np.zeros(prob.shape), prob, ny + 2)
    down = [d for d in range(n) if tuple(sh[d]) == (0.0, -1.0)]
    diag = [d for d in range(n) if tuple(sh[d]) == (-1.0, -1.0)]
    assert len(down) == 2 and len(diag) == 2
    for d in down:
        for y in range(ny):
            assert np.array_equal(S[d, 0, y], prof) and np.array_equal(S[d, 1, y], 0.25 * prof)
    for d in diag:
        for y in range(ny):
            for x in range(nx):
                k_top, k_right = ny - y, nx - x
                want = prof[x + k_top] if k_top < k_right else (0.0 if k_right < k_top else prof[nx - 1])
                assert S[d, 0, y, x] == want, (d, x, y)
