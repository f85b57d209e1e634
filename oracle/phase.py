"""Polarised phase matrix by the rotation-phase-rotation sequence (oracle).

TEST INFRASTRUCTURE ONLY.

Paper: Sec. 2.1.5.  Eq. 13 (Stokes of the pair (d_out, d_in) = R(psi_out)
P(theta) R(psi_in) S), Eq. 14 (theta = arccos(v_out . v_in)), Eq. 16 (Rayleigh
Mueller matrix, reduced form P~ = [[a,b,0,0],[b,a,0,0],[0,0,c,0],[0,0,0,c]]
with a = (1+cos^2)/2, b = -sin^2/2, c = cos), Eq. 17 (column-normalised
weights w(d_out,d_in) = p(theta) dOmega_out / sum_out p dOmega_out), Eq. 21-22
(Mueller rotation: Q' = Q cos2psi + U sin2psi, U' = U cos2psi - Q sin2psi) and
Eq. 25/30 (effect of the LCU: sum over pairs weighted by w).

Readings (see the design notes for the full list):
  * Eq. 15 prints psi = atan2(v_y, v_x), the azimuth of each direction; that
    is not the angle between a meridian plane and the scattering plane, and it
    does not reproduce the printed DOP 9/17 at 75.5 deg (Sec. 3.2.2).  The
    angles used here are the true frame angles: sigma_in rotates the incoming
    meridian frame (e_theta, e_phi) onto the scattering frame (e_par, n), and
    sigma_out rotates the outgoing scattering frame onto the outgoing meridian
    frame.
  * Block of the collision matrix for the pair = w * Z / Z_11, so the I->I
    element of the block is exactly the Eq. 17 weight and sum_out M_II = 1
    (the discrete normalisation of Sec. 2.1.1).  The literal w * P~ counts
    the (1+cos^2)/2 factor twice and loses energy.
  * Heyney-Greenstein and Rayleigh/HG mixtures keep the Rayleigh reduced
    matrix and change only the Eq. 17 weights (phase function p).
  * General scattering matrices (the full-Mueller representation that the
    conclusions name as future work, e.g. Mie particles with P34 != 0): a
    table of the six elements of a mirror-symmetric, macroscopically
    isotropic medium's matrix against the scattering angle,
        F = [[a1, b1, 0, 0], [b1, a2, 0, 0], [0, 0, a3, b2], [0, 0, -b2, a4]]
    in the scattering-plane frame (e_par, n), linearly interpolated in the
    angle (degrees).  It takes the place of P~ in Eq. 13; a1 is the phase
    function of the Eq. 17 weights.  For a single particle with amplitude
    functions S1 (perpendicular) and S2 (parallel), a1 = a2 = (|S1|^2 +
    |S2|^2)/2, b1 = (|S2|^2 - |S1|^2)/2, a3 = a4 = Re(S2 S1*) and
    b2 = -Im(S2 S1*) when V = 2 Im(E_1 E_2*).
"""
import numpy as np


def rayleigh_reduced(cos_t):
    """P~(theta) of Eq. 16 without the 3/(8 pi) factor."""
    c = float(cos_t)
    a = 0.5 * (1.0 + c * c)
    b = -0.5 * (1.0 - c * c)
    return np.array([[a, b, 0.0, 0.0],
                     [b, a, 0.0, 0.0],
                     [0.0, 0.0, c, 0.0],
                     [0.0, 0.0, 0.0, c]])


def mueller_rotation(psi):
    """R(psi) of Eq. 21 in the component form of Eq. 22."""
    c2, s2 = np.cos(2.0 * psi), np.sin(2.0 * psi)
    return np.array([[1.0, 0.0, 0.0, 0.0],
                     [0.0, c2, s2, 0.0],
                     [0.0, -s2, c2, 0.0],
                     [0.0, 0.0, 0.0, 1.0]])


def rpr_angles(dirs, d_out, d_in):
    """(cos theta, sigma_in, sigma_out) for the ordered pair (d_out <- d_in).

    n = k_in x k_out / |.| is the normal of the scattering plane (for theta = 0
    or pi the plane is undefined and n = e_phi(in) is used); the in-plane
    polarisation axes are e_par = n x k.  R(psi) maps Stokes referred to
    (e1, e2) onto Stokes referred to (cos psi e1 + sin psi e2, ...), so
      sigma_in  = angle from e_theta(in) to e_par(in)   (meridian -> scattering)
      sigma_out = angle from e_par(out) to e_theta(out) (scattering -> meridian)
    """
    ki, ko = dirs.k[d_in], dirs.k[d_out]
    cos_t = float(np.clip(np.dot(ko, ki), -1.0, 1.0))
    nrm = np.cross(ki, ko)
    nn = np.linalg.norm(nrm)
    if nn < 1e-12:
        nrm = dirs.e_phi[d_in].copy()
    else:
        nrm = nrm / nn
    epar_in = np.cross(nrm, ki)
    epar_out = np.cross(nrm, ko)
    sig_in = np.arctan2(np.dot(epar_in, dirs.e_phi[d_in]),
                        np.dot(epar_in, dirs.e_theta[d_in]))
    eth_out = dirs.e_theta[d_out]
    sig_out = np.arctan2(np.dot(eth_out, nrm), np.dot(eth_out, epar_out))
    return cos_t, sig_in, sig_out


def table_reduced(cos_t, table):
    """F(theta) from a table of rows (theta_deg, a1, a2, a3, a4, b1, b2),
    linear in theta between rows (rows from 0 to 180 degrees)."""
    tab = np.asarray(table, dtype=np.float64)
    c = float(cos_t)
    # arccos loses half the digits next to +-1: cosines within 1e-12 of +-1
    # are the forward / backward rows themselves
    th = 0.0 if c >= 1.0 - 1e-12 else (180.0 if c <= -1.0 + 1e-12 else np.degrees(np.arccos(c)))
    a1, a2, a3, a4, b1, b2 = (np.interp(th, tab[:, 0], tab[:, j]) for j in range(1, 7))
    return np.array([[a1, b1, 0.0, 0.0],
                     [b1, a2, 0.0, 0.0],
                     [0.0, 0.0, a3, b2],
                     [0.0, 0.0, -b2, a4]])


def check_table(table):
    """Rows (theta_deg, a1, a2, a3, a4, b1, b2): at least two, angles strictly
    increasing from 0 to 180, finite, a1 > 0, and the rows at 0 and 180
    degrees invariant under a rotation of the scattering plane (to 1e-6 of
    a1), where the plane n = e_phi(in) is used."""
    tab = np.asarray(table, dtype=np.float64)
    if tab.ndim != 2 or tab.shape[1] != 7 or tab.shape[0] < 2:
        raise ValueError("table must have shape (>= 2, 7)")
    if not np.all(np.isfinite(tab)):
        raise ValueError("table not finite")
    if tab[0, 0] != 0.0 or tab[-1, 0] != 180.0 or np.any(np.diff(tab[:, 0]) <= 0.0):
        raise ValueError("table angles must increase strictly from 0 to 180 degrees")
    if np.any(tab[:, 1] <= 0.0):
        raise ValueError("table a1 must be > 0")
    # forward and backward the scattering plane is undefined: F must not
    # depend on it (b1 = b2 = 0, a3 = a2 forward, a3 = -a2 backward)
    f, b = tab[0], tab[-1]
    tol = 1e-6
    if (abs(f[5]) > tol * f[1] or abs(f[6]) > tol * f[1] or abs(f[3] - f[2]) > tol * f[1]
            or abs(b[5]) > tol * b[1] or abs(b[6]) > tol * b[1] or abs(b[3] + b[2]) > tol * b[1]):
        raise ValueError("table rows at 0 and 180 degrees must not depend on the scattering plane")
    return tab


def pair_matrix(dirs, d_out, d_in, reduced=None):
    """Z = R(sigma_out) F(theta) R(sigma_in), Eq. 13; F is the Rayleigh P~
    unless `reduced` (a function of cos theta) gives another."""
    cos_t, s_in, s_out = rpr_angles(dirs, d_out, d_in)
    F = rayleigh_reduced(cos_t) if reduced is None else reduced(cos_t)
    return mueller_rotation(s_out) @ F @ mueller_rotation(s_in)


def phase_function(cos_t, kind="rayleigh", g=0.0, mix_ray=1.0, table=None):
    """Scalar phase function p(theta), normalised to 1 over 4 pi.

    rayleigh   3/(16 pi) (1 + cos^2)            (Eq. 16, element 11 x 2)
    hg         (1-g^2) / (4 pi (1+g^2-2g cos)^1.5)
    mix        mix_ray * p_rayleigh + (1-mix_ray) * p_hg
    """
    c = np.asarray(cos_t, dtype=np.float64)
    if kind == "table":
        return table_reduced(c, table)[0, 0]
    pr = 3.0 / (16.0 * np.pi) * (1.0 + c * c)
    if kind == "rayleigh":
        return pr
    phg = (1.0 - g * g) / (4.0 * np.pi * (1.0 + g * g - 2.0 * g * c) ** 1.5)
    if kind == "hg":
        return phg
    if kind == "mix":
        return mix_ray * pr + (1.0 - mix_ray) * phg
    raise ValueError(kind)


def weights(dirs, kind="rayleigh", g=0.0, mix_ray=1.0, table=None):
    """Eq. 17: w[out, in] = p(theta) dOmega_out / sum_out p(theta) dOmega_out."""
    n = dirs.n
    w = np.zeros((n, n))
    for di in range(n):
        for do in range(n):
            ct = float(np.clip(np.dot(dirs.k[do], dirs.k[di]), -1.0, 1.0))
            w[do, di] = phase_function(ct, kind, g, mix_ray, table) * dirs.domega[do]
        w[:, di] /= w[:, di].sum()
    return w


def collision_matrix(dirs, kind="rayleigh", g=0.0, mix_ray=1.0,
                     renorm_irow=False, scalar=False, table=None):
    """The 4n x 4n direction-pair sum of Eq. 25/30.

    Index convention: row/column 4*d + s, s in (I, Q, U, V).  Column block d_in
    is the source direction, row block d_out the destination, so the scattered
    field is (M @ X)[4 d_out + s].

    scalar       keep only the I->I elements (intensity-only transport)
    renorm_irow  subtract from the Q and U columns of the I row the weighted
                 column sums over outgoing directions, so that sum_out of the
                 Q->I and U->I elements is zero and total I is conserved
                 exactly for polarised fields (an option, not in the paper).
    """
    n = dirs.n
    reduced = None
    if kind == "table":
        table = check_table(table)
        reduced = lambda c: table_reduced(c, table)  # noqa: E731
    w = weights(dirs, kind, g, mix_ray, table)
    M = np.zeros((4 * n, 4 * n))
    for di in range(n):
        for do in range(n):
            if scalar:
                blk = np.zeros((4, 4))
                blk[0, 0] = 1.0
            else:
                Z = pair_matrix(dirs, do, di, reduced)
                blk = Z / Z[0, 0]
            M[4 * do:4 * do + 4, 4 * di:4 * di + 4] = w[do, di] * blk
    if renorm_irow and not scalar:
        for di in range(n):
            for j in (1, 2):
                col = 4 * di + j
                tot = sum(M[4 * do, col] for do in range(n))
                for do in range(n):
                    M[4 * do, col] -= w[do, di] * tot
    return M
