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


def pair_matrix(dirs, d_out, d_in):
    """Z = R(sigma_out) P~(theta) R(sigma_in), Eq. 13."""
    cos_t, s_in, s_out = rpr_angles(dirs, d_out, d_in)
    return mueller_rotation(s_out) @ rayleigh_reduced(cos_t) @ mueller_rotation(s_in)


def phase_function(cos_t, kind="rayleigh", g=0.0, mix_ray=1.0):
    """Scalar phase function p(theta), normalised to 1 over 4 pi.

    rayleigh   3/(16 pi) (1 + cos^2)            (Eq. 16, element 11 x 2)
    hg         (1-g^2) / (4 pi (1+g^2-2g cos)^1.5)
    mix        mix_ray * p_rayleigh + (1-mix_ray) * p_hg
    """
    c = np.asarray(cos_t, dtype=np.float64)
    pr = 3.0 / (16.0 * np.pi) * (1.0 + c * c)
    if kind == "rayleigh":
        return pr
    phg = (1.0 - g * g) / (4.0 * np.pi * (1.0 + g * g - 2.0 * g * c) ** 1.5)
    if kind == "hg":
        return phg
    if kind == "mix":
        return mix_ray * pr + (1.0 - mix_ray) * phg
    raise ValueError(kind)


def weights(dirs, kind="rayleigh", g=0.0, mix_ray=1.0):
    """Eq. 17: w[out, in] = p(theta) dOmega_out / sum_out p(theta) dOmega_out."""
    n = dirs.n
    w = np.zeros((n, n))
    for di in range(n):
        for do in range(n):
            ct = float(np.clip(np.dot(dirs.k[do], dirs.k[di]), -1.0, 1.0))
            w[do, di] = phase_function(ct, kind, g, mix_ray) * dirs.domega[do]
        w[:, di] /= w[:, di].sum()
    return w


def collision_matrix(dirs, kind="rayleigh", g=0.0, mix_ray=1.0,
                     renorm_irow=False, scalar=False):
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
    w = weights(dirs, kind, g, mix_ray)
    M = np.zeros((4 * n, 4 * n))
    for di in range(n):
        for do in range(n):
            if scalar:
                blk = np.zeros((4, 4))
                blk[0, 0] = 1.0
            else:
                Z = pair_matrix(dirs, do, di)
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
