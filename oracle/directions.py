"""Direction grid and lattice displacements (oracle; test infrastructure only).

Paper: Sec. 2 (angular domain discretised by zenith and azimuth angles that are
uniformly distributed), Sec. 2.1.1 (discrete normalisation with quadrature
weight 4*pi/n per direction), Sec. 2.1.6 Eq. 33 (displacement per step
l(d) = v(d) dt / dx) and the D2Q9 statement of Sec. 2.1 that the eight lattice
velocities are (-1, 0, 1) in x and y.

Readings taken where the paper is silent (listed with the others in the design
notes):
  * zenith nodes "uniformly distributed" = equal-area cos(theta) midpoints,
    theta_i = arccos(1 - (2i+1)/n_zen); with n_zen = 2 this gives 60/120 deg,
    the only zenith pair the paper's angle table (Sec. 3.2.2) pins.  Explicit
    lists (Table 2 style) and uniform-theta nodes are also accepted.
  * polar axis +z, x = east-west, y = north-south (Sec. 2.1.2, Eq. 13 text).
  * direction index d = i_zen * n_az + j_az.
"""
import numpy as np


def zenith_nodes(n_zen, rule="equal_area", explicit=None):
    """Zenith angles in radians.

    equal_area     theta_i = arccos(1 - (2i+1)/n_zen): every node owns the
                   same solid angle, so dOmega = 4 pi / n is exact (Sec. 2.1.1).
    uniform_theta  theta_i = (i+1) pi / (n_zen+1).
    explicit       the given list of degrees (Table 2 uses 30..75 deg).
    """
    if rule == "explicit":
        return np.radians(np.asarray(explicit, dtype=np.float64))
    i = np.arange(n_zen, dtype=np.float64)
    if rule == "equal_area":
        return np.arccos(1.0 - (2.0 * i + 1.0) / n_zen)
    if rule == "uniform_theta":
        return (i + 1.0) * np.pi / (n_zen + 1.0)
    raise ValueError(rule)


def azimuth_nodes(n_az, offset_deg=0.0):
    """phi_j = offset + 2 pi j / n_az (Table 1: offsets 0 and 22.5 deg)."""
    j = np.arange(n_az, dtype=np.float64)
    return np.radians(offset_deg) + 2.0 * np.pi * j / n_az


class DirectionSet:
    """n = n_zen * n_az unit vectors with their meridian-plane frames.

    k       propagation direction (sin t cos p, sin t sin p, cos t)
    e_theta unit vector along increasing zenith angle (in the meridian plane)
    e_phi   unit vector along increasing azimuth (normal to the meridian plane)
    (e_theta, e_phi, k) is right handed.  Stokes vectors of direction d are
    referred to (e_theta, e_phi): Q > 0 means polarised along e_theta.
    """

    def __init__(self, theta_zen, phi_az):
        th, ph = np.meshgrid(np.asarray(theta_zen, float), np.asarray(phi_az, float),
                             indexing="ij")
        self.theta = th.reshape(-1)
        self.phi = ph.reshape(-1)
        self.n_zen = len(theta_zen)
        self.n_az = len(phi_az)
        self.n = self.theta.size
        st, ct = np.sin(self.theta), np.cos(self.theta)
        sp, cp = np.sin(self.phi), np.cos(self.phi)
        self.k = np.stack([st * cp, st * sp, ct], axis=1)
        self.e_theta = np.stack([ct * cp, ct * sp, -st], axis=1)
        self.e_phi = np.stack([-sp, cp, np.zeros_like(sp)], axis=1)
        # Sec. 2.1.1: omega_d' = 4 pi / n_d
        self.domega = np.full(self.n, 4.0 * np.pi / self.n)


class VectorDirectionSet:
    """An explicit direction set: n unit vectors k (polar axis +z) with their
    solid angles (the weights of the Eq. 17 normalisation; 4 pi / n when not
    given, Sec. 2.1.1).  Zenith and azimuth are those of k; the meridian
    frame is built from them as for the grid (e_theta along increasing
    zenith, e_phi along increasing azimuth).  A vector along the polar axis
    has no meridian plane and is refused."""

    def __init__(self, k, domega=None):
        k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
        if np.any(~np.isfinite(k)) or np.any(np.abs(np.linalg.norm(k, axis=1) - 1.0) > 1e-9):
            raise ValueError("direction vectors must be finite unit vectors")
        self.n = k.shape[0]
        self.n_zen, self.n_az = 1, self.n
        self.theta = np.arccos(np.clip(k[:, 2], -1.0, 1.0))
        self.phi = np.arctan2(k[:, 1], k[:, 0])
        if np.any(np.sin(self.theta) < 1e-9):
            raise ValueError("a direction along the polar axis has no meridian plane")
        st, ct = np.sin(self.theta), np.cos(self.theta)
        sp, cp = np.sin(self.phi), np.cos(self.phi)
        self.k = k.copy()
        self.e_theta = np.stack([ct * cp, ct * sp, -st], axis=1)
        self.e_phi = np.stack([-sp, cp, np.zeros_like(sp)], axis=1)
        if domega is None:
            self.domega = np.full(self.n, 4.0 * np.pi / self.n)
        else:
            self.domega = np.asarray(domega, dtype=np.float64).reshape(self.n).copy()
            if np.any(~np.isfinite(self.domega)) or np.any(self.domega <= 0):
                raise ValueError("solid angles must be finite and positive")


def make_directions(n_zen, n_az, zen_rule="equal_area", az_offset_deg=0.0,
                    zen_explicit_deg=None):
    th = zenith_nodes(n_zen, zen_rule, zen_explicit_deg)
    return DirectionSet(th, azimuth_nodes(n_az, az_offset_deg))


def displacements(dirs, plane, courant=1.0):
    """Lattice displacement per step (l_x, l_y) for every direction, Eq. 33.

    plane = "xy"        projection of k on the horizontal lattice plane,
                        l = courant * (k_x, k_y)
    plane = "xz"        vertical lattice plane (lattice y is altitude),
                        l = courant * (k_x, k_z)
    plane = "xy_d2q9"   D2Q9 velocities: each component of (cos phi, sin phi)
                        rounded to the nearest of {-1, 0, 1} (Sec. 2.1: eight
                        streaming directions along the lattice axes); a
                        component within 1e-6 of +-1/2 is ambiguous and refused.
    """
    if plane == "xy":
        l = courant * dirs.k[:, :2]
    elif plane == "xz":
        l = courant * dirs.k[:, [0, 2]]
    elif plane == "xy_d2q9":
        c = np.stack([np.cos(dirs.phi), np.sin(dirs.phi)], axis=1)
        if np.any(np.abs(np.abs(c) - 0.5) < 1e-6):
            raise ValueError("azimuth ambiguous for D2Q9 snapping")
        l = np.where(c > 0.5, 1.0, np.where(c < -0.5, -1.0, 0.0))
    else:
        raise ValueError(plane)
    l = snap_integers(l)
    if np.any(np.abs(l) > 1.0 + 1e-12):
        raise ValueError("|l| > 1 per step")
    return np.asarray(l, dtype=np.float64)


def snap_integers(l, tol=1e-12):
    """Displacement components within tol of an integer are that integer.

    cos(90 deg) evaluates to 6e-17, not 0: without this an azimuth of 90 deg
    would carry a vanishing x displacement, a 6e-17-weight tap (Eq. 34) and
    a place among the directions leaving through the x+ edge, although it
    moves along the lattice axis."""
    l = np.asarray(l, dtype=np.float64)
    r = np.round(l)
    return np.where(np.abs(l - r) < tol, r, l)
