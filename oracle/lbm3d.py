"""Three-dimensional lattice (oracle).

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Paper: the conclusions state that the lattice formulation extends to three
dimensions and name it as a priority; the paper gives no 3-D scheme, so this
takes its 2-D steps with a third axis:
  * collision (emission, absorption, scattering; Sec. 2.1.3-2.1.5): the
    per-cell operator of lbm.collide, unchanged; it acts on every cell alone,
    so it is applied to the cells of the 3-D lattice in a flattened view;
  * streaming (Sec. 2.1.6, Eq. 33-34): the displacement is the whole
    direction vector, l = courant * (k_x, k_y, k_z), and the pull is the
    product of the 1-D taps of Eq. 34 along x, y and z (trilinear);
  * faces (Sec. 2.1.7, Eq. 39): x-, x+, y-, y+, z-, z+ each periodic (both
    faces of an axis), absorbing (ghosts are zero) or inflow (ghosts carry
    inflow[face, d, :]); a tap outside in z takes its z face, else its
    y face, else its x face.
State S[d, s, z, y, x]; cell index c = (z ny + y) nx + x.
"""
import numpy as np

from . import directions as _dirs
from . import lbm
from . import phase as _phase

FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = range(6)


class Problem3D:
    """A 3-D solve in float64: the flattened per-cell problem `flat` (its
    nx x (ny nz) cells carry the medium; its edges are unused) plus the
    three-axis streaming."""

    def __init__(self, nx, ny, nz, dirs, courant, bc6, M, dt, tau, albedo, emis, jprof,
                 inflow6=None, **opts):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dirs = dirs
        self.n = dirs.n
        self.shifts = _dirs.snap_integers(courant * np.asarray(dirs.k, dtype=np.float64))
        if np.any(np.abs(self.shifts) > 1.0 + 1e-12):
            raise ValueError("|l| > 1 per step")
        self.bc = tuple(int(b) for b in bc6)
        for a in range(3):
            if (self.bc[2 * a] == lbm.BC_PERIODIC) != (self.bc[2 * a + 1] == lbm.BC_PERIODIC):
                raise ValueError("both faces of an axis must be periodic or neither")
        if inflow6 is None:
            inflow6 = np.zeros((6, self.n, 4))
        self.inflow = np.asarray(inflow6, dtype=np.float64).reshape(6, self.n, 4)
        flat = lambda a: None if a is None else np.asarray(a, dtype=np.float64).reshape(  # noqa: E731
            self.nz * self.ny, self.nx)
        if opts.get("dichroism") is not None:
            opts["dichroism"] = flat(opts["dichroism"])
        if opts.get("frac") is not None:
            # [nz, ny, nx] or, for several further phase functions, [K - 1, nz, ny, nx]
            f = np.asarray(opts["frac"], dtype=np.float64)
            opts["frac"] = f.reshape(-1, self.nz * self.ny, self.nx) if f.ndim == 4 else flat(f)
        self.flat = lbm.Problem(self.nx, self.ny * self.nz, dirs, self.shifts[:, :2], M, dt, (0, 0, 0, 0),
                                flat(tau), flat(albedo), flat(emis), jprof, None, **opts)

    @property
    def shape(self):
        return (self.n, 4, self.nz, self.ny, self.nx)


def collide(S, prob):
    """Emission, absorption and scattering at every cell (lbm.collide on the
    flattened cells)."""
    Y = lbm.collide(np.asarray(S, dtype=np.float64).reshape(prob.flat.shape), prob.flat)
    return Y.reshape(prob.shape)


def _fetch(vol, xs, ys, zs, d, prob):
    """vol[4, nz, ny, nx] read at integer (xs, ys, zs) with the face rules."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    if prob.bc[FACE_XM] == lbm.BC_PERIODIC:
        xs = np.mod(xs, nx)
    if prob.bc[FACE_YM] == lbm.BC_PERIODIC:
        ys = np.mod(ys, ny)
    if prob.bc[FACE_ZM] == lbm.BC_PERIODIC:
        zs = np.mod(zs, nz)
    inz = (zs >= 0) & (zs < nz)
    iny = (ys >= 0) & (ys < ny)
    inx = (xs >= 0) & (xs < nx)
    inside = inx & iny & inz
    vals = np.zeros((4,) + xs.shape)
    vals[:, inside] = vol[:, zs[inside], ys[inside], xs[inside]]
    faces = ((zs >= nz, FACE_ZP), (zs < 0, FACE_ZM),
             (inz & (ys >= ny), FACE_YP), (inz & (ys < 0), FACE_YM),
             (inz & iny & (xs >= nx), FACE_XP), (inz & iny & (xs < 0), FACE_XM))
    for mask, face in faces:
        if prob.bc[face] == lbm.BC_INFLOW and np.any(mask):
            vals[:, mask] = prob.inflow[face, d, :, None]
    return vals


def stream(Y, prob):
    """S'[d](x, y, z) = sum over the taps of Eq. 34 along each axis of
    wx wy wz Y[d](x - ox, y - oy, z - oz)."""
    Y = np.asarray(Y, dtype=np.float64).reshape(prob.shape)
    out = np.zeros_like(Y)
    zz, yy, xx = np.meshgrid(np.arange(prob.nz), np.arange(prob.ny), np.arange(prob.nx), indexing="ij")
    for d in range(prob.n):
        lx, ly, lz = prob.shifts[d]
        for ox, wx in lbm._taps(lx):
            for oy, wy in lbm._taps(ly):
                for oz, wz in lbm._taps(lz):
                    out[d] += wx * wy * wz * _fetch(Y[d], xx - ox, yy - oy, zz - oz, d, prob)
    return out


def step(S, prob):
    return stream(collide(S, prob), prob)


def run(S0, prob, nsteps, keep=False):
    S = np.array(S0, dtype=np.float64).reshape(prob.shape)
    hist = [S.copy()] if keep else None
    for _ in range(nsteps):
        S = step(S, prob)
        if keep:
            hist.append(S.copy())
    return (S, hist) if keep else S


def make_problem(spec, medium):
    """A Problem3D from a workload spec (plane "3d") and its medium."""
    if spec.get("dir_xyz") is not None:
        dirs = _dirs.VectorDirectionSet(spec["dir_xyz"], spec.get("dir_domega"))
    else:
        dirs = _dirs.make_directions(spec["n_zen"], spec["n_az"], spec.get("zen_rule", "equal_area"),
                                     spec.get("az_offset_deg", 0.0), spec.get("zen_explicit_deg"))
        if spec.get("dir_domega") is not None:
            dirs.domega = np.asarray(spec["dir_domega"], dtype=np.float64).reshape(dirs.n).copy()
    ph = spec.get("phase", {"kind": "rayleigh"})
    M = _phase.collision_matrix(dirs, ph.get("kind", "rayleigh"), ph.get("g", 0.0),
                                ph.get("mix_ray", 1.0), spec.get("renorm_irow", False),
                                spec.get("scalar", False), ph.get("table"))
    M2 = lbm.mixture_matrices(dirs, spec)
    p3 = Problem3D(spec["nx"], spec["ny"], spec["nz"], dirs, spec.get("courant", 1.0), spec["bc6"], M,
                     spec.get("dt", 1.0), medium["tau"], medium["albedo"], medium["emis"], medium["jprof"],
                     medium.get("inflow"), abs_taylor=spec.get("abs_taylor", False),
                     scat_exp=spec.get("scat_exp", False), fused_taylor=spec.get("fused_taylor", False),
                     M2=M2, frac=medium.get("frac"), dichroism=medium.get("eta"))
    if spec.get("shift") is not None:
        # explicit displacement per step replaces courant * k
        sh = _dirs.snap_integers(np.asarray(spec["shift"], dtype=np.float64).reshape(dirs.n, 3))
        if np.any(np.abs(sh) > 1.0 + 1e-12):
            raise ValueError("|l| > 1 per step")
        p3.shifts = sh
        p3.flat.shifts = sh[:, :2]
    return p3


def stream_transpose(G, prob):
    """Transpose of the linear part of stream(): the forward adds w Y[source]
    into target; the transpose adds w G[target] into source, for sources in
    the lattice only (ghosts are constants and carry no gradient)."""
    G = np.asarray(G, dtype=np.float64).reshape(prob.shape)
    out = np.zeros_like(G)
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for d in range(prob.n):
        lx, ly, lz = prob.shifts[d]
        for ox, wx in lbm._taps(lx):
            for oy, wy in lbm._taps(ly):
                for oz, wz in lbm._taps(lz):
                    xs, ys, zs = xx - ox, yy - oy, zz - oz
                    if prob.bc[FACE_XM] == lbm.BC_PERIODIC:
                        xs = np.mod(xs, nx)
                    if prob.bc[FACE_YM] == lbm.BC_PERIODIC:
                        ys = np.mod(ys, ny)
                    if prob.bc[FACE_ZM] == lbm.BC_PERIODIC:
                        zs = np.mod(zs, nz)
                    inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny) & (zs >= 0) & (zs < nz)
                    for s in range(4):
                        np.add.at(out[d, s], (zs[inside], ys[inside], xs[inside]),
                                  wx * wy * wz * G[d, s][inside])
    return out


def adjoint(S0, prob, nsteps, lam_T):
    """Reverse-mode gradient on a 3-D lattice, the chain rule of oracle.adjoint
    with the 3-D streaming: for t = T-1 .. 0, mu = L^T lambda_{t+1},
    nu = M^T mu (mixed as in the forward step: (1 - sum f_k) M^T mu + sum f_k M_k^T mu),
    lambda_t = alpha mu + beta nu, g_alpha += <mu, X_t>,
    g_beta += <nu, X_t>, g_emis += dt <e lambda_t + (1 - e) mu, jprof>.
    Returns dict(lambda0, g_alpha, g_beta, g_tau, g_albedo, g_emis), per-cell
    arrays [nz, ny, nx]."""
    f = prob.flat
    from .adjoint import dichroic_derivative
    n, C = prob.n, prob.nx * prob.ny * prob.nz
    J = f.emission_field().reshape(prob.shape)
    e = 0.0 if f.fused_taylor else 1.0
    _, hist = run(S0, prob, nsteps, keep=True)
    jp = f.jprof.reshape(n, 4, 1)
    lam = np.array(lam_T, dtype=np.float64).reshape(prob.shape)
    al, be = f.alpha.reshape(C), f.beta.reshape(C)
    g_al, g_be, g_em, g_xi = np.zeros(C), np.zeros(C), np.zeros(C), np.zeros(C)
    for t in range(nsteps - 1, -1, -1):
        X = (hist[t] + e * f.dt * J).reshape(4 * n, C)
        X0 = X
        if f.eta is not None:
            X = lbm.dichroic_absorption(X0, f)
        mu = stream_transpose(lam, prob).reshape(4 * n, C)
        nu = lbm.scatter_product(f, mu, transpose=True)
        g_al += np.sum(mu * X, axis=0)
        g_be += np.sum(nu * X, axis=0)
        lam_x = al[None, :] * mu + be[None, :] * nu
        if f.eta is not None:
            g_xi += np.sum(lam_x * dichroic_derivative(X0, f), axis=0)
            lam_x = lbm.dichroic_absorption(lam_x, f)   # D^T = D (symmetric in I, Q)
        src = e * lam_x + (1.0 - e) * mu
        g_em += f.dt * np.sum(src.reshape(n, 4, C) * jp, axis=(0, 1))
        lam = lam_x.reshape(prob.shape)
    dal_dt, dal_dw, dbe_dt, dbe_dw = lbm.coefficient_derivatives(f.tau, f.albedo, f.abs_taylor, f.scat_exp,
                                                                 f.fused_taylor)
    shp = (prob.nz, prob.ny, prob.nx)
    g_al, g_be, g_xi = g_al.reshape(shp), g_be.reshape(shp), g_xi.reshape(shp)
    eta = 0.0 if f.eta is None else f.eta.reshape(shp)
    return {"lambda0": lam, "g_alpha": g_al, "g_beta": g_be,
            "g_tau": g_al * dal_dt.reshape(shp) + g_be * dbe_dt.reshape(shp)
            + g_xi * (1.0 - f.albedo.reshape(shp)) * eta,
            "g_albedo": g_al * dal_dw.reshape(shp) + g_be * dbe_dw.reshape(shp) - g_xi * f.tau.reshape(shp) * eta,
            "g_emis": g_em.reshape(shp)}


def face_cells(prob, face):
    """Cell indices (z, y, x) of a face in readout order: x faces (y, z),
    y faces (x, z), z faces (x, y), the first index fastest."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    if face in (FACE_XM, FACE_XP):
        x = 0 if face == FACE_XM else nx - 1
        return [(z, y, x) for z in range(nz) for y in range(ny)]
    if face in (FACE_YM, FACE_YP):
        y = 0 if face == FACE_YM else ny - 1
        return [(z, y, x) for z in range(nz) for x in range(nx)]
    z = 0 if face == FACE_ZM else nz - 1
    return [(z, y, x) for y in range(ny) for x in range(nx)]


def outgoing(prob, face):
    """Directions whose displacement leaves through the face, increasing d."""
    axis, sign = face // 2, (-1 if face % 2 == 0 else 1)
    return [d for d in range(prob.n) if sign * prob.shifts[d, axis] > 0]


def readout(S, prob, face):
    """Stokes vectors of the outgoing directions on a face: [cell][k][4]."""
    S = np.asarray(S, dtype=np.float64).reshape(prob.shape)
    cells, dirs = face_cells(prob, face), outgoing(prob, face)
    out = np.zeros((len(cells), len(dirs), 4))
    for e, (z, y, x) in enumerate(cells):
        for k, d in enumerate(dirs):
            out[e, k] = S[d, :, z, y, x]
    return out


def readout_transpose(G, prob, face):
    """A state that is zero except the face entries, which receive G."""
    lam = np.zeros(prob.shape)
    cells, dirs = face_cells(prob, face), outgoing(prob, face)
    for e, (z, y, x) in enumerate(cells):
        for k, d in enumerate(dirs):
            lam[d, :, z, y, x] = G[e, k]
    return lam
