"""The classical polarized lattice-Boltzmann step, its boundaries and readout (oracle).

TEST INFRASTRUCTURE ONLY.

State layout: S[d, s, y, x], float64, d = direction, s in (I, Q, U, V).

One time step (Sec. 2.1.1 Eq. 2, split into the operator chain of Eq. 5 whose
intermediate states are Eq. 8 -> Eq. 10 -> Eq. 32 -> Eq. 39):
  1. emission      X = S + dt * J,  J[d, :, c] = emis[c] * jprof[d, :]
                   (Eq. 6/8; the source is not depleted and is not streamed)
  2. absorption    factor a = exp(-tau_abs)  (Beer-Lambert, Sec. 2.1.4;
                   the first-order Taylor 1 - tau_abs behind a flag)
  3. scattering    survival s = 1 - tau_sca and redistribution 1 - s through
                   the collision matrix M (Eq. 11-12, Eq. 25/30):
                   Y = a * (s X + (1 - s) M X) = alpha X + beta M X
  4. streaming     S' = L(Y), L the bilinear semi-Lagrangian shift of Eq. 34
                   with T_c: f_x -> f_{x-c}, base shift floor(l) and fraction
                   f = l - floor(l) in [0, 1); edges periodic (modulo, Eq. 39),
                   absorbing (zero fill, Sec. 2.1.7) or inflow (prescribed
                   ghost radiance per edge and direction).
with tau_ext the per-step optical depth k_ext * dt of a cell, tau_sca =
albedo * tau_ext, tau_abs = (1 - albedo) * tau_ext.

The literal Eq. 2 form (fused first-order Taylor of Igarashi et al., used by
the paper only for the D1Q2 comparison of Sec. 3.1) is available as
fused_taylor: Y = (1 - tau_ext) S + tau_sca M S + dt J.

Dichroic absorption (see dichroic_absorption) multiplies the two linear
polarisations along the meridian axes by their own absorption factors before
the scattering.

Phase-function mixtures (the per-cell aerosol / cloud fractions that the
paper's conclusion names as the next step, Sec. 4): further collision
matrices M_1 .. M_{K-1} and per-cell fractions f_k >= 0 with sum_k f_k <= 1
of the scattering that follows each, the first matrix taking the rest:
Y = alpha X + beta ((1 - sum_k f_k) M X + sum_k f_k M_k X).  The
redistribution of a cell is the fraction-weighted mixture of K phase
functions, each normalised as in Eq. 17 (K = 2: (1 - f) M X + f M2 X).
"""
import math
import numpy as np

from . import directions as _dirs
from . import phase as _phase

BC_PERIODIC, BC_ABSORBING, BC_INFLOW = 0, 1, 2
EDGE_XM, EDGE_XP, EDGE_YM, EDGE_YP = 0, 1, 2, 3


class Problem:
    """Everything one solve needs, in float64."""

    def __init__(self, nx, ny, dirs, shifts, M, dt, bc, tau, albedo, emis,
                 jprof, inflow=None, abs_taylor=False, scat_exp=False,
                 fused_taylor=False, M2=None, frac=None, dichroism=None):
        self.nx, self.ny = int(nx), int(ny)
        self.dirs = dirs
        self.n = dirs.n
        self.shifts = np.asarray(shifts, dtype=np.float64)
        self.M = np.asarray(M, dtype=np.float64)
        self.dt = float(dt)
        self.bc = tuple(int(b) for b in bc)
        self.tau = np.asarray(tau, dtype=np.float64).reshape(self.ny, self.nx)
        self.albedo = np.asarray(albedo, dtype=np.float64).reshape(self.ny, self.nx)
        self.emis = np.asarray(emis, dtype=np.float64).reshape(self.ny, self.nx)
        self.jprof = np.asarray(jprof, dtype=np.float64).reshape(self.n, 4)
        if inflow is None:
            inflow = np.zeros((4, self.n, 4))
        inflow = np.asarray(inflow, dtype=np.float64)
        # inflow radiance: uniform along each edge [4][n][4], or per edge cell
        # [2 nx + 2 ny][n][4] in the order x- (y = 0..ny-1), x+ (y), y- (x =
        # 0..nx-1), y+ (x); stored per edge cell either way
        npe = 2 * (self.nx + self.ny)
        if inflow.size == 4 * self.n * 4 and inflow.size != npe * self.n * 4:
            inflow = inflow.reshape(4, self.n, 4)
            counts = (self.ny, self.ny, self.nx, self.nx)
            inflow = np.concatenate([np.repeat(inflow[e:e + 1], counts[e], axis=0) for e in range(4)])
        self.inflow_cells = inflow.reshape(npe, self.n, 4)
        self.edge_base = (0, self.ny, 2 * self.ny, 2 * self.ny + self.nx)
        self.abs_taylor = bool(abs_taylor)
        self.scat_exp = bool(scat_exp)
        self.fused_taylor = bool(fused_taylor)
        if (self.bc[0] == BC_PERIODIC) != (self.bc[1] == BC_PERIODIC):
            raise ValueError("x edges must both be periodic or neither")
        if (self.bc[2] == BC_PERIODIC) != (self.bc[3] == BC_PERIODIC):
            raise ValueError("y edges must both be periodic or neither")
        self.alpha, self.beta = coefficients(self.tau, self.albedo, self.abs_taylor,
                                             self.scat_exp, self.fused_taylor)
        # optional phase mixture: M2 is one further collision matrix (frac
        # [ny, nx]) or a sequence of K - 1 of them (frac [K - 1, ny, nx])
        self.mix_M, self.mix_f = None, None
        if M2 is not None:
            Ms = [M2] if np.ndim(M2) == 2 else list(M2)
            if not Ms:
                raise ValueError("a mixture needs at least one further phase function")
            self.mix_M = [np.asarray(m, dtype=np.float64) for m in Ms]
            k = len(self.mix_M)
            f = np.zeros((k, self.ny, self.nx)) if frac is None else frac
            self.mix_f = np.asarray(f, dtype=np.float64).reshape(k, self.ny, self.nx)
            if (np.any(~np.isfinite(self.mix_f)) or np.any(self.mix_f < 0.0)
                    or np.any(self.mix_f.sum(axis=0) > 1.0)):
                raise ValueError("mixture fractions must be >= 0 with a sum <= 1 per cell")
        # optional dichroic absorption: per-cell linear dichroism eta
        self.eta = None
        if dichroism is not None:
            self.eta = np.asarray(dichroism, dtype=np.float64).reshape(self.ny, self.nx)
            if np.any(~np.isfinite(self.eta)) or np.any(np.abs(self.eta) >= 1.0):
                raise ValueError("dichroism eta must satisfy |eta| < 1")
            if self.abs_taylor or self.fused_taylor:
                raise ValueError("dichroic absorption is defined for Beer-Lambert absorption")

    @property
    def M2(self):
        """The first further matrix of a phase mixture (None without one);
        setting None removes the mixture."""
        return None if self.mix_M is None else self.mix_M[0]

    @M2.setter
    def M2(self, value):
        if value is not None:
            raise ValueError("a mixture is given to the constructor")
        self.mix_M, self.mix_f = None, None

    @property
    def frac(self):
        """Per-cell fraction of the first further matrix (None without a mixture)."""
        return None if self.mix_f is None else self.mix_f[0]

    @property
    def shape(self):
        return (self.n, 4, self.ny, self.nx)

    def emission_field(self):
        """J[d, s, y, x] = emis[y, x] * jprof[d, s]."""
        return self.jprof[:, :, None, None] * self.emis[None, None, :, :]


def coefficients(tau, albedo, abs_taylor=False, scat_exp=False, fused_taylor=False):
    """Per-cell (alpha, beta) with Y = alpha X + beta M X.

    Split form: a = exp(-tau_abs) (Taylor: 1 - tau_abs), s = 1 - tau_sca
    (Eq. 11; scat_exp: exp(-tau_sca)), alpha = a s, beta = a (1 - s).
    Eq. 31 needs the survival weight to be non-negative, so s < 0 is refused.
    Fused Taylor (literal Eq. 2): alpha = 1 - tau_ext, beta = tau_sca.
    """
    tau = np.asarray(tau, dtype=np.float64)
    alb = np.asarray(albedo, dtype=np.float64)
    if np.any(~np.isfinite(tau)) or np.any(tau < 0):
        raise ValueError("tau_ext must be finite and >= 0")
    if np.any(~np.isfinite(alb)) or np.any(alb < 0) or np.any(alb > 1):
        raise ValueError("albedo must lie in [0, 1]")
    t_sca = alb * tau
    t_abs = (1.0 - alb) * tau
    if fused_taylor:
        alpha = 1.0 - tau
        beta = t_sca
        if np.any(alpha < 0):
            raise ValueError("fused Taylor form needs tau_ext <= 1")
        return alpha, beta
    a = 1.0 - t_abs if abs_taylor else np.exp(-t_abs)
    if np.any(a < 0):
        raise ValueError("Taylor absorption needs tau_abs <= 1")
    s = np.exp(-t_sca) if scat_exp else 1.0 - t_sca
    if np.any(s < 0):
        raise ValueError("survival 1 - tau_sca < 0 (Eq. 31 needs it >= 0)")
    return a * s, a * (1.0 - s)


def coefficient_derivatives(tau, albedo, abs_taylor=False, scat_exp=False,
                            fused_taylor=False):
    """d(alpha, beta)/d(tau, albedo), by the chain rule on the expressions above."""
    tau = np.asarray(tau, dtype=np.float64)
    alb = np.asarray(albedo, dtype=np.float64)
    if fused_taylor:
        one = np.ones_like(tau)
        return (-one, np.zeros_like(tau), alb * one, tau * one)
    t_abs = (1.0 - alb) * tau
    t_sca = alb * tau
    if abs_taylor:
        a = 1.0 - t_abs
        da_dt, da_dw = -(1.0 - alb), tau
    else:
        a = np.exp(-t_abs)
        da_dt, da_dw = -(1.0 - alb) * a, tau * a
    if scat_exp:
        s = np.exp(-t_sca)
        ds_dt, ds_dw = -alb * s, -tau * s
    else:
        s = 1.0 - t_sca
        ds_dt, ds_dw = -alb, -tau
    dal_dt = da_dt * s + a * ds_dt
    dal_dw = da_dw * s + a * ds_dw
    dbe_dt = da_dt * (1.0 - s) - a * ds_dt
    dbe_dw = da_dw * (1.0 - s) - a * ds_dw
    return dal_dt, dal_dw, dbe_dt, dbe_dw


def _taps(l):
    """Bilinear taps of Eq. 34 along one axis: [(offset, weight), ...].

    Base shift floor(l) and fraction f = l - floor(l) in [0, 1); the pull
    form reads f(x - offset) with offset in {floor(l), floor(l) + 1} and
    weights (1 - f, f).  Zero-weight taps are dropped.
    """
    i0 = math.floor(l)
    f = l - i0
    taps = []
    if 1.0 - f != 0.0:
        taps.append((i0, 1.0 - f))
    if f != 0.0:
        taps.append((i0 + 1, f))
    return taps


def _fetch(plane, xs, ys, d, prob):
    """plane[4, ny, nx] read at integer (xs, ys) with the edge rules.

    Periodic axes wrap.  A point still outside the lattice is a ghost: if it
    is outside in y the y edge it crossed decides, otherwise the x edge;
    absorbing ghosts are zero, inflow ghosts carry the inflow radiance of
    direction d at the edge cell the point lies beyond (its x on a y edge,
    clamped to the lattice at the corners; its y on an x edge).
    """
    nx, ny = prob.nx, prob.ny
    if prob.bc[EDGE_XM] == BC_PERIODIC:
        xs = np.mod(xs, nx)
    if prob.bc[EDGE_YM] == BC_PERIODIC:
        ys = np.mod(ys, ny)
    inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny)
    vals = np.zeros((4,) + xs.shape)
    vals[:, inside] = plane[:, ys[inside], xs[inside]]
    above = ys >= ny
    below = ys < 0
    left = (xs < 0) & ~above & ~below
    right = (xs >= nx) & ~above & ~below
    for mask, edge in ((above, EDGE_YP), (below, EDGE_YM), (left, EDGE_XM),
                       (right, EDGE_XP)):
        if prob.bc[edge] == BC_INFLOW and np.any(mask):
            pos = np.clip(xs[mask], 0, nx - 1) if edge in (EDGE_YM, EDGE_YP) else ys[mask]
            vals[:, mask] = prob.inflow_cells[prob.edge_base[edge] + pos, d, :].T
    return vals


def stream(Y, prob):
    """S'[d](x, y) = sum_{bx,by} wx wy Y[d](x - i0 - bx, y - j0 - by), Eq. 34."""
    out = np.zeros_like(Y)
    yy, xx = np.meshgrid(np.arange(prob.ny), np.arange(prob.nx), indexing="ij")
    for d in range(prob.n):
        lx, ly = prob.shifts[d]
        for ox, wx in _taps(lx):
            for oy, wy in _taps(ly):
                out[d] += wx * wy * _fetch(Y[d], xx - ox, yy - oy, d, prob)
    return out


def stream_transpose(G, prob):
    """Transpose of the linear part of stream(): scatter-add of the pull.

    The forward gathers Y at source (xs, ys) into target (x, y) with weight w;
    the transpose adds w * G[target] into source, for in-lattice sources only
    (ghost values are constants and carry no gradient).
    """
    out = np.zeros_like(G)
    nx, ny = prob.nx, prob.ny
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for d in range(prob.n):
        lx, ly = prob.shifts[d]
        for ox, wx in _taps(lx):
            for oy, wy in _taps(ly):
                xs, ys = xx - ox, yy - oy
                if prob.bc[EDGE_XM] == BC_PERIODIC:
                    xs = np.mod(xs, nx)
                if prob.bc[EDGE_YM] == BC_PERIODIC:
                    ys = np.mod(ys, ny)
                inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny)
                for s in range(4):
                    np.add.at(out[d, s], (ys[inside], xs[inside]),
                              wx * wy * G[d, s][inside])
    return out


def dichroic_absorption(X, prob):
    """Polarisation-dependent part of the absorption (dichroic absorption,
    named as missing in the paper's conclusions).

    The absorption optical depth of direction d becomes the matrix
    tau_abs K_d with K_d = [[1, eta w_d, 0, 0], [eta w_d, 1, 0, 0], [0, 0, 1, 0],
    [0, 0, 0, 1]] in the meridian axes, w_d = sin^2 theta_d (aligned
    particles with their symmetry axis along z: no dichroism along z), so the
    absorption factor exp(-tau_abs K_d) acts on the two linear polarisations
    along e_theta (I + Q) and e_phi (I - Q) as exp(-tau_abs (1 +- eta w_d)).
    The scalar part exp(-tau_abs) is in alpha and beta; this returns X with
    the remaining factors exp(-+tau_abs eta w_d) applied to I +- Q.
    """
    tau_abs = ((1.0 - prob.albedo) * prob.tau * prob.eta).reshape(1, -1)
    w = np.sin(prob.dirs.theta) ** 2
    Xd = X.reshape(prob.n, 4, -1).copy()
    plus = (Xd[:, 0] + Xd[:, 1]) * np.exp(-tau_abs * w[:, None])
    minus = (Xd[:, 0] - Xd[:, 1]) * np.exp(tau_abs * w[:, None])
    Xd[:, 0] = 0.5 * (plus + minus)
    Xd[:, 1] = 0.5 * (plus - minus)
    return Xd.reshape(X.shape)


def scatter_product(prob, X, transpose=False):
    """M X per cell, or with a phase mixture (1 - sum_k f_k) M X + sum_k
    f_k M_k X; with transpose the same with M^T and M_k^T (the adjoint)."""
    op = (lambda A: A.T) if transpose else (lambda A: A)  # noqa: E731
    P = op(prob.M) @ X
    if prob.mix_M is not None:
        f = prob.mix_f.reshape(len(prob.mix_M), 1, -1)
        P = (1.0 - f.sum(axis=0)) * P
        for k, Mk in enumerate(prob.mix_M):
            P = P + f[k] * (op(Mk) @ X)
    return P


def collide(S, prob):
    """Emission, absorption and scattering at every cell (steps 1-3)."""
    n = prob.n
    C = prob.nx * prob.ny
    J = prob.emission_field()
    e = 0.0 if prob.fused_taylor else 1.0
    X = (S + e * prob.dt * J).reshape(4 * n, C)
    if prob.eta is not None:
        # absorption precedes scattering: the dichroic factor acts on X
        X = dichroic_absorption(X, prob)
    al = prob.alpha.reshape(1, C)
    be = prob.beta.reshape(1, C)
    MX = scatter_product(prob, X)
    Y = al * X + be * MX
    Y = Y.reshape(prob.shape)
    if prob.fused_taylor:
        Y = Y + prob.dt * J
    return Y


def step(S, prob):
    """One full step: S_{t+1} = L(collide(S_t))."""
    return stream(collide(S, prob), prob)


def run(S0, prob, nsteps, keep=False):
    """nsteps steps from S0; with keep=True also returns [S_0, ..., S_T]."""
    S = np.array(S0, dtype=np.float64).reshape(prob.shape)
    hist = [S.copy()] if keep else None
    for _ in range(nsteps):
        S = step(S, prob)
        if keep:
            hist.append(S.copy())
    return (S, hist) if keep else S


# ----------------------------------------------------------------- readout --

def outgoing_directions(prob, edge):
    """Directions whose displacement leaves the lattice through `edge`."""
    lx, ly = prob.shifts[:, 0], prob.shifts[:, 1]
    sel = {EDGE_XM: lx < 0, EDGE_XP: lx > 0, EDGE_YM: ly < 0, EDGE_YP: ly > 0}[edge]
    return np.nonzero(sel)[0]


def readout(S, prob, edge):
    """Stokes vectors of the outgoing directions on the edge row/column.

    Returns out[e, k, s]: e runs along the edge (x for y edges, y for x
    edges), k over outgoing_directions(edge) in increasing d.
    """
    dsel = outgoing_directions(prob, edge)
    if edge == EDGE_YP:
        blk = S[dsel, :, prob.ny - 1, :]
    elif edge == EDGE_YM:
        blk = S[dsel, :, 0, :]
    elif edge == EDGE_XP:
        blk = S[dsel, :, :, prob.nx - 1]
    else:
        blk = S[dsel, :, :, 0]
    return np.transpose(blk, (2, 0, 1)).copy()


def dop(I, Q, U, V):
    """Degree of polarisation sqrt(Q^2+U^2+V^2)/I (Sec. 3.2.1, numbered 36); 0 where I = 0."""
    I = np.asarray(I, dtype=np.float64)
    num = np.sqrt(np.asarray(Q) ** 2 + np.asarray(U) ** 2 + np.asarray(V) ** 2)
    out = np.zeros_like(I)
    nz = I > 0
    out[nz] = num[nz] / I[nz]
    return out


def dolp(I, Q, U, eps=1e-6):
    """Degree of linear polarisation, regularised: sqrt(Q^2+U^2+(eps I)^2)/I."""
    I = np.asarray(I, dtype=np.float64)
    return np.sqrt(np.asarray(Q) ** 2 + np.asarray(U) ** 2 + (eps * I) ** 2) / I


def maps(S):
    """Direction-mean intensity and direction-mean per-direction DOP per cell."""
    I_mean = S[:, 0].mean(axis=0)
    dop_mean = dop(S[:, 0], S[:, 1], S[:, 2], S[:, 3]).mean(axis=0)
    return I_mean, dop_mean


def totals(S):
    """Sums of I, Q, U, V over all cells and directions."""
    return S.sum(axis=(0, 2, 3))


def edge_loss(S, prob, edge, eps=1e-6):
    """Sum over the edge and its outgoing directions of (I + DoLP), and dL/dS."""
    out = readout(S, prob, edge)
    I, Q, U = out[..., 0], out[..., 1], out[..., 2]
    r = np.sqrt(Q * Q + U * U + (eps * I) ** 2)
    loss = float(np.sum(I + r / I))
    g = np.zeros_like(out)
    g[..., 0] = 1.0 + (eps * eps * I / r) / I - r / (I * I)
    g[..., 1] = Q / (r * I)
    g[..., 2] = U / (r * I)
    return loss, g


def readout_transpose(g, prob, edge):
    """Scatter a readout gradient g[e, k, s] back into a full state-shaped array."""
    G = np.zeros(prob.shape)
    dsel = outgoing_directions(prob, edge)
    blk = np.transpose(g, (1, 2, 0))
    if edge == EDGE_YP:
        G[dsel, :, prob.ny - 1, :] = blk
    elif edge == EDGE_YM:
        G[dsel, :, 0, :] = blk
    elif edge == EDGE_XP:
        G[dsel, :, :, prob.nx - 1] = blk
    else:
        G[dsel, :, :, 0] = blk
    return G


# ------------------------------------------------------------ construction --

def mixture_matrices(dirs, spec):
    """The further collision matrices of spec["mixture"]: None, one matrix
    for a single phase function (a dict), a list for a list of them."""
    mix = spec.get("mixture")
    if mix is None:
        return None

    def build(ph):
        return _phase.collision_matrix(dirs, ph.get("kind", "rayleigh"), ph.get("g", 0.0),
                                       ph.get("mix_ray", 1.0), spec.get("renorm_irow", False),
                                       spec.get("scalar", False), ph.get("table"))
    return build(mix) if isinstance(mix, dict) else [build(ph) for ph in mix]


def make_problem(spec, medium):
    """Build a Problem from a workload spec and a medium (see workloads)."""
    if spec.get("dir_xyz") is not None:
        dirs = _dirs.VectorDirectionSet(spec["dir_xyz"], spec.get("dir_domega"))
    else:
        dirs = _dirs.make_directions(spec["n_zen"], spec["n_az"], spec.get("zen_rule", "equal_area"),
                                     spec.get("az_offset_deg", 0.0), spec.get("zen_explicit_deg"))
        if spec.get("dir_domega") is not None:
            dirs.domega = np.asarray(spec["dir_domega"], dtype=np.float64).reshape(dirs.n).copy()
    if spec.get("shift") is not None:
        shifts = _dirs.snap_integers(np.asarray(spec["shift"], dtype=np.float64).reshape(dirs.n, 2))
        if np.any(np.abs(shifts) > 1.0 + 1e-12):
            raise ValueError("|l| > 1 per step")
    else:
        shifts = _dirs.displacements(dirs, spec["plane"], spec.get("courant", 1.0))
    ph = spec.get("phase", {"kind": "rayleigh"})
    M = _phase.collision_matrix(dirs, ph.get("kind", "rayleigh"), ph.get("g", 0.0),
                                ph.get("mix_ray", 1.0), spec.get("renorm_irow", False),
                                spec.get("scalar", False), ph.get("table"))
    return Problem(spec["nx"], spec["ny"], dirs, shifts, M, spec.get("dt", 1.0), spec["bc"],
                   medium["tau"], medium["albedo"], medium["emis"], medium["jprof"],
                   medium.get("inflow"), spec.get("abs_taylor", False),
                   spec.get("scat_exp", False), spec.get("fused_taylor", False),
                   M2=mixture_matrices(dirs, spec), frac=medium.get("frac"), dichroism=medium.get("eta"))
