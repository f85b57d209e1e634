"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module only describes problems and draws random inputs: lattice sizes,
direction-grid parameters, boundary kinds, phase-function parameters, per-cell
optical depth / albedo / emission fields, boundary radiances and initial
states.  It contains none of the solver's arithmetic (no directions, phase
matrices, coefficients or streaming); the oracle and the HIP library each build
those themselves from the description.

Every random field is rounded to float32 and returned as float64, so that the
float32 device path and the float64 oracle see bit-identical inputs.

Workloads (the paper's method at the sizes it is benchmarked on here):
  qlbm16       16x16 absorbing, n = 8 (2 zenith x 4 azimuth, D2Q9 shifts), the
               paper's 2-D circuit experiment (statevector emulation)
  plain32      32x32 periodic, n = 8 (2 zenith x 4 azimuth, D2Q9 shifts),
               tau_ext = 1 per step, albedo 0.9, Rayleigh, unpolarised unit
               point source at the centre, 100 steps
  beam512      512x512 vertical plane, n = 32 (4 x 8), lognormal extinction,
               albedo U[0.8, 1], HG(g = 0.7) weights with Rayleigh-shaped
               polarisation, unpolarised beam at solar zenith 30 deg entering
               the top, vacuum sides and bottom, 2000 steps
  prec1024     1024x1024, n = 128 (8 x 16), the beam512 generator, 200 steps
  adjoint256   256x256, n = 32, beam512 generator plus emission U[0, 0.05],
               top-edge (I + DoLP) loss after 500 steps
  (any)        with mixture={phase}: a second phase function and a per-cell
               fraction U[0, 1] of the scattering that follows it; with
               mixture=[{phase}, ...] (K - 1 further phase functions): per-cell
               fractions of all K drawn from the flat Dirichlet distribution,
               frac [K - 1, ny, nx] for the further ones (their sum <= 1)
  (any)        with dichroism=d: a per-cell linear dichroism eta ~ U[-d, d]
               of the absorption
  (any)        with phase={"kind": "table", "table": scattering_table()}: a
               tabulated scattering matrix of an aerosol-like particle
               (forward peak, P12 < 0 at side angles, P34 != 0)
  beam3d       256x256x64 three-dimensional lattice (z = altitude), n = 32,
               the beam512 medium generator at the per-step optical depth of
               a 512 lattice (the 4.2M draws of a 256 one reach tau_sca > 1),
               beam entering the top face z+, absorbing side and bottom
               faces, 500 steps
  spectral64   64 channels 400-900 nm, Rayleigh optical depth ~ lambda^-4 plus
               aerosol HG(0.6), per-channel lattice and direction count drawn
               from {128,256,384,512}^2 x {16,32,64}, 200 steps
"""
import copy
import numpy as np

BC_PERIODIC, BC_ABSORBING, BC_INFLOW = 0, 1, 2

_BASE = {
    "plain32": dict(nx=32, ny=32, n_zen=2, n_az=4, zen_rule="equal_area", az_offset_deg=0.0,
                    plane="xy_d2q9", courant=1.0, bc=(0, 0, 0, 0),
                    phase={"kind": "rayleigh"}, dt=1.0, steps=100, seed=1,
                    medium="uniform", tau0=1.0, albedo0=0.9, source="point"),
    "beam512": dict(nx=512, ny=512, n_zen=4, n_az=8, zen_rule="equal_area", az_offset_deg=0.0,
                    plane="xz", courant=1.0, bc=(1, 1, 1, 2),
                    phase={"kind": "hg", "g": 0.7}, dt=1.0, steps=2000, seed=2,
                    medium="lognormal", tau_ref_n=512, beam_dir=3 * 8 + 0, source="none"),
    "prec1024": dict(nx=1024, ny=1024, n_zen=8, n_az=16, zen_rule="equal_area",
                     az_offset_deg=0.0, plane="xz", courant=1.0, bc=(1, 1, 1, 2),
                     phase={"kind": "hg", "g": 0.7}, dt=1.0, steps=200, seed=3,
                     medium="lognormal", tau_ref_n=1024, beam_dir=6 * 16 + 0,
                     source="none"),
    "beam3d": dict(nx=256, ny=256, nz=64, n_zen=4, n_az=8, zen_rule="equal_area", az_offset_deg=0.0,
                   plane="3d", courant=1.0, bc6=(1, 1, 1, 1, 1, 2),
                   phase={"kind": "hg", "g": 0.7}, dt=1.0, steps=500, seed=7,
                   medium="lognormal", tau_ref_n=512, beam_dir=3 * 8 + 0, source="none"),
    # the paper's 2-D experiment (Sec. 3.2.1): 16 x 16 D2Q9 lattice, 2 x 4
    # directions, Rayleigh scattering, k_ext = 2.5, k_scat = 0.5 in the unit
    # domain (dt = 1/16: tau_ext = 2.5/16 per step, albedo 0.2), a source
    # over the central +-25% of the domain with unit emission summed over the
    # directions, absorbing edges
    "qlbm16": dict(nx=16, ny=16, n_zen=2, n_az=4, zen_rule="equal_area", az_offset_deg=0.0,
                   plane="xy_d2q9", courant=1.0, bc=(1, 1, 1, 1), phase={"kind": "rayleigh"},
                   dt=1.0 / 16.0, steps=4, seed=8, medium="uniform", tau0=2.5 / 16.0, albedo0=0.2,
                   source="box"),
    "adjoint256": dict(nx=256, ny=256, n_zen=4, n_az=8, zen_rule="equal_area",
                       az_offset_deg=0.0, plane="xz", courant=1.0, bc=(1, 1, 1, 2),
                       phase={"kind": "hg", "g": 0.7}, dt=1.0, steps=500, seed=4,
                       medium="lognormal", tau_ref_n=256, beam_dir=3 * 8 + 0,
                       source="uniform_emis",
                       emis_max=0.05, loss_edge=3),
}
# beam_dir: index d = i_zen * n_az + j_az of the downward direction nearest to
# propagation zenith 150 deg (solar zenith 30 deg) at azimuth 0.  Equal-area
# zeniths for n_zen = 4 are 41.4/75.5/104.5/138.6 deg (i = 3 is nearest), for
# n_zen = 8 the nearest is i = 6 (144.3 deg), for n_zen = 2 it is i = 1 (120 deg).
BEAM_ZEN_INDEX = {2: 1, 4: 3, 8: 6}


def spec(name, **over):
    """A workload description (dict) with optional overrides."""
    s = copy.deepcopy(_BASE[name])
    s["name"] = name
    s.update(over)
    if "beam_dir" in s and ("n_zen" in over or "n_az" in over):
        s["beam_dir"] = BEAM_ZEN_INDEX[s["n_zen"]] * s["n_az"]
    return s


def ndir(s):
    return int(s["n_zen"]) * int(s["n_az"])


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def medium(s, seed=None):
    """Per-cell tau_ext (per-step optical depth), albedo, emission; jprof; inflow.

    Arrays are [ny, nx]; jprof [n, 4]; inflow [4 edges, n, 4].
    lognormal: tau = tau_scale * exp(N(0,1)) / N with N the full-size lattice
    side tau_ref_n (unit domain, dt = 1/N as in Sec. 3.2.2), so a reduced test
    lattice keeps the per-step optical-depth distribution; albedo ~ U[0.8, 1].
    """
    rng = np.random.default_rng(s["seed"] if seed is None else seed)
    nx, n = s["nx"], ndir(s)
    nz = int(s.get("nz", 1))
    three_d = s.get("plane") == "3d"
    # a 3-D lattice draws its per-cell fields as nz * ny rows of nx cells
    # (the draws are independent per cell) and returns them as [nz, ny, nx]
    ny = s["ny"] * nz if three_d else s["ny"]
    if s["medium"] == "uniform":
        tau = np.full((ny, nx), s["tau0"])
        alb = np.full((ny, nx), s["albedo0"])
    elif s["medium"] == "lognormal":
        tau = (np.exp(rng.normal(0.0, 1.0, size=(ny, nx))) * s.get("tau_scale", 1.0)
               / s.get("tau_ref_n", ny))
        alb = rng.uniform(0.8, 1.0, size=(ny, nx))
    else:
        raise ValueError(s["medium"])
    emis = np.zeros((ny, nx))
    jprof = np.zeros((n, 4))
    src = s.get("source", "none")
    if src == "point":
        y, x = s.get("source_cell") or (ny // 2, nx // 2)
        emis[y, x] = 1.0
        jprof[:, 0] = 1.0 / n
        if s.get("source_pol") == "linear":
            jprof[:, 1] = 1.0 / n
    elif src == "box":
        # the central half of the lattice in each axis, unit emission summed
        # over the directions; linear polarisation along e_theta if asked
        y0, y1 = ny // 4, ny - ny // 4
        x0, x1 = nx // 4, nx - nx // 4
        emis[y0:y1, x0:x1] = 1.0
        jprof[:, 0] = 1.0 / n
        if s.get("source_pol") == "linear":
            jprof[:, 1] = 1.0 / n
    elif src == "uniform_emis":
        emis = rng.uniform(0.0, s["emis_max"], size=(ny, nx))
        jprof[:, 0] = 1.0
    if three_d:
        inflow = np.zeros((6, n, 4))
        if "beam_dir" in s and s["bc6"][5] == BC_INFLOW:
            inflow[5, s["beam_dir"], 0] = 1.0
    else:
        inflow = np.zeros((4, n, 4))
        if "beam_dir" in s and s["bc"][3] == BC_INFLOW:
            inflow[3, s["beam_dir"], 0] = 1.0
    # phase mixture: per-cell fraction of the scattering that follows the
    # second phase function (drawn after everything else, so the other
    # fields do not depend on whether a mixture is asked for)
    frac = None
    if isinstance(s.get("mixture"), dict):
        frac = _f32(rng.uniform(0.0, 1.0, size=(ny, nx)))
    elif s.get("mixture") is not None:
        # flat Dirichlet over the K components (normalised exponential
        # draws); the further K - 1 shares are kept, shrunk by 2^-20 so that
        # their float32 values still sum to at most 1
        k = len(s["mixture"])
        e = -np.log1p(-rng.uniform(0.0, 1.0, size=(k + 1, ny, nx)))
        frac = _f32(e[1:] / e.sum(axis=0) * (1.0 - 2.0 ** -20))
        assert np.all(frac.astype(np.float64).sum(axis=0) <= 1.0)
    # dichroic absorption: per-cell linear dichroism eta ~ U[-d, d], d < 1
    # (drawn last for the same reason)
    eta = None
    if s.get("dichroism") is not None:
        d = float(s["dichroism"])
        eta = _f32(rng.uniform(-d, d, size=(ny, nx)))
    out = {"tau": _f32(tau), "albedo": _f32(alb), "emis": _f32(emis),
           "jprof": _f32(jprof), "inflow": _f32(inflow), "frac": frac, "eta": eta}
    if three_d:
        for k in ("tau", "albedo", "emis", "frac", "eta"):
            if out[k] is not None:
                out[k] = out[k].reshape(out[k].shape[:-2] + (nz, s["ny"], nx))
    return out


def initial_state(s, kind="zero", seed=None):
    """S0[d, s, y, x] (S0[d, s, z, y, x] on a 3-D lattice): zeros, or random
    physical Stokes vectors (I >= |(Q,U,V)|)."""
    nx, n = s["nx"], ndir(s)
    if s.get("plane") == "3d":
        nz = int(s.get("nz", 1))
        flat = dict(s, ny=s["ny"] * nz, plane="xz")
        return initial_state(flat, kind, seed).reshape(n, 4, nz, s["ny"], nx)
    ny = s["ny"]
    if kind == "zero":
        return np.zeros((n, 4, ny, nx))
    rng = np.random.default_rng(1000 + (s["seed"] if seed is None else seed))
    I = rng.uniform(0.1, 1.0, size=(n, ny, nx))
    v = rng.normal(size=(n, 3, ny, nx))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    p = rng.uniform(0.0, 0.99, size=(n, ny, nx))
    S = np.empty((n, 4, ny, nx))
    S[:, 0] = I
    S[:, 1:] = v * (p * I)[:, None]
    return _f32(S)


def spectral_channels(nchan=64, seed=5):
    """Per-channel descriptions for the spectral batch.

    lambda_k = 400 + 500 k / (nchan - 1) nm.  Rayleigh column optical depth
    0.1 (lambda / 550)^-4, aerosol 0.2 with HG(0.6); the phase function of a
    channel is the optical-depth-weighted mixture.  Lattice side and
    (n_zen, n_az) are drawn per channel.
    """
    rng = np.random.default_rng(seed)
    sides = [128, 256, 384, 512]
    grids = [(2, 8), (4, 8), (4, 16)]
    out = []
    for k in range(nchan):
        lam = 400.0 + 500.0 * k / max(nchan - 1, 1)   # a single channel sits at 400 nm
        t_r = 0.1 * (lam / 550.0) ** -4
        t_a = 0.2
        side = sides[rng.integers(len(sides))]
        nz, na = grids[rng.integers(len(grids))]
        s = dict(nx=side, ny=side, n_zen=nz, n_az=na, zen_rule="equal_area",
                 az_offset_deg=0.0, plane="xz", courant=1.0, bc=(1, 1, 1, 2),
                 phase={"kind": "mix", "g": 0.6, "mix_ray": t_r / (t_r + t_a)},
                 dt=1.0, steps=200, seed=5000 + k, medium="lognormal",
                 tau_scale=(t_r + t_a), tau_ref_n=side, beam_dir=BEAM_ZEN_INDEX[nz] * na,
                 source="none", name="spectral64[%d]" % k, wavelength_nm=lam)
        out.append(s)
    return out


def scattering_table(seed=6, nang=181, g=0.6):
    """A tabulated scattering matrix, rows (theta_deg, a1, a2, a3, a4, b1, b2)
    at nang angles from 0 to 180 degrees, of a synthetic single particle:
    amplitude functions S1 = sqrt(e) exp(i alpha), S2 = sqrt(e) r exp(i beta)
    with an HG(g)-shaped envelope e plus a floor, a parallel/perpendicular
    ratio r = 0.3 + 0.7 cos^2 (side-scattered light polarised), and smooth
    phase lags alpha, beta drawn from the seed, with S2 = S1 forward and
    S2 = -S1 backward (as for any particle with a symmetry plane, so the
    matrix does not depend on the scattering plane where that plane is
    undefined).  Then a1 = a2 = (|S1|^2 +
    |S2|^2) / 2, b1 = (|S2|^2 - |S1|^2) / 2, a3 = a4 = Re(S2 S1*),
    b2 = -Im(S2 S1*) (Stokes V = 2 Im(E_1 E_2*)).  This draws an input; it is
    not the solver's arithmetic.
    """
    rng = np.random.default_rng(seed)
    th = np.linspace(0.0, 180.0, nang)
    t = np.radians(th)
    c = np.cos(t)
    e = (1.0 - g * g) / (1.0 + g * g - 2.0 * g * c) ** 1.5 + 0.05
    r = 0.3 + 0.7 * c * c
    p1, p2 = rng.uniform(0.3, 0.9, size=2)
    alpha = p1 * np.sin(t)
    beta = p2 * np.sin(t) + np.pi * np.sin(0.5 * t) ** 2
    S1 = np.sqrt(e) * np.exp(1j * alpha)
    S2 = np.sqrt(e) * r * np.exp(1j * beta)
    a1 = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2)
    b1 = 0.5 * (np.abs(S2) ** 2 - np.abs(S1) ** 2)
    z = S2 * np.conj(S1)
    tab = np.stack([th, a1, a1, z.real, z.real, b1, -z.imag], axis=1)
    return _f32(tab)
