"""Shared helpers of the GPU parity tests: build a device solver and the
oracle problem from one seeded workload description, and compare fields."""
import numpy as np
import torch

import workloads as W
from oracle import lbm as OL

# Tolerances on the normwise relative error per Stokes component (float32
# state throughout; bf16 / fp16 only in the contraction operands).  The 2e-3
# bf16/fp16 bound holds where the scattered share per step is small
# (beta <= 0.2, the regime of the optically thin per-step media); for
# scattering-dominated media (beta up to 0.8) the contraction's operand
# rounding (2^-9 for bf16) enters every step at full weight and the bound is
# 1e-2; bf16x3 keeps about 16 mantissa bits and is held to 5e-5 there.
TOL = {"fp32": 1e-5, "plain": 1e-5, "bf16x3": 1e-5, "bf16": 2e-3, "fp16": 2e-3}
TOL_THICK = {"fp32": 1e-5, "plain": 1e-5, "bf16x3": 5e-5, "bf16": 1e-2, "fp16": 1e-2}
# gradients: float32 paths 1e-4; the bf16 adjoint 1e-2
GTOL = {"fp32": 1e-4, "plain": 1e-4, "bf16x3": 1e-4, "bf16": 1e-2, "fp16": 1e-2}
# a polarised component smaller than this fraction of the intensity norm is
# judged on the intensity scale (float32 rounding of the intensity-sized
# terms that combine into it bounds its absolute accuracy)
POL_FLOOR = 1e-2


def tolerance(precision, oprob):
    return (TOL if float(oprob.beta.max()) <= 0.2 else TOL_THICK)[precision]


def build(spec, precision="fp32", medium=None):
    import paper_2609_23057_amd as P
    plain = precision == "plain"
    s = dict(spec)
    s["precision"] = "fp32" if plain else precision
    s["plain"] = plain
    prob = P.make_problem(**s)
    solver = P.Solver(prob)
    med = W.medium(spec) if medium is None else medium
    dev = solver.device
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    tensors = (t(med["tau"]), t(med["albedo"]), t(med["emis"]))
    solver.set_medium(*tensors, med["jprof"], med["inflow"])
    solver._tensors = tensors
    oprob = OL.make_problem(spec, med)
    return solver, oprob, med


def to_dev(a, solver):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=solver.device)


def to_np(t):
    return t.detach().cpu().double().numpy()


def stokes_errors(got, ref):
    """Normwise relative error per Stokes component, max-abs / max |ref|, and
    the largest absolute DoLP error over cells with I > 1e-3 max I.

    The scale of Q, U, V is max(own norm, POL_FLOOR * ||I||).
    """
    out = {}
    nI = np.linalg.norm(ref[:, 0])
    for s, name in enumerate("IQUV"):
        den = max(np.linalg.norm(ref[:, s]), POL_FLOOR * nI if s else 0.0, 1e-300)
        out[name] = float(np.linalg.norm(got[:, s] - ref[:, s]) / den)
    out["maxabs"] = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
    I = ref[:, 0]
    m = I > 1e-3 * I.max() if I.max() > 0 else np.zeros_like(I, dtype=bool)
    if np.any(m):
        dr = np.sqrt(ref[:, 1] ** 2 + ref[:, 2] ** 2)[m] / I[m]
        dg = np.sqrt(got[:, 1] ** 2 + got[:, 2] ** 2)[m] / np.maximum(got[:, 0][m], 1e-300)
        out["dolp_abs"] = float(np.abs(dg - dr).max())
    else:
        out["dolp_abs"] = 0.0
    return out


def assert_close(got, ref, tol, what=""):
    e = stokes_errors(got, ref)
    bad = {k: v for k, v in e.items() if k in "IQUV" and v > tol}
    assert not bad and e["maxabs"] < 10 * tol and e["dolp_abs"] < 10 * tol, (what, e)
    return e


def _bf16(a):
    """Round to bfloat16 through float32, to nearest even, as the fragment
    packer does."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def represented(M, precision, scale_of=None):
    """The collision matrix as a 16-bit contraction holds it: bf16, bf16 high
    + low parts (bf16x3), or fp16 (through float32) after the power-of-two
    scale that puts max |scale_of| in [2^12, 2^13) (scale_of = M itself by
    default; a mixture's second matrix takes the first one's scale)."""
    if precision == "bf16":
        return _bf16(M)
    if precision == "bf16x3":
        hi = _bf16(M)
        return hi + _bf16(M - hi)
    if precision == "fp16":
        e = np.frexp(np.abs(M if scale_of is None else scale_of).max())[1]
        sc = 2.0 ** (13 - e)
        return np.asarray(M * sc, dtype=np.float32).astype(np.float16).astype(np.float64) / sc
    return M
