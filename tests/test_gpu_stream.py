"""Streaming alone (Sec. 2.1.6, Eq. 33-34) through rt_stream, against the
float64 oracle's pull.

A pull is a weighted sum of four source values with float32 weights, so the
device result agrees with the oracle to a few float32 roundings of the
largest source value; 2e-6 of max |Y| bounds that with room.  The
vectorised kernel (nx a multiple of 4, 16-byte aligned fields) and the
per-cell kernel perform the same arithmetic and must agree bit for bit.
"""
import types

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import build, to_dev, to_np
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

STREAM_TOL = 2e-6

CASES = [
    # name, overrides: edges, direction counts, lattices with and without nx = 0 mod 4
    ("plain32", {}),                                         # periodic, integer shifts, n = 8
    ("plain32", dict(nx=45, ny=23)),                         # periodic, nx odd
    ("beam512", dict(nx=64, ny=40)),                         # inflow top, absorbing, n = 32
    ("beam512", dict(nx=36, ny=20, n_zen=2, n_az=8)),        # n = 16
    ("beam512", dict(nx=44, ny=28, n_zen=4, n_az=16)),       # n = 64
    ("prec1024", dict(nx=24, ny=18)),                        # n = 128
    ("beam512", dict(nx=8, ny=8)),                           # every quad touches an edge
    ("beam512", dict(nx=4, ny=9)),                           # one quad per row
    ("beam512", dict(nx=33, ny=7)),                          # per-cell kernel
    ("plain32", dict(nx=12, ny=5, bc=(0, 0, 1, 2))),         # periodic x, absorbing bottom, inflow top
]


def random_field(spec, seed):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((W.ndir(spec), 4, spec["ny"], spec["nx"]))
    return Y.astype(np.float32).astype(np.float64)


def with_inflow(spec, med, seed):
    """Random radiance on every inflow edge, so the ghost path is exercised."""
    med = dict(med)
    inflow = np.zeros_like(med["inflow"])
    rng = np.random.default_rng(seed)
    for e, kind in enumerate(spec["bc"]):
        if kind == W.BC_INFLOW:
            inflow[e] = rng.uniform(0.0, 1.0, inflow[e].shape)
    med["inflow"] = inflow.astype(np.float32).astype(np.float64)
    return med


def check(got, ref, what):
    err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
    assert err <= STREAM_TOL, (what, err)
    return err


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-n%d" % (
    c[0], c[1].get("nx", W.spec(c[0])["nx"]), c[1].get("ny", W.spec(c[0])["ny"]),
    W.ndir(W.spec(c[0], **c[1]))))
def test_stream_matches_oracle(case):
    name, over = case
    spec = W.spec(name, **over)
    med = with_inflow(spec, W.medium(spec), 7)
    solver, oprob, _ = build(spec, "fp32", med)
    Y = random_field(spec, 17)
    out = torch.full(solver.shape, float("nan"), device=solver.device)
    solver.stream_field(to_dev(Y, solver), out)
    torch.cuda.synchronize()
    check(to_np(out), OL.stream(Y, oprob), case)


@pytest.mark.parametrize("nx", [64, 45])
def test_stream_vector_and_per_cell_kernels_agree_bitwise(nx):
    """A field 4 bytes off 16-byte alignment takes the per-cell kernel."""
    spec = W.spec("beam512", nx=nx, ny=30)
    med = with_inflow(spec, W.medium(spec), 3)
    solver, oprob, _ = build(spec, "fp32", med)
    Y = to_dev(random_field(spec, 5), solver)
    n = Y.numel()
    buf_in = torch.empty(n + 4, device=solver.device)
    buf_out = torch.full((n + 4,), float("nan"), device=solver.device)
    a_out = torch.full(solver.shape, float("nan"), device=solver.device)
    buf_in[1:n + 1].copy_(Y.reshape(-1))
    solver.stream_field(Y, a_out)
    solver.stream_field(buf_in[1:n + 1], buf_out[1:n + 1])
    torch.cuda.synchronize()
    assert torch.equal(a_out.reshape(-1), buf_out[1:n + 1])
    assert torch.isnan(buf_out[0]) and torch.isnan(buf_out[n + 1])


def test_stream_full_size_beam512():
    """The 512 x 512, n = 32 lattice of the fused workload, every element."""
    spec = W.spec("beam512")
    med = with_inflow(spec, W.medium(spec), 11)
    solver, oprob, _ = build(spec, "fp32", med)
    Y = random_field(spec, 23)
    out = torch.empty(solver.shape, device=solver.device)
    solver.stream_field(to_dev(Y, solver), out)
    torch.cuda.synchronize()
    check(to_np(out), OL.stream(Y, oprob), "beam512")


def test_stream_full_size_prec1024_sampled_directions():
    """1024 x 1024, n = 128: every cell of 12 directions (first, last, the
    beam direction and random ones), each against the oracle's pull of that
    direction alone."""
    spec = W.spec("prec1024")
    med = with_inflow(spec, W.medium(spec), 13)
    solver, oprob, _ = build(spec, "fp32", med)
    n = oprob.n
    rng = np.random.default_rng(29)
    Yd = torch.randn(solver.shape, device=solver.device,
                     generator=torch.Generator(device=solver.device).manual_seed(31))
    out = torch.empty(solver.shape, device=solver.device)
    solver.stream_field(Yd, out)
    torch.cuda.synchronize()
    dirs = sorted({0, n - 1, spec["beam_dir"], *[int(d) for d in rng.integers(0, n, 9)]})
    for d in dirs:
        sub = types.SimpleNamespace(n=1, nx=oprob.nx, ny=oprob.ny, bc=oprob.bc,
                                    shifts=oprob.shifts[d:d + 1], inflow_cells=oprob.inflow_cells[:, d:d + 1],
                                    edge_base=oprob.edge_base)
        ref = OL.stream(to_np(Yd[d:d + 1]), sub)
        check(to_np(out[d:d + 1]), ref, ("prec1024", d))


def test_stream_rejects_overlap_and_missing_medium():
    import paper_2609_23057_amd as P
    spec = W.spec("beam512", nx=16, ny=12)
    solver, _, _ = build(spec, "fp32")
    S = solver.empty_state()
    with pytest.raises(P.RTError):
        solver.stream_field(S, S)
    big = torch.zeros(2 * S.numel(), device=solver.device)
    with pytest.raises(P.RTError):
        solver.stream_field(big[:S.numel()], big[S.numel() // 2:S.numel() // 2 + S.numel()])
    s = dict(spec)
    s["precision"] = "fp32"
    fresh = P.Solver(P.make_problem(**s))
    with pytest.raises(P.RTError):
        fresh.stream_field(S, solver.empty_state())
