"""GPU parity of the HIP solver against the FP64 oracle, through the C ABI.

Every case runs the same seeded workload on both sides and compares the whole
field element by element (normwise relative error per Stokes component).
Sizes are chosen so the oracle finishes in seconds while the lattice still
spans several cell tiles with a ragged tail.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import lbm as OL

from gpu_common import assert_close, build, GTOL, to_dev, to_np, tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run_both(spec, precision, steps, init="zero", medium=None):
    solver, oprob, med = build(spec, precision, medium)
    S0 = W.initial_state(spec, init)
    S = to_dev(S0, solver)
    solver.run(S, steps)
    ref = OL.run(S0, oprob, steps)
    return solver, oprob, to_np(S), ref


FORWARD_CASES = [
    # name, overrides, steps, init
    ("plain32", {}, 100, "zero"),                                    # the 32x32 n=8 workload, full size
    ("plain32", dict(nx=45, ny=23, source_pol="linear"), 40, "random"),
    ("beam512", dict(nx=70, ny=37), 60, "zero"),                     # n = 32, inflow top, absorbing
    ("beam512", dict(nx=33, ny=29, n_zen=2, n_az=8), 50, "random"),  # n = 16
    ("beam512", dict(nx=21, ny=26, n_zen=4, n_az=16), 30, "random"),  # n = 64
    ("prec1024", dict(nx=19, ny=22), 25, "random"),                   # n = 128
    ("prec1024", dict(nx=16, ny=18), 20, "random"),   # 288 cells: the last 64-cell tile's second block is empty
    ("prec1024", dict(nx=96, ny=20), 20, "random"),   # rows of three 32-cell blocks, interior blocks
    ("adjoint256", dict(nx=40, ny=35), 40, "zero"),                   # emission everywhere
]


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("case", FORWARD_CASES, ids=lambda c: "%s-%dx%d-n%d" % (
    c[0], c[1].get("nx", W.spec(c[0])["nx"]), c[1].get("ny", W.spec(c[0])["ny"]),
    W.ndir(W.spec(c[0], **c[1]))))
def test_forward_parity(case, precision):
    name, over, steps, init = case
    spec = W.spec(name, **over)
    _, oprob, got, ref = _run_both(spec, precision, steps, init)
    e = assert_close(got, ref, tolerance(precision, oprob, steps), (name, precision))
    print(name, precision, e)


@pytest.mark.parametrize("opts", [dict(fused_taylor=True), dict(abs_taylor=True),
                                  dict(scat_exp=True), dict(renorm_irow=True), dict(scalar=True),
                                  dict(plane="xy", az_offset_deg=22.5, bc=(0, 0, 0, 0)),
                                  dict(plane="xy", n_az=3, bc=(0, 0, 1, 1)),
                                  dict(zen_rule="explicit", zen_explicit_deg=[30, 45, 60, 75],
                                       n_zen=4, n_az=2, plane="xz")])
@pytest.mark.parametrize("precision", ["fp32", "plain"])
def test_forward_options_parity(opts, precision):
    spec = W.spec("beam512", nx=27, ny=31, n_zen=2, n_az=4, **{k: v for k, v in opts.items()
                                                             if k not in ("n_zen", "n_az")})
    if "n_zen" in opts:
        spec["n_zen"], spec["n_az"] = opts["n_zen"], opts["n_az"]
    if opts.get("n_az") == 3:
        spec["n_az"] = 3
    med = W.medium(spec)
    med["emis"][:] = np.float32(0.01)
    med["jprof"][:, 0] = 1.0
    med["jprof"][:, 1] = np.float32(0.25)
    _, oprob, got, ref = _run_both(spec, precision, 30, "random", med)
    assert_close(got, ref, tolerance(precision, oprob), (opts, precision))


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16"])
def test_single_step_and_checkpoints(precision):
    """rt_step equals one oracle step; rt_run's checkpoints hold S_{kK}."""
    spec = W.spec("beam512", nx=50, ny=44)
    solver, oprob, med = build(spec, precision)
    S0 = W.initial_state(spec, "random")
    a = to_dev(S0, solver)
    b = solver.empty_state()
    solver.step(a, b)
    tol = tolerance(precision, oprob)
    assert_close(to_np(b), OL.step(S0, oprob), tol, "step")
    T, K = 23, 5
    ck = solver.checkpoint_buffer(T, K)
    S = to_dev(S0, solver)
    solver.run(S, T, ck, K)
    _, hist = OL.run(S0, oprob, T, keep=True)
    for k in range(ck.shape[0]):
        assert_close(to_np(ck[k]), hist[k * K], tol, ("ckpt", k))
    assert_close(to_np(S), hist[T], tol, "final")


def test_readout_sums_and_maps():
    spec = W.spec("beam512", nx=48, ny=40)
    solver, oprob, _, = build(spec, "fp32")
    S0 = W.initial_state(spec, "random")
    S = to_dev(S0, solver)
    solver.run(S, 15)
    ref = OL.run(S0, oprob, 15)
    for edge in range(4):
        out, sums = solver.readout(S, edge, sums=True)
        r = OL.readout(ref, oprob, edge)
        assert out.shape == r.shape
        assert np.abs(to_np(out) - r).max() <= 1e-5 * np.abs(r).max()
        assert np.allclose(sums, OL.totals(ref), rtol=1e-5)
    I, D = solver.maps(S)
    Io, Do = OL.maps(ref)
    assert np.abs(to_np(I) - Io).max() <= 1e-5 * Io.max()
    assert np.abs(to_np(D) - Do).max() <= 1e-4


def test_deterministic_bitwise():
    spec = W.spec("beam512", nx=64, ny=64)
    solver, _, _ = build(spec, "bf16")
    S0 = W.initial_state(spec, "random")
    outs = []
    for _ in range(2):
        S = to_dev(S0, solver)
        solver.run(S, 12)
        outs.append(S.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_set_medium_rejects_negative_survival():
    import paper_2609_23057_amd as P
    spec = W.spec("beam512", nx=16, ny=16)
    med = W.medium(spec)
    med["tau"][3, 4] = 1.5
    med["albedo"][3, 4] = 0.9
    with pytest.raises(P.RTError) as ei:
        build(spec, "fp32", med)
    assert ei.value.status == P.RT_ERANGE


# ------------------------------------------------------------------ adjoint --

def _adjoint_case(spec, precision, T, K):
    solver, oprob, med = build(spec, precision)
    S0 = np.zeros(oprob.shape)
    ck = solver.checkpoint_buffer(T, K)
    S = to_dev(S0, solver)
    solver.run(S, T, ck, K)
    ST = OL.run(S0, oprob, T)
    loss, g = OL.edge_loss(ST, oprob, 3)
    lamT = OL.readout_transpose(g, oprob, 3)
    ref = OA.adjoint(S0, oprob, T, lamT)
    g_tau, g_alb, g_em, lam0 = solver.adjoint(T, ck, K, to_dev(lamT, solver), want_lambda0=True)
    return ref, (to_np(g_tau), to_np(g_alb), to_np(g_em), to_np(lam0))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("TK", [(30, 6), (31, 6), (7, 1), (9, 9)])
def test_adjoint_parity(precision, TK):
    T, K = TK
    tol = GTOL[precision]   # the differentiation workload's medium: beta <= 0.1 per step
    spec = W.spec("adjoint256", nx=36, ny=33)
    ref, got = _adjoint_case(spec, precision, T, K)
    for key, arr in zip(("g_tau", "g_albedo", "g_emis", "lambda0"), got):
        r = ref[key]
        assert _rel(arr, r) < tol, (key, _rel(arr, r))


@pytest.mark.parametrize("over", [dict(n_zen=4, n_az=16), dict(nx=40, ny=30, n_zen=8, n_az=16),
                                  dict(bc=(0, 0, 1, 2)), dict(fused_taylor=True)])
def test_adjoint_parity_variants(over):
    spec = W.spec("adjoint256", **dict(dict(nx=30, ny=27), **over))
    ref, got = _adjoint_case(spec, "fp32", 20, 5)
    for key, arr in zip(("g_tau", "g_albedo", "g_emis", "lambda0"), got):
        assert _rel(arr, ref[key]) < 1e-4, (over, key, _rel(arr, ref[key]))


def test_autograd_function_matches_oracle_gradients():
    import paper_2609_23057_amd as P
    spec = W.spec("adjoint256", nx=32, ny=30)
    s = dict(spec)
    s["precision"] = "fp32"
    solver = P.Solver(P.make_problem(**s))
    med = W.medium(spec)
    dev = solver.device
    tau = torch.tensor(med["tau"], dtype=torch.float32, device=dev, requires_grad=True)
    alb = torch.tensor(med["albedo"], dtype=torch.float32, device=dev, requires_grad=True)
    em = torch.tensor(med["emis"], dtype=torch.float32, device=dev, requires_grad=True)
    T = 25
    out = P.RTSolve.apply(tau, alb, em, solver, solver.empty_state(), T, 3, med["jprof"], med["inflow"])
    I, Q, U = out[..., 0], out[..., 1], out[..., 2]
    loss = (I + torch.sqrt(Q * Q + U * U + (1e-6 * I) ** 2) / I).sum()
    loss.backward()
    oprob = OL.make_problem(spec, med)
    S0 = np.zeros(oprob.shape)
    ST = OL.run(S0, oprob, T)
    lo, g = OL.edge_loss(ST, oprob, 3)
    assert abs(loss.item() - lo) < 1e-5 * abs(lo)
    ref = OA.adjoint(S0, oprob, T, OL.readout_transpose(g, oprob, 3))
    assert _rel(to_np(tau.grad), ref["g_tau"]) < 1e-4
    assert _rel(to_np(alb.grad), ref["g_albedo"]) < 1e-4
    assert _rel(to_np(em.grad), ref["g_emis"]) < 1e-4


def test_plain_path_largest_direction_set():
    """n = 256 (8 x 32 directions, 4n = 1024 rows) exceeds the fused kernels;
    the plain float32 path runs it and matches the oracle, and the adjoint,
    which runs on the fused kernels, refuses it with RT_EUNSUPPORTED."""
    import paper_2609_23057_amd as P
    spec = W.spec("beam512", nx=12, ny=10, n_zen=8, n_az=32)
    solver, oprob, _ = build(spec, "plain")
    S0 = W.initial_state(spec, "random")
    S = to_dev(S0, solver)
    solver.run(S, 6)
    assert_close(to_np(S), OL.run(S0, oprob, 6), tolerance("plain", oprob), ("plain n=256",))
    S = solver.empty_state()
    ck = solver.checkpoint_buffer(4, 2)
    solver.run(S, 4, ck, 2)
    with pytest.raises(P.RTError) as ei:
        solver.adjoint(4, ck, 2, solver.empty_state())
    assert ei.value.status == P.RT_EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp32", "plain", "bf16"])
@pytest.mark.parametrize("dims", [(1, 1, (0, 0, 0, 0)), (2, 3, (0, 0, 0, 0)), (5, 1, (1, 1, 1, 2)),
                                  (1, 7, (1, 1, 1, 2)), (3, 2, (0, 0, 1, 2))])
def test_degenerate_lattices(dims, precision):
    """Lattices smaller than every tap reach: a periodic axis of length 1 or 2
    wraps taps onto the same cells several times; absorbing and inflow edges
    surround every cell."""
    nx, ny, bc = dims
    spec = W.spec("beam512", nx=nx, ny=ny, n_zen=2, n_az=8, bc=bc)
    _, oprob, got, ref = _run_both(spec, precision, 12, "random")
    assert_close(got, ref, tolerance(precision, oprob), ("degenerate", dims, precision))


@pytest.mark.parametrize("dims", [(1, 1, (0, 0, 0, 0)), (5, 1, (1, 1, 1, 2)), (3, 2, (0, 0, 1, 2))])
def test_adjoint_degenerate_lattices(dims):
    nx, ny, bc = dims
    spec = W.spec("adjoint256", nx=nx, ny=ny, n_zen=2, n_az=8, bc=bc)
    ref, got = _adjoint_case(spec, "fp32", 9, 3)
    for key, arr in zip(("g_tau", "g_albedo", "g_emis", "lambda0"), got):
        assert _rel(arr, ref[key]) < GTOL["fp32"], (dims, key, _rel(arr, ref[key]))
