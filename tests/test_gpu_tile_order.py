"""The 2-D fused steps' tile order (rt_set_tile_strip): vertical strips of
tiles instead of the lattice's row order change only which tiles are in
flight together, so forward runs, checkpoints and the checkpointed adjoint
are bit-identical in every order, and the oracle is met at the stated
tolerance in strip order."""
import numpy as np
import pytest

import workloads as W
from gpu_common import assert_close, build, gtolerance, to_dev, to_np, tolerance
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# nx = 256: strips of 1, 2 and 4 tiles of 64 cells cover whole rows
CASES = [("beam512", dict(nx=256, ny=21), "fp32"), ("beam512", dict(nx=256, ny=21), "bf16"),
         ("prec1024", dict(nx=256, ny=9), "bf16"), ("prec1024", dict(nx=256, ny=9), "fp16"),
         ("prec1024", dict(nx=256, ny=9), "bf16x3"), ("adjoint256", dict(nx=256, ny=17), "fp32")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-%s" % (c[0], c[1]["nx"], c[1]["ny"], c[2]))
def test_strip_order_is_bit_identical_and_meets_the_oracle(case):
    name, over, precision = case
    spec = W.spec(name, **over)
    solver, oprob, _ = build(spec, precision)
    S0 = W.initial_state(spec, "random")
    T, K = 9, 3
    lam = torch.rand(solver.shape, dtype=torch.float32, device=solver.device)
    out = {}
    for strip in (0, 1, 2, 4):
        solver.set_tile_strip(strip)
        ck = solver.checkpoint_buffer(T, K)
        S = to_dev(S0, solver)
        solver.run(S, T, ck, K)
        g = solver.adjoint(T, ck, K, lam)
        torch.cuda.synchronize()
        out[strip] = (S.clone(), ck.clone(), [x.clone() for x in g])
    for strip in (1, 2, 4):
        assert torch.equal(out[strip][0], out[0][0]), strip
        assert torch.equal(out[strip][1], out[0][1]), strip
        for a, b in zip(out[strip][2], out[0][2]):
            assert torch.equal(a, b), strip
    ref = OL.run(S0, oprob, T)
    assert_close(to_np(out[4][0]), ref, tolerance(precision, oprob, T), (name, precision))
    # the adjoint in strip order against the oracle adjoint of the same lambda_T
    r = OA.adjoint(S0, oprob, T, lam.cpu().double().numpy())
    for key, got in zip(("g_tau", "g_albedo", "g_emis"), out[4][2]):
        gv, rv = got.cpu().double().numpy().reshape(-1), np.asarray(r[key]).reshape(-1)
        if np.linalg.norm(rv) > 0:
            assert np.linalg.norm(gv - rv) / np.linalg.norm(rv) < gtolerance(precision, oprob, T), key


def test_tile_strip_refusal():
    import paper_2609_23057_amd as P
    solver, _, _ = build(W.spec("beam512", nx=64, ny=8), "fp32")
    with pytest.raises(P.RTError) as ei:
        solver.set_tile_strip(-1)
    assert ei.value.status == P.RT_EINVAL
