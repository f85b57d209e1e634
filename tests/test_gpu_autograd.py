"""RTSolve (torch.autograd.Function over the C ABI): several applications on
one solver before a single backward.

Each backward must differentiate the medium its own forward ran with, even
when a later forward on the same solver set another one; the result must
equal the gradients of separate single applications, and the solver must
hold the newest medium again afterwards.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import build, to_dev, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _loss(out):
    I, Q, U = out[..., 0], out[..., 1], out[..., 2]
    return (I + torch.sqrt(Q * Q + U * U + (1e-6 * I) ** 2) / I).sum()


def _leaf(a, solver):
    return to_dev(a, solver).requires_grad_(True)


@pytest.mark.parametrize("ext", [None, "mixture", "mixture3"])
def test_two_applications_before_one_backward(ext):
    import paper_2609_23057_amd as P
    spec = W.spec("adjoint256", nx=30, ny=26)
    if ext == "mixture":
        spec = dict(spec, mixture={"kind": "rayleigh"})
    elif ext == "mixture3":
        spec = dict(spec, mixture=[{"kind": "rayleigh"}, {"kind": "hg", "g": -0.4}])
    solver, _, med = build(spec, "fp32")
    med2 = W.medium(spec, seed=77)
    T = 14
    frac = None
    if ext is not None:
        frac = to_dev(med["frac"], solver)
        solver.set_phase_mixture(spec["mixture"], frac)

    def apply(m):
        leaves = [_leaf(m[k], solver) for k in ("tau", "albedo", "emis")]
        out = P.RTSolve.apply(*leaves, solver, solver.empty_state(), T, 3, med["jprof"], med["inflow"])
        return leaves, out

    # separate applications, one backward each
    ref = []
    for m in (med, med2):
        leaves, out = apply(m)
        _loss(out).backward()
        ref.append([to_np(x.grad) for x in leaves])
    # both applications, then one backward over the sum
    l1, o1 = apply(med)
    l2, o2 = apply(med2)
    (_loss(o1) + 2.0 * _loss(o2)).backward()
    torch.cuda.synchronize()
    for got, want, w in ((l1, ref[0], 1.0), (l2, ref[1], 2.0)):
        for g, r in zip(got, want):
            assert np.array_equal(to_np(g.grad), w * r) or \
                np.abs(to_np(g.grad) - w * r).max() <= 1e-6 * max(np.abs(w * r).max(), 1e-30)
    # the solver holds the newest medium again (and still the mixture)
    tau_now = solver.medium_state()[1][0]
    assert torch.equal(tau_now, l2[0].detach())
    if ext is not None:
        assert solver.medium_state()[2][1] is frac
