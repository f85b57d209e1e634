"""rt_totals_noalloc (the allocation-free variant of rt_readout's totals,
whose partial sums live in the library's static device array) against
rt_readout's float64 sums, through the C ABI: two calls in a row on one
device, the second on a smaller lattice, both bit-identical to the
workspace path (same kernels, same partition of the cells)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import build, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _totals_both(solver, S):
    import paper_2609_23057_amd._abi as A
    ref = np.zeros(4)
    A.rt_readout(solver.ctx, S.data_ptr(), 0, None, ref)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device=solver.device)
    A.rt_totals_noalloc(solver.ctx, S.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref


def test_noalloc_totals_equal_the_workspace_totals_on_two_lattices():
    big = W.spec("beam512", nx=300, ny=211)      # 63300 cells: 248 partial sums
    small = W.spec("beam512", nx=19, ny=7)       # 133 cells: one partial sum
    sb, _, _ = build(big, "fp32")
    ss, _, _ = build(small, "fp32")
    Sb = to_dev(W.initial_state(big, "random"), sb)
    sb.run(Sb, 3)
    Ss = to_dev(W.initial_state(small, "random"), ss)
    ss.run(Ss, 3)
    got_b, ref_b = _totals_both(sb, Sb)
    got_s, ref_s = _totals_both(ss, Ss)
    assert np.all(np.isfinite(ref_b)) and abs(ref_b[0]) > 0
    assert np.array_equal(got_b, ref_b), (got_b, ref_b)
    # the second, smaller call reads none of the first call's partial sums
    assert np.array_equal(got_s, ref_s), (got_s, ref_s)
    # and the sums are those of the field
    host = Ss.double().sum(dim=(0, 2, 3)).cpu().numpy()
    assert np.allclose(got_s, host, rtol=1e-12, atol=1e-12)


def test_noalloc_totals_refuse_null_pointers():
    import paper_2609_23057_amd as P
    import paper_2609_23057_amd._abi as A
    spec = W.spec("beam512", nx=16, ny=16)
    s, _, _ = build(spec, "fp32")
    S = s.empty_state()
    with pytest.raises(P.RTError) as ei:
        A.rt_totals_noalloc(s.ctx, S.data_ptr(), None)
    assert ei.value.status == P.RT_EINVAL
