"""Spectral batch with phase mixtures: channels whose scattering is a per-cell
mixture of phase functions (two or three) run beside single-phase channels
in the batched launches and reproduce their own contexts bit for bit
(states, checkpoints, adjoint gradients); a mixture set or removed between
runs is taken up, also by graph replays."""
import numpy as np
import pytest
import torch

from gpu_common import assert_close, build, to_dev, to_np, tolerance
from oracle import lbm as OL
from test_gpu_batch import SMALL, channel_specs, initial_states, make_batch

pytestmark = pytest.mark.gpu

MIXES = {1: {"kind": "rayleigh"}, 3: [{"kind": "hg", "g": -0.3}, {"kind": "rayleigh"}]}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mixed_specs():
    specs = channel_specs(SMALL)
    for i, mix in MIXES.items():
        specs[i] = dict(specs[i], mixture=mix)
    return specs


def set_mixtures(solvers, specs, meds):
    keep = []
    for ch, s, med in zip(solvers, specs, meds):
        if s.get("mixture") is not None:
            f = to_dev(med["frac"], ch)
            ch.set_phase_mixture(s["mixture"], f)
            keep.append(f)
    return keep


def single_run(s, precision, med, S0, T, K, lam=None):
    single, oprob, _ = build(s, precision, med)
    keep = set_mixtures([single], [s], [med])
    S = S0.clone()
    ck = single.checkpoint_buffer(T, K)
    single.run(S, T, ck, K)
    g = single.adjoint(T, ck, K, lam) if lam is not None else None
    torch.cuda.synchronize()
    del keep
    return S, ck, g, oprob


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp16"])
def test_batch_with_mixed_channels_matches_single_contexts_bitwise(precision):
    specs = mixed_specs()
    batch, meds = make_batch(specs, precision)
    keep = set_mixtures(batch.channels, specs, meds)
    S0 = initial_states(batch, specs)
    T, K = 9, 3
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    batch.run(states, T, ck, K)
    lams = [torch.ones_like(x) * 0.5 for x in states]
    grads = batch.adjoint(T, ck, K, lams)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        S, ck1, g1, oprob = single_run(s, precision, meds[i], S0[i], T, K, lams[i])
        assert torch.equal(S, states[i]), (precision, i)
        assert torch.equal(ck1, ck[i]), (precision, i)
        for a, b, name in zip(grads[i], g1, ("tau", "albedo", "emis")):
            assert torch.equal(a, b), (precision, i, name)
        if i in MIXES:
            assert oprob.mix_M is not None
            ref = OL.run(to_np(S0[i]), oprob, T)
            assert_close(to_np(states[i]), ref, tolerance(precision, oprob, T), (precision, i))
    del keep


def test_mixture_changes_between_runs_and_graph_replays():
    """Eager: no mixture, then mixtures on two channels, then none again.
    Graph mode runs the same sequence on the same buffers (so a recorded
    graph would be replayed unless the change of mixture is noticed) and
    matches each eager result; with a cache budget of one byte (every channel
    a group of its own, on the single-problem kernels) the bits are the same."""
    import paper_2609_23057_amd._abi as A
    specs = mixed_specs()
    batch, meds = make_batch(specs, "bf16")
    S0 = initial_states(batch, specs)
    T, K = 6, 3
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    segs = batch.segment_buffers(K)
    lams = [torch.ones_like(x) for x in states]
    grads = [torch.empty((3, ch.ny, ch.nx), device=ch.device) for ch in batch.channels]

    def run_once():
        for x, x0 in zip(states, S0):
            x.copy_(x0)
        batch.run(states, T, ck, K)
        A.rt_batch_adjoint(batch.handle, T, [c.data_ptr() for c in ck], K, [x.data_ptr() for x in segs],
                           [x.data_ptr() for x in lams], [g[0].data_ptr() for g in grads],
                           [g[1].data_ptr() for g in grads], [g[2].data_ptr() for g in grads])
        torch.cuda.synchronize()
        return [x.clone() for x in states] + [g.clone() for g in grads]

    def sequence():
        out = [run_once()]
        keep = set_mixtures(batch.channels, specs, meds)
        out.append(run_once())
        for i in MIXES:
            batch.channels[i].set_phase_mixture(None, None)
        out.append(run_once())
        del keep
        return out

    eager = sequence()
    assert not all(torch.equal(a, b) for a, b in zip(eager[0], eager[1]))
    assert all(torch.equal(a, b) for a, b in zip(eager[0], eager[2]))
    batch.set_graph(True)
    for rep in range(2):
        graphed = sequence()
        for k in range(3):
            for a, b in zip(graphed[k], eager[k]):
                assert torch.equal(a, b), ("graph", rep, k)
    batch.set_graph(False)
    batch.set_cache_budget(1)
    alone = sequence()
    for k in range(3):
        for a, b in zip(alone[k], eager[k]):
            assert torch.equal(a, b), ("one channel per group", k)


def test_batch_refuses_a_dichroic_channel_but_not_a_mixed_one():
    import paper_2609_23057_amd as P
    specs = mixed_specs()[:2]
    batch, meds = make_batch(specs, "fp32")
    keep = set_mixtures(batch.channels, specs, meds)
    states = initial_states(batch, specs)
    batch.run(states, 2)
    eta = to_dev(np.full((specs[0]["ny"], specs[0]["nx"]), 0.2), batch.channels[0])
    batch.channels[0].set_dichroism(eta)
    with pytest.raises(P.RTError) as ei:
        batch.run(states, 2)
    assert ei.value.status == P.RT_EUNSUPPORTED
    batch.channels[0].set_dichroism(None)
    batch.run(states, 2)
    torch.cuda.synchronize()
    del keep
