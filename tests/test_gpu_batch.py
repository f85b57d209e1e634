"""Spectral batch: independent channels advanced by one launch per time step.

A batch runs the same per-tile kernel body as a single context, so every
channel must reproduce bit for bit what its own context computes (states,
checkpoints, adjoint gradients), and therefore the float64 oracle within the
precision's tolerance.  Graph mode must replay the eager result exactly.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import GTOL, assert_close, build, tolerance, to_dev, to_np
from oracle import adjoint as OA
from oracle import lbm as OL

pytestmark = pytest.mark.gpu

# ragged channels: lattice (nx, ny) and direction grid (n_zen, n_az) -> n = 8, 16, 32, 64, 16
SMALL = [((40, 36), (2, 4)), ((33, 30), (2, 8)), ((64, 48), (4, 8)), ((48, 40), (4, 16)), ((20, 70), (2, 8))]


def channel_specs(layout, seed=11):
    base = W.spectral_channels(len(layout), seed=seed)
    out = []
    for s, ((nx, ny), (nz, na)) in zip(base, layout):
        s = dict(s)
        s.update(nx=nx, ny=ny, n_zen=nz, n_az=na, beam_dir=W.BEAM_ZEN_INDEX[nz] * na)
        out.append(s)
    return out


def make_batch(specs, precision):
    import paper_2609_23057_amd as P
    probs = []
    for s in specs:
        d = dict(s)
        d["precision"] = precision
        probs.append(P.make_problem(**d))
    batch = P.Batch(probs)
    meds = []
    for ch, s in zip(batch.channels, specs):
        med = W.medium(s)
        t = [to_dev(med[k], ch) for k in ("tau", "albedo", "emis")]
        ch.set_medium(*t, med["jprof"], med["inflow"])
        ch._tensors = t
        meds.append(med)
    return batch, meds


def initial_states(batch, specs, seed=3):
    states = []
    for ch, s in zip(batch.channels, specs):
        rng = np.random.default_rng(seed + s["nx"] * 7 + s["ny"])
        S0 = np.abs(rng.standard_normal(ch.shape)) * 0.1
        S0[:, 1:] *= 0.3
        states.append(to_dev(S0, ch))
    return states


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3", "fp16"])
def test_batch_forward_matches_single_contexts_bitwise(precision):
    specs = channel_specs(SMALL)
    batch, meds = make_batch(specs, precision)
    S0 = initial_states(batch, specs)
    T, K = 13, 4
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    batch.run(states, T, ck, K)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        single, _, _ = build(s, precision, meds[i])
        S = S0[i].clone()
        ck1 = single.checkpoint_buffer(T, K)
        single.run(S, T, ck1, K)
        torch.cuda.synchronize()
        assert torch.equal(S, states[i]), (precision, i, s["nx"], s["ny"], s["n_zen"] * s["n_az"])
        assert torch.equal(ck1, ck[i]), (precision, i)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_batch_channels_match_oracle(precision):
    specs = channel_specs(SMALL)
    batch, meds = make_batch(specs, precision)
    S0 = initial_states(batch, specs)
    T = 6
    states = [s.clone() for s in S0]
    batch.run(states, T)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        oprob = OL.make_problem(s, meds[i])
        ref = OL.run(to_np(S0[i]), oprob, T)
        got = to_np(states[i])
        assert_close(got, ref, tolerance(precision, oprob), (precision, i))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_batch_adjoint_matches_single_contexts_bitwise(precision):
    specs = channel_specs(SMALL)
    batch, meds = make_batch(specs, precision)
    S0 = initial_states(batch, specs)
    T, K = 9, 3
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    batch.run(states, T, ck, K)
    lams = []
    for i, ch in enumerate(batch.channels):
        g = torch.randn((ch.nx, ch.nout[3], 4), generator=torch.Generator().manual_seed(i)).to(ch.device)
        lams.append(ch.readout_adjoint(3, g))
    grads = batch.adjoint(T, ck, K, lams)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        single, _, _ = build(s, precision, meds[i])
        S = S0[i].clone()
        ck1 = single.checkpoint_buffer(T, K)
        single.run(S, T, ck1, K)
        g1 = single.adjoint(T, ck1, K, lams[i])
        torch.cuda.synchronize()
        for a, b, name in zip(grads[i], g1, ("tau", "albedo", "emis")):
            assert torch.equal(a, b), (precision, i, name)


def test_batch_adjoint_matches_oracle_gradients():
    specs = channel_specs(SMALL[:3])
    batch, meds = make_batch(specs, "fp32")
    S0 = initial_states(batch, specs)
    T, K = 7, 3
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    batch.run(states, T, ck, K)
    lams, gouts = [], []
    for i, ch in enumerate(batch.channels):
        g = torch.randn((ch.nx, ch.nout[3], 4), generator=torch.Generator().manual_seed(10 + i)).to(ch.device)
        gouts.append(to_np(g))
        lams.append(ch.readout_adjoint(3, g))
    grads = batch.adjoint(T, ck, K, lams)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        oprob = OL.make_problem(s, meds[i])
        res = OA.adjoint(to_np(S0[i]), oprob, T, OL.readout_transpose(gouts[i], oprob, 3))
        for got, key in zip(grads[i], ("g_tau", "g_albedo", "g_emis")):
            ref = res[key]
            err = np.abs(to_np(got) - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err < GTOL["fp32"], (i, key, err)


def test_batch_graph_replays_match_eager():
    specs = channel_specs(SMALL)
    batch, meds = make_batch(specs, "bf16")
    S0 = initial_states(batch, specs)
    T, K = 10, 4
    eager = [s.clone() for s in S0]
    ck_e = batch.checkpoint_buffers(T, K)
    batch.run(eager, T, ck_e, K)
    lams = [ch.readout_adjoint(3, torch.ones((ch.nx, ch.nout[3], 4), device=ch.device)) for ch in batch.channels]
    g_eager = batch.adjoint(T, ck_e, K, lams)
    torch.cuda.synchronize()

    batch.set_graph(True)
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    segs = batch.segment_buffers(K)
    grads = [torch.empty((3, ch.ny, ch.nx), device=ch.device) for ch in batch.channels]
    import paper_2609_23057_amd._abi as A
    for rep in range(3):
        for s, s0 in zip(states, S0):
            s.copy_(s0)
        junk = torch.randn(1024, device="cuda").sum()   # eager work between replays
        batch.run(states, T, ck, K)
        A.rt_batch_adjoint(batch.handle, T, [c.data_ptr() for c in ck], K, [s.data_ptr() for s in segs],
                           [l.data_ptr() for l in lams], [g[0].data_ptr() for g in grads],
                           [g[1].data_ptr() for g in grads], [g[2].data_ptr() for g in grads])
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i in range(len(specs)):
            assert torch.equal(states[i], eager[i]), ("replay", rep, i)
            assert torch.equal(ck[i], ck_e[i]), ("replay ckpt", rep, i)
            for a, b in zip(grads[i], g_eager[i]):
                assert torch.equal(a, b), ("replay adjoint", rep, i)
    batch.set_graph(False)


def test_batch_rejects_mixed_precision_and_unsupported_sizes():
    import paper_2609_23057_amd as P
    specs = channel_specs(SMALL[:2])
    p0 = P.make_problem(**dict(specs[0], precision="bf16"))
    p1 = P.make_problem(**dict(specs[1], precision="fp32"))
    with pytest.raises(P.RTError):
        P.Batch([p0, p1])
    p2 = P.make_problem(**dict(specs[0], precision="bf16", n_zen=8, n_az=16))   # n = 128
    with pytest.raises(P.RTError):
        P.Batch([p0, p2])


def test_spectral64_full_size_channels_match_single_and_oracle():
    """The 64-channel workload at full size, in the bench's configuration
    (bf16): two steps of the whole batch; sampled channels against their own
    contexts (bitwise) and the two smallest against the oracle."""
    specs = W.spectral_channels(64)
    batch, meds = make_batch(specs, "bf16")
    states = [torch.zeros(ch.shape, device=ch.device) for ch in batch.channels]
    T = 2
    batch.run(states, T)
    torch.cuda.synchronize()
    order = sorted(range(64), key=lambda i: specs[i]["nx"] * specs[i]["nx"] * specs[i]["n_zen"] * specs[i]["n_az"])
    sampled = sorted({order[0], order[1], order[31], order[63], 0, 63})
    for i in sampled:
        single, _, _ = build(specs[i], "bf16", meds[i])
        S = torch.zeros(single.shape, device=single.device)
        single.run(S, T)
        torch.cuda.synchronize()
        assert torch.equal(S, states[i]), i
        del single
    for i in order[:2]:
        oprob = OL.make_problem(specs[i], meds[i])
        ref = OL.run(np.zeros(oprob.shape), oprob, T)
        assert_close(to_np(states[i]), ref, tolerance("bf16", oprob), ("spectral64", i))


def test_single_channel_batch_matches_its_context_bitwise():
    specs = channel_specs(SMALL[2:3])
    batch, meds = make_batch(specs, "bf16")
    S0 = initial_states(batch, specs)
    T, K = 7, 3
    states = [s.clone() for s in S0]
    ck = batch.checkpoint_buffers(T, K)
    batch.run(states, T, ck, K)
    single, _, _ = build(specs[0], "bf16", meds[0])
    S = S0[0].clone()
    ck1 = single.checkpoint_buffer(T, K)
    single.run(S, T, ck1, K)
    torch.cuda.synchronize()
    assert torch.equal(S, states[0])
    assert torch.equal(ck1, ck[0])


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_block_size_of_a_class_does_not_change_results(precision):
    """Every admissible block size of every channel class (the tuning table
    of rt_batch_set_tuning) and every grouping of the channels (the cache
    budget) gives the same bits: forward with checkpoints and the adjoint."""
    import paper_2609_23057_amd as P
    specs = channel_specs(SMALL)
    batch, _ = make_batch(specs, precision)
    classes = batch.classes()
    assert [c[0] for c in classes] == sorted(c[0] for c in classes)
    assert sum(c[2] for c in classes) == len(specs)
    T, K = 7, 3

    def run_all():
        states = initial_states(batch, specs)
        ck = batch.checkpoint_buffers(T, K)
        batch.run(states, T, ck, K)
        lams = [torch.ones_like(x) for x in states]
        grads = batch.adjoint(T, ck, K, lams)
        torch.cuda.synchronize()
        return [x.clone() for x in states] + [g.clone() for gs in grads for g in gs]

    ref = run_all()
    for W_, bw0, _ in classes:
        for bw in (1, 2, 4, 8):
            if bw < W_ or bw % W_ or bw == bw0:
                continue
            batch.set_tuning(W_, bw)
            got = run_all()
            assert all(torch.equal(a, b) for a, b in zip(got, ref)), (W_, bw)
        batch.set_tuning(W_, bw0)
    # the temporal blocking: all channels together, or one channel per group
    for budget in (0, 1):
        batch.set_cache_budget(budget)
        got = run_all()
        assert all(torch.equal(a, b) for a, b in zip(got, ref)), budget
    with pytest.raises(P.RTError) as ei:
        batch.set_tuning(classes[-1][0], 3)
    assert ei.value.status == P.RT_EINVAL
    with pytest.raises(P.RTError):
        batch.set_tuning(99, 8)
