#!/usr/bin/env python3
"""Throughput of the polarized LBM radiative-transfer solver on one MI355X.

One timed step is one pass of the whole hot path over the beam512 workload
(512x512 lattice, n = 32 directions = 4 zenith x 8 azimuth, lognormal
extinction, albedo U[0.8,1], HG(0.7) weights with Rayleigh polarisation,
solar beam entering the top, 2000 time steps):
  forward run of T steps with sqrt(T) checkpoints (fused stream + collide
  kernel), top-edge readout, readout adjoint, and the checkpointed adjoint
  over T steps (segment recompute + fused adjoint kernel + gradient chain).
value = (C n T forward + C n T adjoint) Stokes cell-direction updates per
second of that step.  All inputs are resident in HBM before timing starts.

Extras (skipped with --no-extras): forward rates at 1024x1024, n = 128 per
contraction precision, the stand-alone streaming kernel's HBM rate at beam512
and prec1024, the forward step at beam512 with each extension of the operator
(tabulated scattering matrix, per-cell phase mixture, dichroic absorption),
the 256x256x64 three-dimensional lattice, the 64-channel spectral batch (one launch per channel class and step,
eager and as a replayed HIP graph), and the statevector emulation of the paper's circuit on its 16x16, n = 8
lattice (29 qubits).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2609_23057_amd", "csrc", "rt_kernels.hip")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel_key)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0}


def step_work(C, n):
    """Algorithmic work of one fused step launch over C cells and n directions.

    bytes: 32 per cell-direction (read 16 B and write 16 B of float32 Stokes
    state) plus 12 per cell (alpha, beta, emission);
    flops: 20 n per cell-direction, the nonzeros of the collision matrix
    (3n x 3n for I, Q, U plus n x n for V: 10 n^2 multiply-adds per cell);
    executed: the dense 4n x 4n contraction the matrix cores perform, 32 n per
    cell-direction (the zero IQU-V blocks included)."""
    return {"bytes": C * (32.0 * n + 12.0), "flops": 20.0 * n * n * C,
            "executed_flops": 32.0 * n * n * C}


def roofline(nbytes, flops, launch_us, precision):
    """Roofline of one fused step launch: the bound is whichever of HBM
    traffic (8 TB/s) and the algorithmic contraction on the matrix cores (peak
    of the contraction dtype) takes longer at peak."""
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops / (MFMA_PEAK_TFLOPS[precision] * 1e12)
    sec = launch_us * 1e-6
    hbm = {"achieved": nbytes / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    mfma = {"achieved": flops / sec / 1e12, "peak": MFMA_PEAK_TFLOPS[precision], "unit": "TFLOP/s"}
    for r in (hbm, mfma):
        r["frac"] = r["achieved"] / r["peak"]
    main, other = (hbm, mfma) if t_hbm >= t_mfma else (mfma, hbm)
    out = dict(main)
    out["bound"] = "hbm" if main is hbm else "mfma"
    out["secondary"] = dict(other)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def loss_grad(out):
    """d/d(readout) of sum(I + DoLP), DoLP = sqrt(Q^2+U^2+(1e-6 I)^2)/I (torch ops on the readout)."""
    import torch
    I, Q, U = out[..., 0], out[..., 1], out[..., 2]
    Ic = torch.clamp(I, min=1e-30)
    r = torch.sqrt(Q * Q + U * U + (1e-6 * Ic) ** 2)
    g = torch.zeros_like(out)
    g[..., 0] = 1.0 + 1e-12 / r - r / (Ic * Ic)
    g[..., 1] = Q / (r * Ic)
    g[..., 2] = U / (r * Ic)
    return g


def make_solver(spec, precision):
    """precision: fp32 / bf16 / fp16 / bf16x3 (fused matrix-core step) or
    plain (float32 streaming kernel + vector-ALU collision)."""
    import numpy as np
    import torch
    import paper_2609_23057_amd as P
    import workloads as W
    s = dict(spec)
    s["precision"] = "fp32" if precision == "plain" else precision
    s["plain"] = precision == "plain"
    solver = P.Solver(P.make_problem(**s))
    med = W.medium(spec)
    dev = solver.device
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    solver._med = (t(med["tau"]), t(med["albedo"]), t(med["emis"]))
    solver.set_medium(*solver._med, med["jprof"], med["inflow"])
    return solver


def cpu_baseline(spec, nsteps=3):
    """The FP64 oracle on the host cores: nsteps forward steps of the full
    512x512 lattice plus the adjoint over them (the oracle's adjoint re-runs
    the forward and stores every state)."""
    import numpy as np
    import workloads as W
    from oracle import adjoint as OA
    from oracle import lbm as OL
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    med = W.medium(spec)
    prob = OL.make_problem(spec, med)
    S0 = np.zeros(prob.shape)
    t0 = time.perf_counter()
    ST = OL.run(S0, prob, nsteps)
    _, g = OL.edge_loss(ST, prob, 3)
    OA.adjoint(S0, prob, nsteps, OL.readout_transpose(g, prob, 3))
    dt = time.perf_counter() - t0
    C, n = spec["nx"] * spec["ny"], W.ndir(spec)
    return {"value": 2.0 * C * n * nsteps / dt, "unit": "Stokes cell-direction updates/s",
            "cores": int(threads), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "float64 NumPy oracle, %d forward steps + adjoint over them on the full "
                      "512x512 n=32 lattice (%.1f s); host has %d logical CPUs (%s)"
                      % (nsteps, dt, os.cpu_count() or 0, cpu_model())}


def precision_extras(T=20, warm=3):
    """Forward throughput of the fused step at 1024x1024, n = 128 per contraction precision."""
    import torch
    import workloads as W
    spec = W.spec("prec1024")
    C, n = spec["nx"] * spec["ny"], W.ndir(spec)
    res = {}
    for prec in ("plain", "fp32", "bf16", "bf16x3", "fp16"):
        _log("bench: prec1024 %s" % prec)
        solver = make_solver(spec, prec)
        S = solver.empty_state()
        solver.run(S, warm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.run(S, T)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[prec] = {"cell_dir_updates_per_s": C * n * T / (ms / 1e3), "ms_per_time_step": ms / T}
        if prec != "plain":
            # T + 1 launches (T - 1 fused, one collide-only, one stream), all
            # one read and one write of the state: their mean stands for the
            # fused kernel's launch
            wk = step_work(C, n)
            us = ms * 1e3 / (T + 1)
            res[prec]["roofline"] = dict(roofline(wk["bytes"], wk["flops"], us, prec), avg_launch_us=us,
                                         algorithmic_bytes_per_launch=wk["bytes"],
                                         algorithmic_flops_per_launch=wk["flops"],
                                         executed_mfma_flops_per_launch=wk["executed_flops"])
        del solver, S
        torch.cuda.empty_cache()
    for k in res:
        res[k]["speedup_vs_fused_fp32"] = (res[k]["cell_dir_updates_per_s"]
                                           / res["fp32"]["cell_dir_updates_per_s"])
        res[k]["speedup_vs_plain_fp32"] = (res[k]["cell_dir_updates_per_s"]
                                           / res["plain"]["cell_dir_updates_per_s"])
    return {"workload": "prec1024: 1024x1024, n=128 (8x16), forward steps", "steps": T, "rates": res}


def extension_extras(T=20, warm=3):
    """Forward rate of the fused step at beam512 with each extension of the
    operator beside the plain workload, per contraction precision: a
    tabulated scattering matrix (P12, P34 != 0), a per-cell phase-function
    mixture (HG(0.7) and Rayleigh, fraction U[0, 1]; two contractions per
    cell), a mixture of four phase functions (HG(0.7), Rayleigh, HG(-0.3),
    Rayleigh / HG(0.5); flat Dirichlet fractions; four contractions per cell)
    and dichroic absorption (eta U[-0.8, 0.8]; applied in the gather).
    For the plain workload, the mixture and the dichroism also the
    checkpointed adjoint over the same steps (per-step cost and adjoint /
    checkpointed-forward ratio)."""
    import numpy as np
    import torch
    import workloads as W
    base = W.spec("beam512")
    C, n = base["nx"] * base["ny"], W.ndir(base)
    variants = {
        "single": (base, None),
        "table": (W.spec("beam512", phase={"kind": "table", "table": W.scattering_table()}), None),
        "mixture": (W.spec("beam512", mixture={"kind": "rayleigh"}), "mixture"),
        "mixture4": (W.spec("beam512", mixture=[{"kind": "rayleigh"}, {"kind": "hg", "g": -0.3},
                                                {"kind": "mix", "g": 0.5, "mix_ray": 0.4}]), "mixture"),
        "dichroism": (W.spec("beam512", dichroism=0.8), "dichroism"),
    }
    res = {}
    for prec in ("fp32", "bf16"):
        out = {}
        for name, (spec, ext) in variants.items():
            _log("bench: beam512 %s %s" % (prec, name))
            solver = make_solver(spec, prec)
            med = W.medium(spec)
            if ext == "mixture":
                extra = torch.tensor(np.ascontiguousarray(med["frac"]), dtype=torch.float32, device=solver.device)
                solver.set_phase_mixture(spec["mixture"], extra)
            elif ext == "dichroism":
                extra = torch.tensor(np.ascontiguousarray(med["eta"]), dtype=torch.float32, device=solver.device)
                solver.set_dichroism(extra)
            S = solver.empty_state()
            solver.run(S, warm)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            solver.run(S, T)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            out[name] = {"cell_dir_updates_per_s": C * n * T / (ms / 1e3), "ms_per_time_step": ms / T}
            if name in ("single", "mixture", "mixture4", "dichroism"):
                # the checkpointed forward and its adjoint (recompute + adjoint steps)
                K = max(1, int(math.ceil(math.sqrt(T))))
                ck = solver.checkpoint_buffer(T, K)
                seg = solver.segment_buffer(K)
                lam = torch.rand_like(S)
                S0 = S.clone()
                e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                solver.run(S0, T, ck, K)
                e2.record()
                solver.adjoint(T, ck, K, lam, seg)
                e3.record()
                torch.cuda.synchronize()
                out[name]["adjoint_ms_per_step"] = e2.elapsed_time(e3) / T
                out[name]["adjoint_fwd_ratio"] = e2.elapsed_time(e3) / e0.elapsed_time(e2)
                del ck, seg, lam, S0
            del solver, S
            torch.cuda.empty_cache()
        for name in variants:
            out[name]["cost_vs_single"] = out[name]["ms_per_time_step"] / out["single"]["ms_per_time_step"]
        res[prec] = out
    return {"workload": "beam512 (512x512, n=32), forward steps: plain workload, tabulated scattering matrix, "
                        "per-cell HG(0.7)/Rayleigh mixture, four-phase mixture, dichroic absorption",
            "steps": T, "rates": res}


def three_d_extras(T=10, warm=2, reps=20):
    """The 3-D lattice (beam3d: 256 x 256 x 64, n = 32): forward steps per
    contraction precision (fp32: the trilinear pull fused into the next
    collision's gather, T - 1 fused launches between a first collision and a
    last pull; bf16: per-cell collision, then the trilinear pull, every
    step), the checkpointed forward and its adjoint (recompute, reverse pull,
    adjoint collision), and the 3-D streaming kernel alone (HIP events around
    `reps` launches on the solver's stream) against the HBM peak at 32
    algorithmic bytes per cell-direction."""
    import torch
    import workloads as W
    spec = W.spec("beam3d")
    C, n = spec["nx"] * spec["ny"] * spec["nz"], W.ndir(spec)
    res = {}
    for prec in ("fp32", "bf16"):
        _log("bench: beam3d %s" % prec)
        solver = make_solver(spec, prec)
        S = solver.empty_state()
        solver.run(S, warm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.run(S, T)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[prec] = {"cell_dir_updates_per_s": C * n * T / (ms / 1e3), "ms_per_time_step": ms / T}
        # forward with sqrt(T) checkpoints, then the checkpointed adjoint of a
        # whole-state lambda_T (reverse trilinear pull + adjoint collision)
        K = max(1, int(math.ceil(math.sqrt(T))))
        ck = solver.checkpoint_buffer(T, K)
        seg = solver.segment_buffer(K)
        lam = torch.rand_like(S)
        S0 = S.clone()
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.run(S0, T, ck, K)
        e2.record()
        solver.adjoint(T, ck, K, lam, seg)
        e3.record()
        torch.cuda.synchronize()
        res[prec]["checkpointed_forward_ms_per_step"] = e0.elapsed_time(e2) / T
        res[prec]["adjoint_ms_per_step"] = e2.elapsed_time(e3) / T
        res[prec]["adjoint_fwd_ratio"] = e2.elapsed_time(e3) / e0.elapsed_time(e2)
        del ck, seg, lam, S0
        if prec == "fp32":
            b = torch.empty_like(S)
            solver.stream_field(S, b)
            torch.cuda.synchronize()
            e0.record()
            for i in range(reps):
                solver.stream_field(S, b) if i % 2 == 0 else solver.stream_field(b, S)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            nbytes = 32.0 * C * n
            gbs = nbytes / (us * 1e-6) / 1e9
            res["stream3d"] = {"avg_launch_us": us, "algorithmic_bytes_per_launch": nbytes, "achieved": gbs,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "bound": "hbm"}
            del b
        del solver, S
        torch.cuda.empty_cache()
    return {"workload": "beam3d: 256x256x64 lattice, n=32 (4x8), forward steps (fp32: trilinear pull fused into the "
                        "next collision; bf16: collision + trilinear streaming)",
            "steps": T, "rates": res}


def streaming_extras(reps=50):
    """The stand-alone streaming kernel (rt_stream, Eq. 34 pull with the
    workload's edges) at beam512 and prec1024: average launch time over
    `reps` launches (HIP events on the solver's stream) and algorithmic HBM
    traffic 32 B per cell-direction (16 B read, 16 B written) against the
    8 TB/s peak."""
    import torch
    import workloads as W
    res = {}
    for name in ("beam512", "prec1024"):
        spec = W.spec(name)
        C, n = spec["nx"] * spec["ny"], W.ndir(spec)
        solver = make_solver(spec, "fp32")
        a = torch.rand(solver.shape, device=solver.device)
        b = torch.empty_like(a)
        for _ in range(3):
            solver.stream_field(a, b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            solver.stream_field(a, b) if i % 2 == 0 else solver.stream_field(b, a)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        nbytes = 32.0 * C * n
        gbs = nbytes / (us * 1e-6) / 1e9
        res[name] = {"avg_launch_us": us, "algorithmic_bytes_per_launch": nbytes, "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "bound": "hbm"}
        del solver, a, b
        torch.cuda.empty_cache()
    return res


def _time_ms(fn, reps=1):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_autotune(batch, states, steps=20):
    """The tuning table of a batch: for every channel class (waves per tile
    W), the forward step time with each admissible block size (W, 2W, ... up
    to 8 waves; the other classes at their chosen size), and the fastest
    kept; then the cache budget of the temporal blocking (channel groups
    that complete every step before the next group starts; 0 = all channels
    step together).  Also the same channels stepped as separate contexts
    (every step of one channel, then the next, on the same stream) for
    comparison."""
    table = {}
    for W, bw0, nch in batch.classes():
        cands = [b for b in (1, 2, 4, 8) if b >= W and b % W == 0]
        ms = {}
        for bw in cands:
            batch.set_tuning(W, bw)
            batch.run(states, 2)
            ms[bw] = _time_ms(lambda: batch.run(states, steps)) / steps
        best = min(ms, key=ms.get)
        batch.set_tuning(W, best)
        table[str(W)] = {"channels": nch, "default_block_waves": bw0, "ms_per_step_by_block_waves": ms,
                         "chosen_block_waves": best}
    budgets = {}
    for mib in (0, 64, 128, 192, 256, "one channel per group"):
        batch.set_cache_budget(1 if isinstance(mib, str) else mib << 20)
        batch.run(states, 2)
        budgets[mib] = _time_ms(lambda: batch.run(states, steps)) / steps
    best_budget = min(budgets, key=budgets.get)
    batch.set_cache_budget(1 if isinstance(best_budget, str) else best_budget << 20)
    batched = _time_ms(lambda: batch.run(states, steps)) / steps

    def separate():
        for ch, x in zip(batch.channels, states):
            ch.run(x, steps)
    separate()
    sep = _time_ms(separate) / steps
    return {"classes": table, "ms_per_step_by_cache_budget_mib": budgets, "chosen_cache_budget_mib": best_budget,
            "batched_forward_ms_per_step": batched,
            "separate_contexts_forward_ms_per_step": sep, "batched_speedup_vs_separate": sep / batched}


def statevector_extras(T=4, warm=1):
    """The statevector emulation of the paper's one-step circuit (Sec. 2.1.2 -
    2.1.8) on its 16x16 D2Q9 lattice with 2 x 4 directions (29 qubits, a
    2^29-amplitude float64 statevector): time per emulated step (encode,
    every gate, post-selection, decode; HIP events around rt_sv_step on the
    solver's stream), the statevector bytes its gate, fused-gate and
    translation launches move, and the agreement with the classical step
    after T steps (the oracle's float64 step; the paper's Tables 1-2 report
    1e-13).  The same steps with every gate launched alone (no fused passes)
    are timed beside it."""
    import numpy as np
    import torch
    import paper_2609_23057_amd._abi as A
    import workloads as W
    from oracle import lbm as OL
    spec = W.spec("qlbm16")
    _log("bench: statevector emulation (qlbm16)")
    solver = make_solver(spec, "fp32")
    nq, ndata = A.rt_sv_qubits(solver.ctx)
    work = solver.sv_workspace()
    S0 = np.asarray(W.initial_state(spec, "zero"))
    S = torch.zeros(S0.shape, dtype=torch.float64, device=solver.device)
    runs = {}
    for fuse in (0, 3):
        A.rt_sv_set_fusion(solver.ctx, fuse)
        S.zero_()
        for _ in range(warm):
            solver.sv_step(S, work=work)
        S.zero_()
        torch.cuda.synchronize()
        times, probs = [], []
        for _ in range(T):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            S, p = solver.sv_step(S, work=work)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            probs.append(p)
        runs[fuse] = (sum(times) / len(times), probs, A.rt_sv_launch_count(solver.ctx),
                      A.rt_sv_gate_count(solver.ctx))
    ms, probs, launches, (gates, shifts, nbytes) = runs[3]
    med = W.medium(spec)
    ref = OL.run(S0, OL.make_problem(spec, med), T)
    got = S.cpu().numpy()
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"workload": "qlbm16: 16x16 D2Q9 lattice, n=8 (2x4), k_ext=2.5, k_scat=0.5, dt=1/16, central source, "
                       "absorbing edges; %d emulated steps with re-encoding" % T,
           "qubits": nq, "data_qubits": ndata, "statevector_bytes": 8 << nq,
           "gates": gates, "translations": shifts, "launches": launches, "ms_per_step": ms,
           "unfused": {"launches": runs[0][2], "ms_per_step": runs[0][0], "bytes_per_step": runs[0][3][2]},
           "success_probability": probs,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "bytes_per_step": nbytes,
                        "note": "statevector bytes the launches read and write (8 per amplitude; amplitudes "
                                "known to be zero are not read) over the whole step time"},
           "max_abs_diff_vs_classical": float(np.abs(got - ref).max()),
           "rel_l2_diff_vs_classical": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    del work, solver
    torch.cuda.empty_cache()
    return out


def spectral_extras(T=200, only_tune=False):
    """The 64-channel spectral batch (per-channel lattice 128^2..512^2 and
    n = 16..64, bf16 contraction): the per-class tuning table (batch_autotune),
    then a forward run of T steps with sqrt(T) checkpoints, top-edge readout
    adjoint and the batched adjoint, each step one launch per channel class;
    timed eagerly and as a replayed HIP graph."""
    import numpy as np
    import torch
    import paper_2609_23057_amd as P
    import paper_2609_23057_amd._abi as A
    import workloads as W
    specs = W.spectral_channels(64)
    batch = P.Batch([P.make_problem(**dict(s, precision="bf16")) for s in specs])
    keep = []
    for ch, s in zip(batch.channels, specs):
        med = W.medium(s)
        t = [torch.tensor(np.ascontiguousarray(med[k]), dtype=torch.float32, device=ch.device)
             for k in ("tau", "albedo", "emis")]
        ch.set_medium(*t, med["jprof"], med["inflow"])
        keep.append(t)
    K = max(1, int(math.ceil(math.sqrt(T))))
    states = [torch.zeros(ch.shape, device=ch.device) for ch in batch.channels]
    _log("bench: spectral64 tuning table")
    tuning = batch_autotune(batch, states)
    if only_tune:
        return {"workload": "spectral64 forward steps, bf16", "tuning": tuning}
    for x in states:
        x.zero_()
    ck = batch.checkpoint_buffers(T, K)
    segs = batch.segment_buffers(K)
    lams = [torch.empty(ch.shape, device=ch.device) for ch in batch.channels]
    grads = [torch.empty((3, ch.ny, ch.nx), device=ch.device) for ch in batch.channels]
    ptrs = lambda xs: [x.data_ptr() for x in xs]  # noqa: E731

    def forward():
        for x in states:
            x.zero_()
        batch.run(states, T, ck, K)

    def adjoint():
        for ch, x, lam in zip(batch.channels, states, lams):
            A.rt_readout_adjoint(ch.ctx, 3, loss_grad(ch.readout(x, 3)).data_ptr(), lam.data_ptr())
        A.rt_batch_adjoint(batch.handle, T, ptrs(ck), K, ptrs(segs), ptrs(lams), [g[0].data_ptr() for g in grads],
                           [g[1].data_ptr() for g in grads], [g[2].data_ptr() for g in grads])

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    res = {}
    for mode in ("eager", "graph"):
        batch.set_graph(mode == "graph")
        _log("bench: spectral64 %s" % mode)
        forward()
        adjoint()
        torch.cuda.synchronize()
        res[mode] = {"forward_ms": timed(forward), "adjoint_ms": timed(adjoint)}
    batch.set_graph(False)
    upd = float(sum(ch.nx * ch.ny * ch.n for ch in batch.channels))
    g = res["graph"]
    return {"workload": "spectral64: 64 channels, 400-900 nm, lattices 128^2..512^2, n in {16, 32, 64}, "
                        "bf16 contraction, T=%d, checkpoints every %d steps" % (T, K),
            "cell_dir_per_step": upd, "time_steps": T, "ms": res,
            "forward_cell_dir_updates_per_s": upd * T / (g["forward_ms"] / 1e3),
            "forward_adjoint_cell_dir_updates_per_s": 2 * upd * T / ((g["forward_ms"] + g["adjoint_ms"]) / 1e3),
            "adjoint_fwd_ratio": g["adjoint_ms"] / g["forward_ms"],
            "graph_speedup_forward": res["eager"]["forward_ms"] / g["forward_ms"],
            "tuning": tuning}


def profile_run(name, precision, T, adjoint=False):
    """A short run of one workload for counter and trace runs of rocprofv3:
    a device copy of one state (reads and writes its bytes once: the
    calibration of FETCH_SIZE and WRITE_SIZE), then T forward steps, and with
    `adjoint` the checkpointed forward and adjoint over them."""
    import torch
    import workloads as W
    if name == "spectral64":
        # the 64-channel batch: a 2 GiB device copy (the counter calibration),
        # then T batched forward steps
        import numpy as np
        import paper_2609_23057_amd as P
        specs = W.spectral_channels(64)
        batch = P.Batch([P.make_problem(**dict(s, precision=precision)) for s in specs])
        keep = []
        for ch, s in zip(batch.channels, specs):
            med = W.medium(s)
            t = [torch.tensor(np.ascontiguousarray(med[k]), dtype=torch.float32, device=ch.device)
                 for k in ("tau", "albedo", "emis")]
            ch.set_medium(*t, med["jprof"], med["inflow"])
            keep.append(t)
        a = torch.zeros(1 << 29, dtype=torch.float32, device=batch.device)
        torch.empty_like(a).copy_(a)
        del a
        states = [torch.zeros(ch.shape, device=ch.device) for ch in batch.channels]
        torch.cuda.synchronize()
        _log("profile: spectral64 %s, %d forward steps" % (precision, T))
        batch.run(states, T)
        torch.cuda.synchronize()
        cells = [(s["nx"] * s["ny"], W.ndir(s)) for s in specs]
        print(json.dumps({"profile": name, "precision": precision, "steps": T,
                          "algorithmic_bytes_per_step": sum(C * (32 * n + 12) for C, n in cells),
                          "cell_dir_per_step": sum(C * n for C, n in cells)}), flush=True)
        return
    spec = W.spec(name)
    solver = make_solver(spec, precision)
    S = solver.empty_state()
    b = torch.empty_like(S)
    b.copy_(S)
    torch.cuda.synchronize()
    _log("profile: %s %s, %d forward steps" % (name, precision, T))
    solver.run(S, T)
    if adjoint:
        K = max(1, int(math.ceil(math.sqrt(T))))
        ck = solver.checkpoint_buffer(T, K)
        S0 = solver.empty_state()
        solver.run(S0, T, ck, K)
        lam = torch.rand_like(S)
        _log("profile: adjoint over %d steps" % T)
        solver.adjoint(T, ck, K, lam)
    torch.cuda.synchronize()
    print(json.dumps({"profile": name, "precision": precision, "steps": T, "adjoint": adjoint,
                      "state_bytes": S.numel() * 4}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tsteps", type=int, default=None, help="time steps per pass (default 2000)")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "bf16", "fp16", "bf16x3"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile", default=None,
                    choices=("beam512", "prec1024", "adjoint256", "beam3d", "qlbm16", "spectral64"),
                    help="only a short run of this workload in --precision (for rocprofv3 runs)")
    ap.add_argument("--profile-adjoint", action="store_true", help="with --profile: also the adjoint")
    ap.add_argument("--batch-autotune", action="store_true",
                    help="only the spectral batch's tuning table (block waves per channel class)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver build runs on a single GPU; multi-GPU runs (--gpus %d) are "
              "not part of it" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.profile == "qlbm16":
        # the statevector emulation (its circuit's gate kernels)
        print(json.dumps(statevector_extras(T=args.tsteps or 2, warm=0)), flush=True)
        return
    if args.profile:
        profile_run(args.profile, args.precision, args.tsteps or 8, args.profile_adjoint)
        return
    if args.batch_autotune:
        print(json.dumps(spectral_extras(only_tune=True)), flush=True)
        return
    spec = W.spec("beam512")
    T = args.tsteps or spec["steps"]
    C, n = spec["nx"] * spec["ny"], W.ndir(spec)
    K = max(1, int(math.ceil(math.sqrt(T))))
    _log("bench: building solver (beam512, %s)" % args.precision)
    solver = make_solver(spec, args.precision)
    S0 = solver.empty_state()
    S = solver.empty_state()
    ck = solver.checkpoint_buffer(T, K)
    seg = solver.segment_buffer(K)
    edge = 3

    fwd_events = []

    def one_step(timed=False):
        S.copy_(S0)
        if timed:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            fwd_events.append(ev)
            ev[0].record()
        solver.run(S, T, ck, K)
        if timed:
            ev[1].record()
        out = solver.readout(S, edge)
        lam = solver.readout_adjoint(edge, loss_grad(out))
        return solver.adjoint(T, ck, K, lam, seg)

    for i in range(args.warmup):
        _log("bench: warmup %d" % i)
        one_step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        one_step(timed=True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    _log("bench: timed %d steps, %.1f ms/step (wall %.2f s)" % (args.steps, ms_per_step, wall))

    # Forward run inside the timed region (events on the solver's stream, which
    # is torch's current stream): T + 1 launches of one-read-one-write steps
    # (T - 1 fused, one collide-only, one stream); their mean is the fused
    # kernel's launch time.
    ms_fwd = sum(a.elapsed_time(b) for a, b in fwd_events) / len(fwd_events)
    ms_adj_est = ms_per_step - ms_fwd
    avg_fused_us = ms_fwd * 1e3 / (T + 1)
    wk = step_work(C, n)
    bytes_per_launch, flops_per_launch = wk["bytes"], wk["flops"]
    roof = roofline(bytes_per_launch, flops_per_launch, avg_fused_us, args.precision)

    line = {
        "metric": "Stokes cell-direction updates/s (forward + adjoint hot path)",
        "value": 2.0 * C * n * T / (ms_per_step / 1e3),
        "unit": "Stokes cell-direction updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "beam512: 512x512 lattice, n=32 (4 zenith x 8 azimuth), T=%d time "
                               "steps; forward with sqrt(T) checkpoints + readout + adjoint" % T,
                   "nx": 512, "ny": 512, "ndir": n, "time_steps": T, "ckpt_every": K,
                   "contraction_precision": args.precision},
        "roofline": dict(roof, kernel="fused_kernel (forward step)",
                         traffic=measured_traffic("fused_fwd_beam512_%s" % args.precision),
                         avg_launch_us=avg_fused_us,
                         algorithmic_bytes_per_launch=bytes_per_launch,
                         algorithmic_flops_per_launch=flops_per_launch,
                         executed_mfma_flops_per_launch=wk["executed_flops"]),
        "phases": {"forward_ms": ms_fwd, "adjoint_ms": ms_adj_est,
                   "adjoint_fwd_ratio": ms_adj_est / ms_fwd,
                   "forward_cell_dir_updates_per_s": C * n * T / (ms_fwd / 1e3)},
    }
    if not args.no_extras:
        del ck, seg
        torch.cuda.empty_cache()
        line["precision_speedup"] = precision_extras()
        torch.cuda.empty_cache()
        line["streaming"] = streaming_extras()
        torch.cuda.empty_cache()
        line["extensions"] = extension_extras()
        torch.cuda.empty_cache()
        line["three_d"] = three_d_extras()
        torch.cuda.empty_cache()
        line["spectral_batch"] = spectral_extras()
        torch.cuda.empty_cache()
        line["statevector"] = statevector_extras()
        torch.cuda.empty_cache()
    if not args.no_cpu:
        _log("bench: cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
