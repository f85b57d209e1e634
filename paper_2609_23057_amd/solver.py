"""Torch-facing wrapper of the C ABI: owns a context and its workspace tensor.

PyTorch supplies device memory and the stream; every computation is a call
into librtlbm.so.  Tensors must be contiguous float32 on the current CUDA/HIP
device.  State tensors have shape [n, 4, ny, nx] (the ABI layout S[d][s][y][x]).
"""
import ctypes

import numpy as np
import torch

from . import _abi as A

_ZEN = {"equal_area": A.RT_ZEN_EQUAL_AREA, "uniform_theta": A.RT_ZEN_UNIFORM_THETA,
        "explicit": A.RT_ZEN_EXPLICIT}
_PLANE = {"xy": A.RT_PLANE_XY, "xz": A.RT_PLANE_XZ, "xy_d2q9": A.RT_PLANE_XY_D2Q9, "3d": A.RT_PLANE_3D}
_PHASE = {"rayleigh": A.RT_PHASE_RAYLEIGH, "hg": A.RT_PHASE_HG, "mix": A.RT_PHASE_MIX, "table": A.RT_PHASE_TABLE}


def make_problem(nx, ny, n_zen, n_az, zen_rule="equal_area", zen_explicit_deg=None,
                 az_offset_deg=0.0, plane="xy", courant=1.0, bc=(0, 0, 0, 0), phase=None,
                 dt=1.0, precision="fp32", abs_taylor=False, scat_exp=False, fused_taylor=False,
                 renorm_irow=False, scalar=False, plain=False, nz=1, bc6=None, dir_xyz=None,
                 dir_domega=None, shift=None, mixture=None, mix_max=None, **_ignored):
    """An RtProblem from keyword arguments (names follow the ABI struct).
    mix_max defaults to the number of further phase functions a list
    `mixture` names (one for a single phase function, or none)."""
    phase = phase or {"kind": "rayleigh"}
    p = A.RtProblem()
    p.nx, p.ny, p.n_zen, p.n_az = int(nx), int(ny), int(n_zen), int(n_az)
    p.zen_rule = _ZEN[zen_rule]
    if zen_rule == "explicit":
        arr = (ctypes.c_double * int(n_zen))(*[float(z) for z in zen_explicit_deg])
        p._zen_keepalive = arr
        p.zen_deg = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    p.az_offset_deg = float(az_offset_deg)
    p.plane = _PLANE[plane]
    p.courant = float(courant)
    if plane == "3d":
        # faces x-, x+, y-, y+, z-, z+
        faces = bc6 if bc6 is not None else tuple(bc) + (0, 0)
        for e in range(4):
            p.bc[e] = int(faces[e])
        p.bc_z[0], p.bc_z[1] = int(faces[4]), int(faces[5])
        p.nz = int(nz)
    else:
        for e in range(4):
            p.bc[e] = int(bc[e])
    p.phase = _PHASE[phase.get("kind", "rayleigh")]
    p.g = float(phase.get("g", 0.0))
    p.mix_ray = float(phase.get("mix_ray", 1.0))
    if phase.get("kind") == "table":
        # rows (theta_deg, a1, a2, a3, a4, b1, b2); the library copies them at rt_init
        tab = np.ascontiguousarray(phase["table"], dtype=np.float64).reshape(-1, 7)
        p._table_keepalive = tab
        p.n_table = tab.shape[0]
        p.table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # explicit direction set (host arrays; the library copies them at rt_init)
    for name, arr, width in (("dir_xyz", dir_xyz, 3), ("dir_domega", dir_domega, 1),
                             ("shift", shift, 3 if plane == "3d" else 2)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
            if a.size != width * p.n_zen * p.n_az:
                raise ValueError("%s needs %d values" % (name, width * p.n_zen * p.n_az))
            setattr(p, "_%s_keepalive" % name, a)
            setattr(p, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    p.dt = float(dt)
    flags = 0
    flags |= A.RT_ABS_TAYLOR if abs_taylor else 0
    flags |= A.RT_SCAT_EXP if scat_exp else 0
    flags |= A.RT_FUSED_TAYLOR if fused_taylor else 0
    flags |= A.RT_RENORM_IROW if renorm_irow else 0
    flags |= A.RT_SCALAR if scalar else 0
    flags |= A.RT_PLAIN if plain else 0
    p.flags = flags
    p.precision = A.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if mix_max is None:
        mix_max = len(mixture) if isinstance(mixture, (list, tuple)) else 0
    p.mix_max = int(mix_max)
    return p


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class Solver:
    """One context: problem, workspace and stream (torch's current stream).

    A Solver made by Batch.channel() views a channel of a batch: it shares the
    batch's context, workspace and stream and does not own them."""

    def __init__(self, problem, device=None, stream=None, _ctx=None, _owner=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the solver needs a HIP device")
        self.problem = problem
        A.rt_validate(problem)
        self.device = torch.device(device or "cuda")
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.n = problem.n_zen * problem.n_az
        self.nx, self.ny = problem.nx, problem.ny
        self.nz = problem.nz if problem.plane == A.RT_PLANE_3D else 1
        # per-cell fields are [ny, nx] ([nz, ny, nx] on a 3-D lattice)
        self.cells = (self.nz, self.ny, self.nx) if problem.plane == A.RT_PLANE_3D else (self.ny, self.nx)
        self.shape = (self.n, 4) + self.cells
        if _ctx is None:
            nbytes = A.rt_workspace_bytes(problem)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.ctx = A.rt_init(problem, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
            self._owned = True
        else:
            self.ctx, self._owner, self._owned = _ctx, _owner, False
        self.nout = [A.rt_num_outgoing(problem, e) for e in range(6 if len(self.cells) == 3 else 4)]
        # What the context holds (medium, phase mixture, dichroism) and a
        # generation count bumped by every call that changes it, so that
        # RTSolve.backward can tell whether its forward's medium is still set.
        self._gen = 0
        self._medium = None
        self._mixture = None
        self._eta = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and getattr(self, "_owned", False) and A is not None and \
                getattr(A, "rt_destroy", None) is not None:
            A.rt_destroy(ctx)
            self.ctx = None

    # -- helpers ---------------------------------------------------------------
    def empty_state(self):
        return torch.zeros(self.shape, dtype=torch.float32, device=self.device)

    def state_bytes(self):
        return A.rt_state_bytes(self.problem)

    def describe(self):
        dirs = np.zeros((self.n, 6))
        M = np.zeros((4 * self.n, 4 * self.n))
        A.rt_describe(self.problem, dirs, M)
        return dirs, M

    # -- ABI calls -----------------------------------------------------------------
    def set_medium(self, tau, albedo, emis, jprof, inflow=None):
        """inflow: host [edges][n][4] (the same radiance along each edge; [6][n][4]
        faces on a 3-D lattice), or a device tensor [2 nx + 2 ny][n][4] of
        radiance per edge cell (rt_set_inflow), or None (zero)."""
        jp = np.ascontiguousarray(jprof, dtype=np.float32).reshape(self.n, 4)
        nfaces = 6 if len(self.cells) == 3 else 4   # faces of a 3-D lattice, edges of a 2-D one
        per_cell = isinstance(inflow, torch.Tensor) and inflow.is_cuda
        inf = None if (inflow is None or per_cell) else \
            np.ascontiguousarray(inflow, dtype=np.float32).reshape(nfaces, self.n, 4)
        A.rt_set_medium(self.ctx, _ptr(tau), _ptr(albedo), _ptr(emis), jp, inf)
        if per_cell:
            A.rt_set_inflow(self.ctx, _ptr(inflow))
        self._medium = (tau, albedo, emis, jp, inflow if per_cell else inf)
        self._gen += 1

    def set_phase_mixture(self, phase, frac):
        """Per-cell mixture: a fraction frac (device [ny, nx] float32) of the
        scattering follows `phase` ({"kind", "g", "mix_ray"}); with a list of
        K - 1 phase functions, frac is [K - 1, ny, nx] (each >= 0, their sum
        <= 1 per cell) and the context's own phase function keeps the rest.
        None removes the mixture."""
        self._gen += 1
        if phase is None:
            A.rt_set_phase_mixture(self.ctx, -1, 0.0, 1.0, None)
            self._mixture = None
            return
        if isinstance(phase, (list, tuple)):
            ncell = int(np.prod(self.cells))
            if frac is None or frac.numel() != len(phase) * ncell:
                raise ValueError("frac needs [%d, cells] values" % len(phase))
            A.rt_set_phase_mixture_k(self.ctx, [_PHASE[p.get("kind", "rayleigh")] for p in phase],
                                     [float(p.get("g", 0.0)) for p in phase],
                                     [float(p.get("mix_ray", 1.0)) for p in phase], _ptr(frac))
            self._mixture = ([dict(p) for p in phase], frac)
            return
        A.rt_set_phase_mixture(self.ctx, _PHASE[phase.get("kind", "rayleigh")], float(phase.get("g", 0.0)),
                               float(phase.get("mix_ray", 1.0)), _ptr(frac))
        self._mixture = (dict(phase), frac)

    def set_dichroism(self, eta):
        """Dichroic absorption with per-cell linear dichroism eta (device
        [ny, nx] float32, |eta| < 1); None removes it."""
        self._gen += 1
        A.rt_set_dichroism(self.ctx, _ptr(eta))
        self._eta = eta

    def sv_step(self, S_in, S_out=None, work=None):
        """One step of the statevector emulation of the paper's circuit:
        S_in, S_out float64 device tensors [n, 4, ny, nx]; work (optional) a
        uint8 device tensor of rt_sv_workspace_bytes().  Returns (S_out,
        success probability)."""
        if S_out is None:
            S_out = torch.empty_like(S_in)
        if S_in.dtype != torch.float64 or S_out.dtype != torch.float64:
            raise TypeError("the statevector emulation takes float64 fields")
        if work is None:
            work = self.sv_workspace()
        p = A.rt_sv_step(self.ctx, work.data_ptr(), work.numel(), S_in.data_ptr(), S_out.data_ptr())
        return S_out, p

    def sv_workspace(self):
        nbytes = A.rt_sv_workspace_bytes(self.ctx)
        if nbytes == 0:
            raise A.RTError(A.RT_EUNSUPPORTED, A.rt_last_error(self.ctx))
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def set_tile_strip(self, tiles):
        """2-D lattices: vertical strips of `tiles` tiles as the fused steps'
        tile order (0: row order); the result does not depend on it."""
        A.rt_set_tile_strip(self.ctx, int(tiles))

    def set_layer_block(self, layers):
        """3-D lattices: layers per block of the fused step's tile order (0:
        the library's default); the result does not depend on it."""
        A.rt_set_layer_block(self.ctx, int(layers))

    def medium_state(self):
        """Everything the context's operator depends on beyond the problem:
        (generation, medium, mixture, dichroism), for restore_medium()."""
        return (self._gen, self._medium, self._mixture, self._eta)

    def restore_medium(self, state):
        """Sets again what medium_state() returned, if anything changed since."""
        gen, medium, mixture, eta = state
        if gen == self._gen:
            return
        # the order keeps every intermediate combination valid: dichroism and
        # a mixture exclude each other, so the one to drop goes first
        if self._eta is not None and eta is None:
            self.set_dichroism(None)
        if self._mixture is not None and mixture is None:
            self.set_phase_mixture(None, None)
        if medium is not None:
            self.set_medium(*medium)
        if mixture is not None:
            self.set_phase_mixture(*mixture)
        if eta is not None:
            self.set_dichroism(eta)
        self._gen = gen

    def step(self, S_in, S_out):
        A.rt_step(self.ctx, _ptr(S_in), _ptr(S_out))

    def stream_field(self, S_in, S_out):
        A.rt_stream(self.ctx, _ptr(S_in), _ptr(S_out))

    def run(self, S, nsteps, ckpt=None, ckpt_every=0):
        A.rt_run(self.ctx, _ptr(S), int(nsteps), _ptr(ckpt), int(ckpt_every))

    def edge_cells(self, edge):
        """Cells of an edge (2-D) or face (3-D: x faces ny nz, y faces nx nz, z faces nx ny)."""
        if len(self.cells) == 3:
            return (self.ny * self.nz, self.nx * self.nz, self.nx * self.ny)[edge // 2]
        return self.ny if edge < 2 else self.nx

    def readout(self, S, edge, sums=False):
        out = torch.empty((self.edge_cells(edge), self.nout[edge], 4), dtype=torch.float32, device=self.device)
        h = np.zeros(4) if sums else None
        A.rt_readout(self.ctx, _ptr(S), int(edge), _ptr(out) if out.numel() else None, h)
        return (out, h) if sums else out

    def sums(self, S):
        h = np.zeros(4)
        A.rt_readout(self.ctx, _ptr(S), 0, None, h)
        return h

    def maps(self, S):
        I = torch.empty(self.cells, dtype=torch.float32, device=self.device)
        D = torch.empty_like(I)
        A.rt_maps(self.ctx, _ptr(S), _ptr(I), _ptr(D))
        return I, D

    def readout_adjoint(self, edge, gout):
        lam = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        A.rt_readout_adjoint(self.ctx, int(edge), _ptr(gout.contiguous()), _ptr(lam))
        return lam

    def checkpoint_buffer(self, nsteps, ckpt_every):
        nck = (nsteps + ckpt_every - 1) // ckpt_every
        return torch.empty((nck,) + self.shape, dtype=torch.float32, device=self.device)

    def segment_buffer(self, ckpt_every):
        k = max(ckpt_every - 1, 1)
        return torch.empty((k,) + self.shape, dtype=torch.float32, device=self.device)

    def adjoint(self, nsteps, ckpt, ckpt_every, lamT, seg=None, want_lambda0=False):
        seg = self.segment_buffer(ckpt_every) if seg is None else seg
        g = torch.empty((3,) + self.cells, dtype=torch.float32, device=self.device)
        lam0 = torch.empty(self.shape, dtype=torch.float32, device=self.device) if want_lambda0 else None
        A.rt_adjoint(self.ctx, int(nsteps), _ptr(ckpt), int(ckpt_every), _ptr(seg), _ptr(lamT),
                     _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(lam0))
        return (g[0], g[1], g[2], lam0) if want_lambda0 else (g[0], g[1], g[2])

    def synchronize(self):
        A.rt_synchronize(self.ctx)


def sqrt_checkpoint_interval(nsteps):
    """K = ceil(sqrt(T)) steps between checkpoints."""
    return max(1, int(np.ceil(np.sqrt(nsteps))))


class RTSolve(torch.autograd.Function):
    """Edge readout after nsteps as a differentiable function of the medium.

    forward(tau, albedo, emis, solver, S0, nsteps, edge, jprof, inflow) ->
    readout [edge length, outgoing directions, 4]; backward returns
    (dL/dtau, dL/dalbedo, dL/demis).  The forward stores sqrt(T) checkpoints;
    the backward replays each segment and runs the fused adjoint kernels.
    Several applications may share one solver before a backward: each
    backward sets the medium (and phase mixture / dichroism) its forward ran
    with again if another call changed it, and afterwards puts back what the
    solver held.
    """

    @staticmethod
    def forward(ctx, tau, albedo, emis, solver, S0, nsteps, edge, jprof, inflow=None):
        tau, albedo, emis = tau.contiguous(), albedo.contiguous(), emis.contiguous()
        solver.set_medium(tau, albedo, emis, jprof, inflow)
        K = sqrt_checkpoint_interval(nsteps)
        ck = solver.checkpoint_buffer(nsteps, K)
        S = S0.clone()
        solver.run(S, nsteps, ck, K)
        out = solver.readout(S, edge)
        # the medium tensors are saved so that autograd notices in-place changes
        ctx.save_for_backward(tau, albedo, emis)
        ctx.solver, ctx.nsteps, ctx.edge, ctx.K = solver, nsteps, edge, K
        ctx.ck = ck
        ctx.medium_state = solver.medium_state()
        return out

    @staticmethod
    def backward(ctx, gout):
        s = ctx.solver
        ctx.saved_tensors   # raises if a medium tensor was modified in place
        current = s.medium_state()
        s.restore_medium(ctx.medium_state)
        lam = s.readout_adjoint(ctx.edge, gout.contiguous().float())
        g_tau, g_alb, g_em = s.adjoint(ctx.nsteps, ctx.ck, ctx.K, lam)
        s.restore_medium(current)
        return g_tau, g_alb, g_em, None, None, None, None, None, None


class Batch:
    """Spectral batch: independent channels advanced together, one launch per
    time step over all channels' tiles.  Per-channel medium, readout and
    readout adjoint go through the channel views (Solver objects)."""

    def __init__(self, problems, device=None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the batch needs a HIP device")
        self.problems = list(problems)
        self.device = torch.device(device or "cuda")
        self.stream = stream or torch.cuda.current_stream(self.device)
        nbytes = A.rt_batch_workspace_bytes(self.problems)
        if nbytes == 0:
            raise A.RTError(A.RT_EINVAL, A.rt_batch_last_error())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.handle = A.rt_batch_init(self.problems, aligned, nbytes, self.stream.cuda_stream)
        self.channels = [Solver(p, self.device, self.stream, _ctx=A.rt_batch_channel(self.handle, i), _owner=self)
                         for i, p in enumerate(self.problems)]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and A is not None and getattr(A, "rt_batch_destroy", None) is not None:
            self.channels = []
            A.rt_batch_destroy(h)
            self.handle = None

    def __len__(self):
        return len(self.problems)

    def empty_states(self):
        return [c.empty_state() for c in self.channels]

    def set_graph(self, enabled):
        A.rt_batch_set_graph(self.handle, enabled)

    def classes(self):
        """[(waves per tile, block waves, channels)] of every channel class."""
        return A.rt_batch_classes(self.handle)

    def set_tuning(self, waves_per_tile, block_waves):
        """Block size (waves) of the launches of one channel class."""
        A.rt_batch_set_tuning(self.handle, waves_per_tile, block_waves)

    def set_cache_budget(self, nbytes):
        """Working-set budget of the channel groups that complete every step
        before the next group starts (0: all channels step together)."""
        A.rt_batch_set_cache_budget(self.handle, nbytes)

    def run(self, states, nsteps, ckpts=None, ckpt_every=0):
        A.rt_batch_run(self.handle, [_ptr(s) for s in states], int(nsteps),
                       None if ckpts is None else [_ptr(c) for c in ckpts], int(ckpt_every))

    def checkpoint_buffers(self, nsteps, ckpt_every):
        return [c.checkpoint_buffer(nsteps, ckpt_every) for c in self.channels]

    def segment_buffers(self, ckpt_every):
        return [c.segment_buffer(ckpt_every) for c in self.channels]

    def adjoint(self, nsteps, ckpts, ckpt_every, lamTs, segs=None):
        segs = self.segment_buffers(ckpt_every) if segs is None else segs
        grads = [torch.empty((3, c.ny, c.nx), dtype=torch.float32, device=self.device) for c in self.channels]
        A.rt_batch_adjoint(self.handle, int(nsteps), [_ptr(c) for c in ckpts], int(ckpt_every),
                           [_ptr(s) for s in segs], [_ptr(l) for l in lamTs],
                           [_ptr(g[0]) for g in grads], [_ptr(g[1]) for g in grads], [_ptr(g[2]) for g in grads])
        return [(g[0], g[1], g[2]) for g in grads]

    def synchronize(self):
        A.rt_batch_synchronize(self.handle)
