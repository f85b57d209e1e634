"""ctypes binding of librtlbm.so: the C ABI of include/rt_lbm.h under the same names.

Argument marshalling only: every step of the solver runs in the HIP library.
Device pointers are passed as integers (for example tensor.data_ptr()).  A
non-RT_OK status raises RTError carrying rt_last_error().  If the library has
not been built, importing this module raises ImportError: there is no fallback.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_size_t, c_uint32, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtlbm.so")

RT_OK, RT_EINVAL, RT_ERANGE, RT_ESTATE, RT_ENOMEM, RT_EDEVICE, RT_EUNSUPPORTED = range(7)
RT_FP32, RT_BF16, RT_FP16, RT_BF16X3 = range(4)
RT_ZEN_EQUAL_AREA, RT_ZEN_UNIFORM_THETA, RT_ZEN_EXPLICIT = range(3)
RT_PLANE_XY, RT_PLANE_XZ, RT_PLANE_XY_D2Q9, RT_PLANE_3D = range(4)
RT_BC_PERIODIC, RT_BC_ABSORBING, RT_BC_INFLOW = range(3)
RT_PHASE_RAYLEIGH, RT_PHASE_HG, RT_PHASE_MIX, RT_PHASE_TABLE = range(4)
RT_ABS_TAYLOR, RT_SCAT_EXP, RT_FUSED_TAYLOR, RT_RENORM_IROW, RT_SCALAR, RT_PLAIN = (
    1, 2, 4, 8, 16, 32)

PRECISIONS = {"fp32": RT_FP32, "bf16": RT_BF16, "fp16": RT_FP16, "bf16x3": RT_BF16X3}


class RtProblem(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("n_zen", c_int32), ("n_az", c_int32),
                ("zen_rule", c_int32), ("zen_deg", POINTER(c_double)),
                ("az_offset_deg", c_double), ("plane", c_int32), ("courant", c_double),
                ("bc", c_int32 * 4), ("phase", c_int32), ("g", c_double), ("mix_ray", c_double),
                ("dt", c_double), ("flags", c_uint32), ("precision", c_int32),
                ("n_table", c_int32), ("table", POINTER(c_double)),
                ("nz", c_int32), ("bc_z", c_int32 * 2),
                ("dir_xyz", POINTER(c_double)), ("dir_domega", POINTER(c_double)), ("shift", POINTER(c_double)),
                ("mix_max", c_int32)]


RT_MIX_MAX = 7


class RTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_STATUS = {RT_OK: "RT_OK", RT_EINVAL: "RT_EINVAL", RT_ERANGE: "RT_ERANGE",
           RT_ESTATE: "RT_ESTATE", RT_ENOMEM: "RT_ENOMEM", RT_EDEVICE: "RT_EDEVICE",
           RT_EUNSUPPORTED: "RT_EUNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError("librtlbm.so is not built; run python paper_2609_23057_amd/build.py")
# torch ships its own HIP runtime under the same soname (libamdhip64.so.7); it
# must be the one loaded, so that the library and torch share one runtime (and
# one view of the device, streams and memory).  Import torch before the CDLL.
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

_P = POINTER(RtProblem)
_SIGS = {
    "rt_validate": (c_int32, [_P]),
    "rt_workspace_bytes": (c_size_t, [_P]),
    "rt_state_bytes": (c_size_t, [_P]),
    "rt_describe": (c_int32, [_P, c_void_p, c_void_p]),
    "rt_num_outgoing": (c_int32, [_P, c_int32]),
    "rt_init": (c_int32, [_P, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "rt_set_medium": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rt_set_phase_mixture": (c_int32, [c_void_p, c_int32, c_double, c_double, c_void_p]),
    "rt_set_phase_mixture_k": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rt_set_dichroism": (c_int32, [c_void_p, c_void_p]),
    "rt_set_layer_block": (c_int32, [c_void_p, c_int32]),
    "rt_set_tile_strip": (c_int32, [c_void_p, c_int32]),
    "rt_set_inflow": (c_int32, [c_void_p, c_void_p]),
    "rt_step": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "rt_stream": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "rt_run": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32]),
    "rt_readout": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "rt_maps": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "rt_totals_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "rt_sv_qubits": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "rt_sv_workspace_bytes": (c_size_t, [c_void_p]),
    "rt_sv_gate_count": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_double)]),
    "rt_sv_step": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p, POINTER(c_double)]),
    "rt_sv_set_fusion": (c_int32, [c_void_p, c_int32]),
    "rt_sv_launch_count": (c_int32, [c_void_p, POINTER(c_int32)]),
    "rt_readout_adjoint": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "rt_adjoint_segment_bytes": (c_size_t, [_P, c_int32]),
    "rt_adjoint": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p]),
    "rt_batch_workspace_bytes": (c_size_t, [_P, c_int32]),
    "rt_batch_init": (c_int32, [_P, c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "rt_batch_channel": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
    "rt_batch_run": (c_int32, [c_void_p, POINTER(c_void_p), c_int32, POINTER(c_void_p), c_int32]),
    "rt_batch_adjoint": (c_int32, [c_void_p, c_int32, POINTER(c_void_p), c_int32, POINTER(c_void_p),
                                   POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                   POINTER(c_void_p)]),
    "rt_batch_num_classes": (c_int32, [c_void_p, POINTER(c_int32)]),
    "rt_batch_class": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "rt_batch_set_tuning": (c_int32, [c_void_p, c_int32, c_int32]),
    "rt_batch_set_cache_budget": (c_int32, [c_void_p, c_size_t]),
    "rt_batch_set_graph": (c_int32, [c_void_p, c_int32]),
    "rt_batch_synchronize": (c_int32, [c_void_p]),
    "rt_batch_destroy": (c_int32, [c_void_p]),
    "rt_batch_last_error": (c_char_p, [c_void_p]),
    "rt_synchronize": (c_int32, [c_void_p]),
    "rt_destroy": (c_int32, [c_void_p]),
    "rt_status_str": (c_char_p, [c_int32]),
    "rt_last_error": (c_char_p, [c_void_p]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status, ctx=None):
    if status != RT_OK:
        msg = _lib.rt_last_error(ctx)
        raise RTError(status, msg.decode() if msg else "")


def rt_status_str(status):
    return _lib.rt_status_str(status).decode()


def rt_last_error(ctx=None):
    m = _lib.rt_last_error(ctx)
    return m.decode() if m else ""


def rt_validate(p):
    _check(_lib.rt_validate(ctypes.byref(p)))


def rt_workspace_bytes(p):
    return int(_lib.rt_workspace_bytes(ctypes.byref(p)))


def rt_state_bytes(p):
    return int(_lib.rt_state_bytes(ctypes.byref(p)))


def rt_describe(p, h_dirs=None, h_M=None):
    """h_dirs / h_M: numpy float64 arrays ([n,6], [4n,4n]) or None."""
    _check(_lib.rt_describe(ctypes.byref(p),
                            None if h_dirs is None else h_dirs.ctypes.data,
                            None if h_M is None else h_M.ctypes.data))


def rt_num_outgoing(p, edge):
    return int(_lib.rt_num_outgoing(ctypes.byref(p), edge))


def rt_init(p, d_ws, ws_bytes, stream):
    out = c_void_p()
    _check(_lib.rt_init(ctypes.byref(p), d_ws, ws_bytes, stream, ctypes.byref(out)))
    return out.value


def rt_set_medium(ctx, d_tau, d_albedo, d_emis, h_jprof, h_inflow=None):
    """h_jprof / h_inflow: numpy float32 arrays ([n,4], [4,n,4]) or None."""
    _check(_lib.rt_set_medium(ctx, d_tau, d_albedo, d_emis, h_jprof.ctypes.data,
                              None if h_inflow is None else h_inflow.ctypes.data), ctx)


def rt_set_phase_mixture(ctx, phase2, g2, mix_ray2, d_frac):
    """phase2 < 0 removes the mixture; d_frac: device [ny][nx] float32 in [0, 1]."""
    _check(_lib.rt_set_phase_mixture(ctx, phase2, g2, mix_ray2, d_frac), ctx)


def rt_set_phase_mixture_k(ctx, phases, gs, mix_rays, d_frac):
    """K - 1 = len(phases) further phase functions (host lists; empty removes
    the mixture); d_frac: device [K - 1][ny][nx] float32, each >= 0, sum <= 1."""
    k = len(phases)
    if not (len(gs) == len(mix_rays) == k):
        raise ValueError("phases, gs and mix_rays must have one entry per further phase function")
    ph = (c_int32 * max(k, 1))(*phases)
    g = (c_double * max(k, 1))(*gs)
    mr = (c_double * max(k, 1))(*mix_rays)
    _check(_lib.rt_set_phase_mixture_k(ctx, k, ph, g, mr, d_frac if k else None), ctx)


def rt_set_dichroism(ctx, d_eta):
    """d_eta: device [ny][nx] float32 with |eta| < 1, or None to remove it."""
    _check(_lib.rt_set_dichroism(ctx, d_eta), ctx)


def rt_set_layer_block(ctx, layers):
    """3-D lattices: layers per block of the fused step's tile order (0: default)."""
    _check(_lib.rt_set_layer_block(ctx, layers), ctx)


def rt_set_tile_strip(ctx, tiles):
    """2-D fused steps: tile order in vertical strips of `tiles` tiles (0: row order)."""
    _check(_lib.rt_set_tile_strip(ctx, tiles), ctx)


def rt_set_inflow(ctx, d_inflow):
    _check(_lib.rt_set_inflow(ctx, d_inflow), ctx)


def rt_step(ctx, d_S_in, d_S_out):
    _check(_lib.rt_step(ctx, d_S_in, d_S_out), ctx)


def rt_stream(ctx, d_in, d_out):
    _check(_lib.rt_stream(ctx, d_in, d_out), ctx)


def rt_run(ctx, d_S, nsteps, d_ckpt=None, ckpt_every=0):
    _check(_lib.rt_run(ctx, d_S, nsteps, d_ckpt, ckpt_every), ctx)


def rt_readout(ctx, d_S, edge, d_out=None, h_sums=None):
    """h_sums: numpy float64 array of 4 or None."""
    _check(_lib.rt_readout(ctx, d_S, edge, d_out,
                           None if h_sums is None else h_sums.ctypes.data), ctx)


def rt_totals_noalloc(ctx, d_S, d_sums):
    _check(_lib.rt_totals_noalloc(ctx, d_S, d_sums), ctx)


def rt_sv_qubits(ctx):
    """(total qubits, data qubits) of the context's emulated circuit."""
    nq, nd = c_int32(0), c_int32(0)
    _check(_lib.rt_sv_qubits(ctx, ctypes.byref(nq), ctypes.byref(nd)), ctx)
    return nq.value, nd.value


def rt_sv_workspace_bytes(ctx):
    return _lib.rt_sv_workspace_bytes(ctx)


def rt_sv_gate_count(ctx):
    """(gate launches, translation launches, statevector bytes moved) per step."""
    g, s, b = c_int32(0), c_int32(0), c_double(0.0)
    _check(_lib.rt_sv_gate_count(ctx, ctypes.byref(g), ctypes.byref(s), ctypes.byref(b)), ctx)
    return g.value, s.value, b.value


def rt_sv_set_fusion(ctx, max_qubits):
    """Target qubits of a fused gate pass (0 .. 3; 0: every gate alone)."""
    _check(_lib.rt_sv_set_fusion(ctx, int(max_qubits)), ctx)


def rt_sv_launch_count(ctx):
    n = c_int32()
    _check(_lib.rt_sv_launch_count(ctx, ctypes.byref(n)), ctx)
    return n.value


def rt_sv_step(ctx, d_work, work_bytes, d_S_in, d_S_out):
    """One emulated circuit step (float64 fields); returns the success probability."""
    p = c_double(0.0)
    _check(_lib.rt_sv_step(ctx, d_work, work_bytes, d_S_in, d_S_out, ctypes.byref(p)), ctx)
    return p.value


def rt_maps(ctx, d_S, d_I_mean, d_dop_mean):
    _check(_lib.rt_maps(ctx, d_S, d_I_mean, d_dop_mean), ctx)


def rt_readout_adjoint(ctx, edge, d_gout, d_lambdaT):
    _check(_lib.rt_readout_adjoint(ctx, edge, d_gout, d_lambdaT), ctx)


def rt_adjoint_segment_bytes(p, ckpt_every):
    return int(_lib.rt_adjoint_segment_bytes(ctypes.byref(p), ckpt_every))


def rt_adjoint(ctx, nsteps, d_ckpt, ckpt_every, d_seg, d_lambdaT, d_g_tau, d_g_albedo, d_g_emis,
               d_lambda0=None):
    _check(_lib.rt_adjoint(ctx, nsteps, d_ckpt, ckpt_every, d_seg, d_lambdaT, d_g_tau,
                           d_g_albedo, d_g_emis, d_lambda0), ctx)


def _bcheck(status, b=None):
    if status != RT_OK:
        msg = _lib.rt_batch_last_error(b)
        raise RTError(status, msg.decode() if msg else "")


def _ptrs(seq):
    """Host array of device pointers (None -> NULL array)."""
    if seq is None:
        return None
    return (c_void_p * len(seq))(*[int(x) if x else None for x in seq])


def _probs(probs):
    arr = (RtProblem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = p
    return arr


def rt_batch_workspace_bytes(probs):
    return int(_lib.rt_batch_workspace_bytes(_probs(probs), len(probs)))


def rt_batch_init(probs, d_ws, ws_bytes, stream):
    out = c_void_p()
    _bcheck(_lib.rt_batch_init(_probs(probs), len(probs), d_ws, ws_bytes, stream, ctypes.byref(out)))
    return out.value


def rt_batch_channel(b, ch):
    out = c_void_p()
    _bcheck(_lib.rt_batch_channel(b, ch, ctypes.byref(out)), b)
    return out.value


def rt_batch_run(b, d_states, nsteps, d_ckpts=None, ckpt_every=0):
    """d_states / d_ckpts: sequences of per-channel device pointers (ints)."""
    _bcheck(_lib.rt_batch_run(b, _ptrs(d_states), nsteps, _ptrs(d_ckpts), ckpt_every), b)


def rt_batch_adjoint(b, nsteps, d_ckpts, ckpt_every, d_segs, d_lambdaT, d_g_tau, d_g_albedo, d_g_emis):
    _bcheck(_lib.rt_batch_adjoint(b, nsteps, _ptrs(d_ckpts), ckpt_every, _ptrs(d_segs), _ptrs(d_lambdaT),
                                  _ptrs(d_g_tau), _ptrs(d_g_albedo), _ptrs(d_g_emis)), b)


def rt_batch_classes(b):
    """[(waves per tile, block waves, channels)] of every channel class."""
    n = c_int32(0)
    _bcheck(_lib.rt_batch_num_classes(b, ctypes.byref(n)), b)
    out = []
    for k in range(n.value):
        w, bw, nc = c_int32(0), c_int32(0), c_int32(0)
        _bcheck(_lib.rt_batch_class(b, k, ctypes.byref(w), ctypes.byref(bw), ctypes.byref(nc)), b)
        out.append((w.value, bw.value, nc.value))
    return out


def rt_batch_set_tuning(b, waves_per_tile, block_waves):
    _bcheck(_lib.rt_batch_set_tuning(b, int(waves_per_tile), int(block_waves)), b)


def rt_batch_set_cache_budget(b, nbytes):
    _bcheck(_lib.rt_batch_set_cache_budget(b, int(nbytes)), b)


def rt_batch_set_graph(b, enabled):
    _bcheck(_lib.rt_batch_set_graph(b, int(enabled)), b)


def rt_batch_synchronize(b):
    _bcheck(_lib.rt_batch_synchronize(b), b)


def rt_batch_destroy(b):
    _bcheck(_lib.rt_batch_destroy(b))


def rt_batch_last_error(b=None):
    m = _lib.rt_batch_last_error(b)
    return m.decode() if m else ""


def rt_synchronize(ctx):
    _check(_lib.rt_synchronize(ctx), ctx)


def rt_destroy(ctx):
    _check(_lib.rt_destroy(ctx))
