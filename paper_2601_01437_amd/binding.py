"""ctypes binding of ``include/irlnqs.h`` (argument marshalling only).

Every function keeps the name of its C entry point and forwards to it; all
arithmetic runs in the HIP library ``lib/libirlnqs.so``.  Device arrays are
torch tensors on the current HIP device (their ``data_ptr()`` is passed), host
arrays are numpy arrays, streams default to torch's current stream.  The
library is required: importing this module without it raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int8, c_int32, c_int64, c_size_t, c_uint8
from ctypes import c_uint32, c_uint64, c_void_p

import numpy as np
# torch owns the device memory and streams the library works on, so both must run
# on one HIP runtime.  torch ships its own libamdhip64.so.7 (same soname as the
# system's), and whichever is loaded first serves the process: load torch before
# the library so the library's HIP and HSA dependencies resolve to torch's copies.
# (Loaded the other way round, the library's first device call found no device.)
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libirlnqs.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_01437_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/irlnqs.h) -------------------------------------------
IRL_OK, IRL_ENOTCONV, IRL_ESTEP = 0, 1, 2
IRL_EINVAL, IRL_ENOMEM, IRL_EDEVICE, IRL_ESTATE = -1, -2, -3, -4
IRL_FP64, IRL_FP32 = 0, 1
IRL_MODE_A, IRL_MODE_P, IRL_MODE_C = 0, 1, 2
IRL_WS_FP64, IRL_WS_FP32, IRL_WS_BLOCK, IRL_WS_FACTORED, IRL_WS_SAMPLED = 1, 2, 4, 8, 16
IRL_STEP_WS_CURRENT, IRL_STEP_NO_EVAL_AFTER, IRL_STEP_NO_UPDATE, IRL_STEP_NO_POLISH = 1, 2, 4, 8
IRL_STEP_FULL_CYCLES = 16
IRL_STEP_GRAPH = 32
IRL_STEP_WARM_START = 64
IRL_SYS_FORCE_HASH = 1
IRL_SYS_FORCE_PULL = 2
IRL_SYS_STORE_SLICED = 4
IRL_SYS_STORE_BLOCKS = 8
IRL_TUNE_LUT_BLOCKS, IRL_TUNE_PULL_BLOCKS, IRL_TUNE_PULL_WAVES = 0, 1, 2
STAT_KINDS = ("dtilde_build", "ham_apply", "gemv", "gemv_t", "reduce", "energy", "lanczos", "ritz",
              "gemv_fp32", "gemv_t_fp32", "vmc")

STATUS_NAMES = {0: "IRL_OK", 1: "IRL_ENOTCONV", 2: "IRL_ESTEP", -1: "IRL_EINVAL",
                -2: "IRL_ENOMEM", -3: "IRL_EDEVICE", -4: "IRL_ESTATE"}


class IrlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class irl_system_desc(ctypes.Structure):
    _fields_ = [("n_orb", c_int32), ("n_alpha", c_int32), ("n_beta", c_int32),
                ("h", c_void_p), ("g", c_void_p), ("e_core", c_double),
                ("dets", c_void_p), ("n_dets", c_int64), ("flags", c_uint32)]


class irl_system_info(ctypes.Structure):
    _fields_ = [("n_dets", c_int64), ("n_orb", c_int32), ("n_alpha", c_int32),
                ("n_beta", c_int32), ("full_space", c_int32), ("n_alpha_strings", c_int64),
                ("n_beta_strings", c_int64), ("max_connections", c_int64),
                ("device_bytes", c_size_t), ("ham_kernel", c_int32), ("stored_col_blocks", c_int32),
                ("stored_elements", c_int64)]


class irl_nqs_desc(ctypes.Structure):
    _fields_ = [("V", c_int32), ("H", c_int32), ("theta", c_void_p)]


class irl_eval_out(ctypes.Structure):
    _fields_ = [("Z", c_double), ("E", c_double), ("grad", c_void_p)]


class irl_solver_opts(ctypes.Structure):
    _fields_ = [("m", c_int32), ("k_keep", c_int32), ("tol", c_double),
                ("max_restarts", c_int32), ("precision", c_int32), ("mode", c_int32),
                ("seed", c_uint64), ("flags", c_uint32), ("block", c_int32)]


class irl_adam_opts(ctypes.Structure):
    _fields_ = [("lr", c_double), ("beta1", c_double), ("beta2", c_double), ("eps", c_double)]


class irl_vmc_out(ctypes.Structure):
    _fields_ = [("E_sampled", c_double), ("E_exact", c_double), ("E_loc_var", c_double),
                ("n_unique", c_int64), ("n_samples", c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class irl_step_result(ctypes.Structure):
    _fields_ = [("E_before", c_double), ("E_after", c_double), ("lambda_min", c_double),
                ("residual_est", c_double), ("residual_explicit", c_double),
                ("tol_used", c_double), ("c0", c_double), ("gap", c_double),
                ("norm_T", c_double), ("n_apply", c_int32), ("n_restart", c_int32),
                ("converged", c_int32), ("n_apply_lo", c_int32), ("ms_eval", c_double),
                ("ms_solve", c_double), ("ms_after", c_double), ("n_graph_cycles", c_int32),
                ("reserved", c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_SYS = c_void_p
_sigs = {
    "irl_system_create": (c_int32, [POINTER(irl_system_desc), c_void_p, POINTER(_SYS)]),
    "irl_system_destroy": (None, [_SYS]),
    "irl_system_info_get": (c_int32, [_SYS, POINTER(irl_system_info)]),
    "irl_system_store_hamiltonian": (c_int32, [_SYS, c_size_t, POINTER(c_size_t), c_void_p]),
    "irl_last_error": (c_char_p, [_SYS]),
    "irl_workspace_query": (c_int32, [_SYS, c_int64, c_uint32, POINTER(c_size_t)]),
    "irl_nqs_evaluate": (c_int32, [_SYS, POINTER(irl_nqs_desc), c_void_p, c_size_t, c_uint32,
                                   POINTER(irl_eval_out), c_void_p]),
    "irl_dtilde_set": (c_int32, [_SYS, c_void_p, c_int64, c_int64, c_int32, c_void_p, c_size_t,
                                 c_uint32, c_void_p]),
    "irl_apply_lm_operator": (c_int32, [_SYS, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                                        c_int32, c_void_p]),
    "irl_apply_lm_operator_block": (c_int32, [_SYS, c_void_p, c_size_t, c_void_p, c_int64, c_int32,
                                              c_void_p, c_void_p, c_int64, c_int32, c_void_p]),
    "irl_apply_hamiltonian": (c_int32, [_SYS, c_void_p, c_void_p, c_void_p]),
    "irl_step": (c_int32, [_SYS, POINTER(irl_nqs_desc), POINTER(irl_solver_opts), c_void_p,
                           c_size_t, c_uint32, c_void_p, c_void_p, POINTER(irl_step_result),
                           c_void_p]),
    "irl_solver_opts_default": (None, [POINTER(irl_solver_opts)]),
    "irl_adam_step": (c_int32, [_SYS, POINTER(irl_nqs_desc), c_void_p, c_size_t, c_uint32,
                                POINTER(irl_adam_opts), c_void_p, c_void_p, c_int64,
                                POINTER(irl_eval_out), c_void_p]),
    "irl_vmc_sample": (c_int32, [_SYS, c_void_p, c_size_t, c_void_p, c_int64, c_void_p, c_void_p,
                                 POINTER(irl_vmc_out), c_void_p]),
    "irl_stats_enable": (c_int32, [_SYS, c_int32]),
    "irl_stats_select": (c_int32, [_SYS, c_uint32]),
    "irl_stats_get": (c_int32, [_SYS, c_void_p, c_void_p, c_void_p]),
    "irl_tune_set": (c_int32, [_SYS, c_int32, c_int32]),
    "irl_tune_get": (c_int32, [_SYS, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "irl_batch_create": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32,
                                   POINTER(c_void_p)]),
    "irl_batch_destroy": (None, [c_void_p]),
    "irl_batch_step": (c_int32, [c_void_p, POINTER(irl_solver_opts), c_void_p, c_void_p, c_void_p,
                                 c_void_p]),
    "irl_debug_keys": (c_int32, [_SYS, c_void_p]),
    "irl_debug_lookup": (c_int32, [_SYS, c_void_p, c_int64, c_void_p]),
    "irl_lookup_noalloc": (c_int32, [_SYS, c_void_p, c_int64, c_void_p, c_void_p]),
    "irl_debug_diagonal": (c_int32, [_SYS, c_void_p]),
    "irl_debug_excitations": (c_int32, [_SYS, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_int64, POINTER(c_int64)]),
    "irl_debug_jacobian": (c_int32, [_SYS, c_void_p, c_size_t, c_int64, c_int64, c_void_p, c_void_p,
                                     POINTER(c_int32), POINTER(c_int64)]),
    "irl_debug_lanczos": (c_int32, [_SYS, c_void_p, c_size_t, c_void_p, c_int32, c_int32, c_int32,
                                    c_void_p, c_void_p, c_void_p, c_void_p]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sigs)


def _stream(stream):
    if stream is not None:
        return c_void_p(int(stream))
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _check(rc, sys=None, ok=(IRL_OK,)):
    if rc in ok:
        return rc
    msg = _lib.irl_last_error(sys)
    raise IrlError(rc, (msg or b"").decode())


# ---- same-named wrappers -----------------------------------------------------

def irl_system_create(n, n_alpha, n_beta, h, g, dets=None, e_core=0.0, flags=0, stream=None):
    """Returns an opaque handle (c_void_p).  h, g, dets: host numpy arrays."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert h.size == n * n and g.size == n ** 4
    d = irl_system_desc(n, n_alpha, n_beta, h.ctypes.data, g.ctypes.data, float(e_core), None, 0,
                        flags)
    if dets is not None:
        dets = np.ascontiguousarray(dets, dtype=np.uint64)
        d.dets = dets.ctypes.data
        d.n_dets = dets.size
    out = _SYS()
    _check(_lib.irl_system_create(ctypes.byref(d), _stream(stream), ctypes.byref(out)))
    return out


def irl_system_destroy(sys):
    _lib.irl_system_destroy(sys)


def irl_system_info_get(sys):
    info = irl_system_info()
    _check(_lib.irl_system_info_get(sys, ctypes.byref(info)), sys)
    return info


def irl_system_store_hamiltonian(sys, max_bytes, stream=None):
    """Returns (stored: bool, bytes_needed).  Over budget is not an error here:
    the system stays matrix-free and stored is False."""
    need = c_size_t()
    rc = _lib.irl_system_store_hamiltonian(sys, int(max_bytes), ctypes.byref(need), _stream(stream))
    _check(rc, sys, ok=(IRL_OK, IRL_ENOMEM))
    return rc == IRL_OK, need.value


def irl_last_error(sys=None):
    return (_lib.irl_last_error(sys) or b"").decode()


def irl_workspace_query(sys, ncols, ws_flags):
    nbytes = c_size_t()
    _check(_lib.irl_workspace_query(sys, ncols, ws_flags, ctypes.byref(nbytes)), sys)
    return nbytes.value


def irl_nqs_evaluate(sys, V, H, theta, ws, ws_flags, grad=None, stream=None):
    """theta, ws, grad: device tensors.  Returns (Z, E)."""
    nqs = irl_nqs_desc(V, H, theta.data_ptr())
    out = irl_eval_out(0.0, 0.0, None if grad is None else grad.data_ptr())
    _check(_lib.irl_nqs_evaluate(sys, ctypes.byref(nqs), _ptr(ws), ws.numel() * ws.element_size(),
                                 ws_flags, ctypes.byref(out), _stream(stream)), sys)
    return out.Z, out.E


def irl_adam_step(sys, V, H, theta, ws, ws_flags, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, grad=None, stream=None):
    """One Adam step on theta (device, in place); m, v: device moment tensors (P).
    Returns (Z, E) at theta before the update."""
    nqs = irl_nqs_desc(V, H, theta.data_ptr())
    o = irl_adam_opts(lr, beta1, beta2, eps)
    out = irl_eval_out(0.0, 0.0, None if grad is None else grad.data_ptr())
    _check(_lib.irl_adam_step(sys, ctypes.byref(nqs), _ptr(ws), ws.numel() * ws.element_size(), ws_flags,
                              ctypes.byref(o), _ptr(m), _ptr(v), t, ctypes.byref(out), _stream(stream)), sys)
    return out.Z, out.E


def irl_vmc_sample(sys, ws, u, rows=None, grad=None, stream=None):
    """u: device float64 tensor of uniforms; rows: optional device int64 tensor of
    the same length; grad: optional device float64 tensor (P).  Returns irl_vmc_out."""
    out = irl_vmc_out()
    _check(_lib.irl_vmc_sample(sys, _ptr(ws), ws.numel() * ws.element_size(), _ptr(u), u.numel(),
                               _ptr(rows), _ptr(grad), ctypes.byref(out), _stream(stream)), sys)
    return out


def irl_dtilde_set(sys, D, ws, ws_flags, stream=None):
    """D: device tensor (n_dets x ncols), float64 or float32, row-major."""
    import torch
    dtype = IRL_FP64 if D.dtype == torch.float64 else IRL_FP32
    assert D.dim() == 2 and D.stride(1) == 1
    _check(_lib.irl_dtilde_set(sys, _ptr(D), D.stride(0), D.shape[1], dtype, _ptr(ws),
                               ws.numel() * ws.element_size(), ws_flags, _stream(stream)), sys)


def irl_apply_lm_operator(sys, ws, v, yH, yS, precision=IRL_FP64, stream=None):
    _check(_lib.irl_apply_lm_operator(sys, _ptr(ws), ws.numel() * ws.element_size(), _ptr(v),
                                      _ptr(yH), _ptr(yS), precision, _stream(stream)), sys)


def irl_apply_lm_operator_block(sys, ws, V, YH, YS, precision=IRL_FP64, stream=None):
    """V, YH, YS: device float64 tensors of shape (nb, ldv) / (nb, ldy), one vector per row."""
    nb = V.shape[0]
    assert V.stride(1) == 1 and YH.stride(1) == 1 and YS.stride(1) == 1 and YH.stride(0) == YS.stride(0)
    _check(_lib.irl_apply_lm_operator_block(sys, _ptr(ws), ws.numel() * ws.element_size(), _ptr(V), V.stride(0),
                                            nb, _ptr(YH), _ptr(YS), YH.stride(0), precision, _stream(stream)),
           sys)


def irl_apply_hamiltonian(sys, w, u, stream=None):
    _check(_lib.irl_apply_hamiltonian(sys, _ptr(w), _ptr(u), _stream(stream)), sys)


def irl_solver_opts_default():
    o = irl_solver_opts()
    _lib.irl_solver_opts_default(ctypes.byref(o))
    return o


def irl_step(sys, opts, ws, ws_flags, V=None, H=None, theta=None, dtheta=None, ritz=None,
             stream=None, allow=(IRL_OK, IRL_ENOTCONV, IRL_ESTEP)):
    """One optimisation step.  Returns (status, irl_step_result)."""
    nqs = None
    if theta is not None:
        nqs = irl_nqs_desc(V, H, theta.data_ptr())
    res = irl_step_result()
    rc = _lib.irl_step(sys, None if nqs is None else ctypes.byref(nqs), ctypes.byref(opts),
                       _ptr(ws), ws.numel() * ws.element_size(), ws_flags, _ptr(dtheta),
                       _ptr(ritz), ctypes.byref(res), _stream(stream))
    _check(rc, sys, ok=allow)
    return rc, res


def irl_stats_enable(sys, on=True):
    _check(_lib.irl_stats_enable(sys, 1 if on else 0), sys)


def irl_stats_select(sys, kinds=None):
    """Time only the named kinds (names of STAT_KINDS); None: every kind."""
    mask = (1 << len(STAT_KINDS)) - 1 if kinds is None else sum(1 << STAT_KINDS.index(k) for k in kinds)
    _check(_lib.irl_stats_select(sys, mask), sys)


def irl_stats_get(sys, stream=None):
    """{kind: (total_ms, launches)} since the last irl_stats_enable."""
    ms = np.zeros(len(STAT_KINDS), dtype=np.float64)
    cnt = np.zeros(len(STAT_KINDS), dtype=np.int64)
    _check(_lib.irl_stats_get(sys, ms.ctypes.data, cnt.ctypes.data, _stream(stream)), sys)
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(STAT_KINDS)}


def irl_tune_set(sys, knob, value):
    _check(_lib.irl_tune_set(sys, int(knob), int(value)), sys)


def irl_tune_get(sys, knob, hidden=1):
    """(value, applies): the knob's value (0 = default) and whether the system uses it."""
    value, applies = c_int32(0), c_int32(0)
    _check(_lib.irl_tune_get(sys, int(knob), int(hidden), ctypes.byref(value), ctypes.byref(applies)), sys)
    return int(value.value), bool(applies.value)


def irl_batch_create(systems, nqs, ws, ws_flags):
    """systems: handles; nqs: list of (V, H, theta tensor); ws: list of device uint8 tensors."""
    n = len(systems)
    sys_arr = (c_void_p * n)(*[s.value if isinstance(s, c_void_p) else s for s in systems])
    nqs_arr = (irl_nqs_desc * n)(*[irl_nqs_desc(V, H, th.data_ptr()) for V, H, th in nqs])
    ws_arr = (c_void_p * n)(*[w.data_ptr() for w in ws])
    sizes = (c_size_t * n)(*[w.numel() * w.element_size() for w in ws])
    out = c_void_p()
    _check(_lib.irl_batch_create(n, sys_arr, nqs_arr, ws_arr, sizes, ws_flags, ctypes.byref(out)),
           systems[0])
    return out


def irl_batch_destroy(batch):
    _lib.irl_batch_destroy(batch)


def irl_batch_step(batch, opts, count, dtheta=None, first_system=None, stream=None):
    """Returns (list of irl_step_result, list of status codes)."""
    res = (irl_step_result * count)()
    status = (c_int32 * count)()
    dth = None
    if dtheta is not None:
        dth = (c_void_p * count)(*[None if t is None else t.data_ptr() for t in dtheta])
    _check(_lib.irl_batch_step(batch, ctypes.byref(opts), dth, res, status, _stream(stream)),
           first_system)
    return list(res), list(status)


def irl_debug_keys(sys, n_dets):
    out = np.empty(n_dets, dtype=np.uint64)
    _check(_lib.irl_debug_keys(sys, out.ctypes.data), sys)
    return out


def irl_debug_lookup(sys, keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    rows = np.empty(keys.size, dtype=np.int32)
    _check(_lib.irl_debug_lookup(sys, keys.ctypes.data, keys.size, rows.ctypes.data), sys)
    return rows


def irl_lookup_noalloc(sys, keys, stream=None):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    rows = np.empty(keys.size, dtype=np.int32)
    _check(_lib.irl_lookup_noalloc(sys, keys.ctypes.data, keys.size, rows.ctypes.data, _stream(stream)), sys)
    return rows


def irl_debug_diagonal(sys, n_dets):
    out = np.empty(n_dets, dtype=np.float64)
    _check(_lib.irl_debug_diagonal(sys, out.ctypes.data), sys)
    return out


def irl_debug_jacobian(sys, ws, row0, nrows):
    """(psi, rows, kind): psi FP64[nrows]; rows d (kind 0, FP64 nrows x H) or
    D~ rows (kind 1 FP64, kind 2 FP32; nrows x (P+1))."""
    kind, nc = c_int32(0), c_int64(0)
    _check(_lib.irl_debug_jacobian(sys, _ptr(ws), ws.numel(), row0, 0, None, None, ctypes.byref(kind),
                                   ctypes.byref(nc)), sys)
    psi = np.empty(nrows, dtype=np.float64)
    rows = np.empty((nrows, nc.value), dtype=np.float32 if kind.value == 2 else np.float64)
    _check(_lib.irl_debug_jacobian(sys, _ptr(ws), ws.numel(), row0, nrows, psi.ctypes.data, rows.ctypes.data,
                                   ctypes.byref(kind), ctypes.byref(nc)), sys)
    return psi, rows, kind.value


def irl_debug_excitations(sys, row, cap=70000):
    tgt = np.empty(cap, dtype=np.int32)
    sg = np.empty(cap, dtype=np.int8)
    kd = np.empty(cap, dtype=np.uint8)
    hv = np.empty(cap, dtype=np.float64)
    cnt = c_int64()
    _check(_lib.irl_debug_excitations(sys, row, tgt.ctypes.data, sg.ctypes.data, kd.ctypes.data,
                                      hv.ctypes.data, cap, ctypes.byref(cnt)), sys)
    c = cnt.value
    return tgt[:c].copy(), sg[:c].copy(), kd[:c].copy(), hv[:c].copy()


def irl_debug_lanczos(sys, ws, v1, j_end, ncols, precision=IRL_FP64, mode=IRL_MODE_A, stream=None):
    V = np.empty((j_end + 1, ncols), dtype=np.float64)
    a = np.empty(j_end, dtype=np.float64)
    b = np.empty(j_end, dtype=np.float64)
    _check(_lib.irl_debug_lanczos(sys, _ptr(ws), ws.numel() * ws.element_size(), _ptr(v1), j_end,
                                  precision, mode, V.ctypes.data, a.ctypes.data, b.ctypes.data,
                                  _stream(stream)), sys)
    return V, a, b
