"""Convenience owner of one system handle and its workspace (torch device memory).

Marshalling only: every method forwards to one C entry point.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class System:
    """A determinant set with its Hamiltonian on the current HIP device."""

    def __init__(self, n, n_alpha, n_beta, h, g, dets=None, e_core=0.0, flags=0, device=None):
        self.device = torch.device(device or "cuda")
        self.n, self.na, self.nb = n, n_alpha, n_beta
        with torch.cuda.device(self.device):
            self.handle = B.irl_system_create(n, n_alpha, n_beta, h, g, dets=dets, e_core=e_core,
                                              flags=flags)
        self.info = B.irl_system_info_get(self.handle)
        self.ns = self.info.n_dets
        self.ws = None
        self.ws_flags = 0
        self.ncols = 0

    # -- lifetime --
    def close(self):
        if self.handle is not None:
            B.irl_system_destroy(self.handle)
            self.handle = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def store_hamiltonian(self, max_bytes):
        """Store H's rows in device memory if they fit in max_bytes; returns
        (stored, bytes_needed)."""
        with torch.cuda.device(self.device):
            stored, need = B.irl_system_store_hamiltonian(self.handle, max_bytes)
        self.info = B.irl_system_info_get(self.handle)
        return stored, need

    # -- workspace --
    def workspace(self, ncols, ws_flags=B.IRL_WS_FP64):
        nbytes = B.irl_workspace_query(self.handle, ncols, ws_flags)
        if self.ws is None or self.ws.numel() < nbytes or self.ws_flags != ws_flags or self.ncols != ncols:
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws_flags = ws_flags
        self.ncols = ncols
        return self.ws

    # -- calls --
    def keys(self):
        return B.irl_debug_keys(self.handle, self.ns)

    def diagonal(self):
        return B.irl_debug_diagonal(self.handle, self.ns)

    def lookup(self, keys):
        return B.irl_debug_lookup(self.handle, keys)

    def excitations(self, row):
        return B.irl_debug_excitations(self.handle, row)

    def jacobian_rows(self, row0, nrows):
        """(psi, rows, kind) of the current evaluation (see irl_debug_jacobian)."""
        return B.irl_debug_jacobian(self.handle, self.ws, row0, nrows)

    def evaluate(self, V, H, theta, ws_flags=B.IRL_WS_FP64, want_grad=True):
        P = V * H + H + V
        ws = self.workspace(P + 1, ws_flags)
        grad = torch.empty(P, dtype=torch.float64, device=self.device) if want_grad else None
        Z, E = B.irl_nqs_evaluate(self.handle, V, H, theta, ws, ws_flags, grad=grad)
        return Z, E, grad

    def adam_step(self, V, H, theta, m, v, t, ws_flags=B.IRL_WS_FP64, grad=None, **opts):
        """One Adam step on theta (in place); returns (Z, E) before the update."""
        P = V * H + H + V
        self.workspace(P + 1, ws_flags)
        return B.irl_adam_step(self.handle, V, H, theta, self.ws, ws_flags, m, v, t, grad=grad, **opts)

    def vmc_sample(self, u, want_rows=False, want_grad=False):
        """Draw len(u) samples (u: device float64 uniforms) and switch the workspace
        to the sampled estimators; returns (irl_vmc_out, rows or None, F or None)."""
        rows = torch.empty(u.numel(), dtype=torch.int64, device=self.device) if want_rows else None
        grad = torch.empty(self.ncols - 1, dtype=torch.float64, device=self.device) if want_grad else None
        out = B.irl_vmc_sample(self.handle, self.ws, u, rows=rows, grad=grad)
        return out, rows, grad

    def set_dtilde(self, D, ws_flags=B.IRL_WS_FP64):
        ws = self.workspace(D.shape[1], ws_flags)
        B.irl_dtilde_set(self.handle, D, ws, ws_flags)

    def apply(self, v, precision=B.IRL_FP64):
        yH = torch.empty(self.ncols, dtype=torch.float64, device=self.device)
        yS = torch.empty_like(yH)
        B.irl_apply_lm_operator(self.handle, self.ws, v, yH, yS, precision)
        return yH, yS

    def apply_block(self, V, precision=B.IRL_FP64):
        """V: (nb, P+1) device float64; returns (YH, YS) of the same shape."""
        YH = torch.empty_like(V)
        YS = torch.empty_like(V)
        B.irl_apply_lm_operator_block(self.handle, self.ws, V, YH, YS, precision)
        return YH, YS

    def apply_hamiltonian(self, w):
        u = torch.empty_like(w)
        B.irl_apply_hamiltonian(self.handle, w, u)
        return u

    def step(self, theta=None, V=None, H=None, m=20, k_keep=1, tol=1e-12, max_restarts=300,
             precision=B.IRL_FP64, mode=B.IRL_MODE_A, seed=0, flags=0, ws_flags=None,
             want_dtheta=True, want_ritz=False, block=0):
        o = B.irl_solver_opts_default()
        o.m, o.k_keep, o.tol, o.max_restarts = m, k_keep, tol, max_restarts
        o.precision, o.mode, o.seed, o.flags, o.block = precision, mode, seed, flags, block
        if ws_flags is None:
            ws_flags = self.ws_flags or (B.IRL_WS_FP64 if precision == B.IRL_FP64 else B.IRL_WS_FP32)
        if theta is not None:
            P = V * H + H + V
            ws = self.workspace(P + 1, ws_flags)
        else:
            ws = self.ws
            P = self.ncols - 1
        dth = torch.empty(P, dtype=torch.float64, device=self.device) if want_dtheta else None
        ritz = None
        if want_ritz:
            ritz = torch.empty(P + 1 if mode != B.IRL_MODE_P else P, dtype=torch.float64,
                               device=self.device)
        rc, res = B.irl_step(self.handle, o, ws, ws_flags, V=V, H=H, theta=theta, dtheta=dth,
                             ritz=ritz)
        return rc, res, dth, ritz


def to_device(x, device="cuda", dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(device)


class Batch:
    """Independent optimisations stepped together with grouped kernels."""

    def __init__(self, systems, thetas, Vs, Hs, ws_flags=B.IRL_WS_FP64):
        self.systems = list(systems)
        self.thetas = list(thetas)
        self.ws = [s.workspace(V * H + H + V + 1, ws_flags) for s, V, H in zip(self.systems, Vs, Hs)]
        self.Ps = [V * H + H + V for V, H in zip(Vs, Hs)]
        self.ws_flags = ws_flags
        self.handle = B.irl_batch_create([s.handle for s in self.systems],
                                         list(zip(Vs, Hs, self.thetas)), self.ws, ws_flags)

    def step(self, m=20, k_keep=1, tol=1e-12, max_restarts=300, precision=B.IRL_FP64,
             mode=B.IRL_MODE_A, seed=0, flags=0, want_dtheta=False):
        o = B.irl_solver_opts_default()
        o.m, o.k_keep, o.tol, o.max_restarts = m, k_keep, tol, max_restarts
        o.precision, o.mode, o.seed, o.flags = precision, mode, seed, flags
        dth = None
        if want_dtheta:
            dth = [torch.empty(P, dtype=torch.float64, device=s.device)
                   for s, P in zip(self.systems, self.Ps)]
        res, status = B.irl_batch_step(self.handle, o, len(self.systems), dtheta=dth,
                                       first_system=self.systems[0].handle)
        return res, status, dth

    def close(self):
        if self.handle is not None:
            B.irl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
