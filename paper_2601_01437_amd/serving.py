"""Step serving with continuous admission.

A request is one IRL optimisation step (Methods, "The IRL for Wavefunction
Optimization") of its own network on one resident system class.  Each class
keeps a pool of resident slots (a system handle plus a workspace that holds
that slot's D~ and Krylov state) sized up front to the device memory the class
is allowed (HBM admission).  A lane per class (one host thread, one HIP stream
at the default priority) loops: it admits every request of its class that has
arrived, up to the free slots, steps them together (one batch of grouped
launches, or the solo path for a single request or a class the batch does not
take), and returns them.  Requests that arrive while a lane is busy join its
next admission.  Lanes run concurrently, so a long step of a large class does
not hold back the small classes.

Marshalling and scheduling only: every step runs in the HIP library.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from .system import Batch, System


@dataclass
class Request:
    rid: int
    cls: str
    arrival: float            # seconds after the start of the run
    theta: np.ndarray         # network parameters [a, b, W] (host)
    start: float = float("nan")
    end: float = float("nan")
    status: int = -99
    lambda_min: float = float("nan")
    E_before: float = float("nan")
    E_after: float = float("nan")
    n_apply: int = 0
    converged: int = 0
    batch_size: int = 0


@dataclass
class ClassSpec:
    name: str
    n: int
    na: int
    nb: int
    V: int
    H: int
    h: np.ndarray
    g: np.ndarray
    dets: np.ndarray | None = None
    m: int = 20
    k_keep: int = 1
    tol: float = 1e-12
    precision: int = B.IRL_FP32
    slots: int = 1
    store_rows_bytes: int = 0     # device bytes allowed for stored H rows per slot
    factored: bool = False        # FP64 through the factored Jacobian instead of a D~ copy

    @property
    def P(self) -> int:
        return self.V * self.H + self.H + self.V

    @property
    def ws_flags(self) -> int:
        if self.precision == B.IRL_FP64:
            return B.IRL_WS_FACTORED if self.factored else B.IRL_WS_FP64
        return B.IRL_WS_FP32


class ClassPool:
    """Resident slots of one class: system handles, workspaces, theta buffers."""

    def __init__(self, spec: ClassSpec, device="cuda"):
        self.spec = spec
        self.systems, self.thetas = [], []
        for _ in range(spec.slots):
            s = System(spec.n, spec.na, spec.nb, spec.h, spec.g, dets=spec.dets, device=device)
            if spec.store_rows_bytes and not s.info.full_space:
                s.store_hamiltonian(spec.store_rows_bytes)
            s.workspace(spec.P + 1, spec.ws_flags)
            self.systems.append(s)
            self.thetas.append(torch.empty(spec.P, dtype=torch.float64, device=device))
        # the batch takes rows of at most 8192 columns
        self.batchable = spec.P + 1 <= 8192

    def device_bytes(self) -> int:
        return sum(s.info.device_bytes + s.ws.numel() for s in self.systems)

    def step(self, reqs: list[Request]):
        """One optimisation step of each request (len(reqs) <= slots), on the
        current stream; fills the result fields."""
        sp = self.spec
        for r, th in zip(reqs, self.thetas):
            th.copy_(torch.from_numpy(r.theta))
        opts = dict(m=sp.m, k_keep=sp.k_keep, tol=sp.tol, precision=sp.precision)
        if len(reqs) == 1 or not self.batchable:
            for r, s, th in zip(reqs, self.systems, self.thetas):
                rc, res, _, _ = s.step(th, sp.V, sp.H, ws_flags=sp.ws_flags, want_dtheta=False, **opts)
                _fill(r, rc, res, 1)
            return
        nr = len(reqs)
        bt = Batch(self.systems[:nr], self.thetas[:nr], [sp.V] * nr, [sp.H] * nr, ws_flags=sp.ws_flags)
        try:
            res, status, _ = bt.step(**opts)
        finally:
            bt.close()
        for r, rs, st in zip(reqs, res, status):
            _fill(r, st, rs, nr)

    def close(self):
        for s in self.systems:
            s.close()
        self.systems, self.thetas = [], []


def _fill(r: Request, rc, res, nbatch):
    r.status = int(rc)
    r.lambda_min = res.lambda_min
    r.E_before = res.E_before
    r.E_after = res.E_after
    r.n_apply = res.n_apply
    r.converged = res.converged
    r.batch_size = nbatch


class Server:
    """Runs requests against resident class pools; one lane per class."""

    def __init__(self, pools: dict[str, ClassPool]):
        self.pools = pools

    def _lane(self, name: str, reqs: list[Request], t0: float, errors: list):
        pool = self.pools[name]
        stream = torch.cuda.Stream()     # default priority
        try:
            with torch.cuda.stream(stream):
                i = 0
                while i < len(reqs):
                    now = time.perf_counter() - t0
                    if reqs[i].arrival > now:
                        time.sleep(min(reqs[i].arrival - now, 0.05))
                        continue
                    j = i
                    while j < len(reqs) and j - i < len(pool.systems) and reqs[j].arrival <= now:
                        j += 1
                    group = reqs[i:j]
                    i = j
                    start = time.perf_counter() - t0
                    pool.step(group)
                    stream.synchronize()
                    end = time.perf_counter() - t0
                    for r in group:
                        r.start, r.end = start, end
        except Exception as e:  # surfaced by run()
            errors.append((name, e))

    def run(self, requests: list[Request]) -> float:
        """Serve the requests (arrival times relative to now); returns the
        makespan in seconds.  Blocks until every request is done."""
        by_cls = {name: sorted([r for r in requests if r.cls == name], key=lambda r: r.arrival)
                  for name in self.pools}
        errors: list = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lanes = [threading.Thread(target=self._lane, args=(name, rs, t0, errors), daemon=True)
                 for name, rs in by_cls.items() if rs]
        for th in lanes:
            th.start()
        for th in lanes:
            th.join()
        torch.cuda.synchronize()
        if errors:
            name, e = errors[0]
            raise RuntimeError(f"lane {name} failed: {e}") from e
        return max((r.end for r in requests), default=0.0)


def run_sequential(pools: dict[str, ClassPool], requests: list[Request]) -> float:
    """Reference schedule: one request at a time in arrival order, solo path,
    on the current stream; returns the makespan in seconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.start = time.perf_counter() - t0
        pools[r.cls].step([r])
        torch.cuda.current_stream().synchronize()
        r.end = time.perf_counter() - t0
    return max((r.end for r in requests), default=0.0)


def latency_summary(requests: list[Request]) -> dict:
    lat = np.array([r.end - r.arrival for r in requests])
    out = {"n": int(lat.size)}
    if lat.size:
        out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                    "p99_ms": float(np.percentile(lat, 99) * 1e3),
                    "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)})
    return out
