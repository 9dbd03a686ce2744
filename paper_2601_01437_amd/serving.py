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
    spec: "ClassSpec | None" = None   # the request's own class (FootprintServer)


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


# --------------------------------------------------------------------------
# Admission by footprint: requests of any system class (n, electrons, set,
# network width), admitted when the device bytes of their slot fit a budget.


def _binom(n: int, k: int) -> int:
    from math import comb
    return comb(n, k) if 0 <= k <= n else 0


def estimate_system_bytes(n: int, na: int, nb: int, n_dets: int | None) -> int:
    """Upper bound on the device bytes of a determinant system before it is
    created (keys, diagonal, integrals, lookup tables, and on full spaces the
    rank and per-string move tables of the string-product Hamiltonian and its
    dense same-spin matrices), with a margin.  The exact figure is read from the
    created system (irl_system_info.device_bytes)."""
    cA, cB = _binom(n, na), _binom(n, nb)
    full = n_dets is None or (n_dets == cA * cB and n <= 24)
    ns = cA * cB if full else int(n_dets)
    b = 16 * ns + 8 * (n * n + n ** 4)
    if full:
        b += 8 * (1 << n) + 4 * (cA + cB)
        for N, nstr in ((na, cA), (nb, cB)):
            ns1 = max(N * (n - N), 1)
            nd = max(_binom(N, 2) * _binom(n - N, 2), 1)
            b += nstr * (ns1 * 14 + nd * 12 + n * n * 8)
            if nstr <= 2048:
                b += 8 * nstr * nstr
    else:
        cap = 64
        while cap < 2 * ns:
            cap <<= 1
        # hash and membership bitmap; beta-major and alpha-major block tables (string
        # -> block, block starts, and the alpha-major rows with their beta strings)
        b += 12 * cap + (1 << 25) // 8 + 8 * (1 << min(n, 24)) + 8 * (ns + 1) + 8 * ns
    return int(b * 1.25) + (4 << 20)


@dataclass
class Slot:
    """A resident system with its workspace and parameter buffer."""
    key: tuple
    system: System
    theta: torch.Tensor
    nbytes: int
    last_used: float = 0.0


class FootprintAdmission:
    """Host bookkeeping of admission by footprint (no device work): the bytes of
    resident slots against a budget, idle slots per class key kept for reuse and
    evicted least recently used first when a new slot needs the room.

    create(spec, room) returns a Slot, or the exact bytes the slot needs when that
    exceeds room; the first creation of a class is tried against an estimate,
    later ones against the class's known size."""

    def __init__(self, budget_bytes: int, create, destroy):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0
        self.idle: dict = {}
        self.known: dict = {}        # class key -> bytes of its slot
        self._create = create
        self._destroy = destroy
        self.created = self.evicted = self.reused = 0

    def _make_room(self, need: int, keep_key) -> bool:
        """Evict idle slots of other classes (least recently used first) until need
        fits; evicts nothing when even all of them would not make the room."""
        evictable = sum(s.nbytes for k, lst in self.idle.items() if k != keep_key for s in lst)
        if self.used - evictable + need > self.budget:
            return False
        while self.used + need > self.budget:
            _, k, i = min((s.last_used, k, i) for k, lst in self.idle.items() if k != keep_key
                          for i, s in enumerate(lst))
            s = self.idle[k].pop(i)
            self._destroy(s)
            self.used -= s.nbytes
            self.evicted += 1
        return True

    def acquire(self, key, spec, estimate: int):
        """A slot for one request of class `key`, or None when it does not fit now."""
        if self.idle.get(key):
            self.reused += 1
            return self.idle[key].pop()
        need = self.known.get(key, estimate)
        if not self._make_room(need, key):
            return None
        res = self._create(spec, self.budget - self.used)
        if not isinstance(res, Slot):
            self.known[key] = int(res)
            if not self._make_room(int(res), key):
                return None
            res = self._create(spec, self.budget - self.used)
            if not isinstance(res, Slot):
                return None
        self.known[key] = res.nbytes
        self.used += res.nbytes
        self.peak = max(self.peak, self.used)
        self.created += 1
        return res

    def release(self, slot: Slot, now: float) -> None:
        slot.last_used = now
        self.idle.setdefault(slot.key, []).append(slot)

    def close(self) -> None:
        for lst in self.idle.values():
            for s in lst:
                self._destroy(s)
                self.used -= s.nbytes
        self.idle = {}


def class_key(spec: ClassSpec) -> tuple:
    """Requests with equal keys can share slots (and a batch)."""
    import hashlib
    h = hashlib.sha256()
    for a in (spec.h, spec.g) + ((spec.dets,) if spec.dets is not None else ()):
        h.update(np.ascontiguousarray(a).tobytes())
    return (spec.n, spec.na, spec.nb, spec.V, spec.H, spec.precision, spec.factored, spec.m, spec.k_keep,
            h.hexdigest())


class FootprintServer:
    """Serves requests of any class (Request.spec) under a device-byte budget.

    The dispatcher admits arrived requests in arrival order: a request takes an
    idle slot of its class, or a new slot (system, stored rows as far as the room
    allows, workspace) when the estimated system bytes plus the workspace bytes
    from irl_workspace_query fit the budget after evicting idle slots of other
    classes; a request that does not fit waits while later ones that fit go
    ahead.  Admitted requests start at once: up to `lanes` lanes (a host thread
    and a HIP stream each, default priority) run concurrently, and a lane takes
    every admitted request of one class waiting at that moment as one batch (up
    to `max_batch`).  Slots return to the idle pool after the step."""

    def __init__(self, budget_bytes: int, lanes: int = 4, max_batch: int = 8, device="cuda"):
        self.device = device
        self.lanes = lanes
        self.max_batch = max_batch
        self.adm = FootprintAdmission(budget_bytes, self._create, self._destroy)

    def _create(self, spec: ClassSpec, room: int):
        """A slot of the class (system, stored rows when the class asks for them and
        they fit its allowance, workspace, parameters), or the bytes it needs when
        that exceeds room (nothing is kept then)."""
        s = System(spec.n, spec.na, spec.nb, spec.h, spec.g, dets=spec.dets, device=self.device)
        try:
            ws_bytes = B.irl_workspace_query(s.handle, spec.P + 1, spec.ws_flags)
            need = s.info.device_bytes + ws_bytes + spec.P * 8
            rows = 0
            if spec.store_rows_bytes and not s.info.full_space:
                stored, rows = s.store_hamiltonian(0)     # the byte count only
                if rows > spec.store_rows_bytes:
                    rows = 0
                need += rows
            if need > room:
                s.close()
                return need
            if rows:
                s.store_hamiltonian(rows)
            s.workspace(spec.P + 1, spec.ws_flags)
            theta = torch.empty(spec.P, dtype=torch.float64, device=self.device)
            nbytes = s.info.device_bytes + s.ws.numel() + theta.numel() * 8
        except Exception:
            s.close()
            raise
        return Slot(class_key(spec), s, theta, nbytes)

    @staticmethod
    def _destroy(slot: Slot) -> None:
        slot.system.close()

    def _step(self, spec: ClassSpec, reqs: list, slots: list) -> None:
        for r, sl in zip(reqs, slots):
            sl.theta.copy_(torch.from_numpy(r.theta))
        opts = dict(m=spec.m, k_keep=spec.k_keep, tol=spec.tol, precision=spec.precision)
        if len(reqs) == 1 or spec.P + 1 > 8192:
            for r, sl in zip(reqs, slots):
                rc, res, _, _ = sl.system.step(sl.theta, spec.V, spec.H, ws_flags=spec.ws_flags,
                                               want_dtheta=False, **opts)
                _fill(r, rc, res, 1)
            return
        bt = Batch([sl.system for sl in slots], [sl.theta for sl in slots], [spec.V] * len(reqs),
                   [spec.H] * len(reqs), ws_flags=spec.ws_flags)
        try:
            res, status, _ = bt.step(**opts)
        finally:
            bt.close()
        for r, rs, st in zip(reqs, res, status):
            _fill(r, st, rs, len(reqs))

    def run(self, requests: list[Request]) -> float:
        """Serve the requests (Request.spec set, arrival times relative to now);
        returns the makespan in seconds."""
        import queue
        reqs = sorted(requests, key=lambda r: r.arrival)
        ready: dict = {}                 # class key -> list of (request, slot) admitted, not yet started
        lock = threading.Condition()
        done_slots: "queue.Queue" = queue.Queue()
        errors: list = []
        busy = [0]
        t0 = [0.0]

        def lane():
            stream = torch.cuda.Stream()     # default priority
            while True:
                with lock:
                    while not ready and not stop[0]:
                        lock.wait(0.05)
                    if not ready and stop[0]:
                        return
                    key = next(iter(ready))
                    group = ready[key][:self.max_batch]
                    ready[key] = ready[key][self.max_batch:]
                    if not ready[key]:
                        del ready[key]
                    busy[0] += 1
                try:
                    with torch.cuda.stream(stream):
                        start = time.perf_counter() - t0[0]
                        self._step(group[0][0].spec, [g[0] for g in group], [g[1] for g in group])
                        stream.synchronize()
                        end = time.perf_counter() - t0[0]
                    for r, _ in group:
                        r.start, r.end = start, end
                except Exception as e:  # surfaced by run()
                    errors.append(e)
                finally:
                    for _, sl in group:
                        done_slots.put(sl)
                    with lock:
                        busy[0] -= 1
                        lock.notify_all()

        stop = [False]
        torch.cuda.synchronize()
        t0[0] = time.perf_counter()
        threads = [threading.Thread(target=lane, daemon=True) for _ in range(self.lanes)]
        for th in threads:
            th.start()
        pending: list = []
        i = 0
        try:
            while i < len(reqs) or pending:
                now = time.perf_counter() - t0[0]
                while i < len(reqs) and reqs[i].arrival <= now:
                    pending.append(reqs[i])
                    i += 1
                while not done_slots.empty():
                    self.adm.release(done_slots.get(), time.perf_counter() - t0[0])
                admitted = []
                for r in pending:
                    est = estimate_system_bytes(r.spec.n, r.spec.na, r.spec.nb,
                                                None if r.spec.dets is None else len(r.spec.dets))
                    slot = self.adm.acquire(class_key(r.spec), r.spec, est)
                    if slot is not None:
                        admitted.append((r, slot))
                if admitted:
                    ids = {id(r) for r, _ in admitted}
                    pending = [r for r in pending if id(r) not in ids]
                    with lock:
                        for r, sl in admitted:
                            ready.setdefault(sl.key, []).append((r, sl))
                        lock.notify_all()
                if errors:
                    break
                if not admitted:
                    if pending:
                        with lock:
                            idle_run = busy[0] == 0 and not ready and done_slots.empty()
                        if idle_run:
                            # nothing runs and nothing can be released: the first
                            # waiting request does not fit even with every idle slot of
                            # another class evicted
                            raise RuntimeError(f"request {pending[0].rid} does not fit the budget "
                                               f"of {self.adm.budget} bytes")
                    time.sleep(0.002)
        finally:
            with lock:
                stop[0] = True
                lock.notify_all()
            for th in threads:
                th.join()
            while not done_slots.empty():
                self.adm.release(done_slots.get(), time.perf_counter() - t0[0])
        torch.cuda.synchronize()
        if errors:
            raise RuntimeError(f"lane failed: {errors[0]}") from errors[0]
        return max((r.end for r in requests), default=0.0)

    def close(self) -> None:
        self.adm.close()
