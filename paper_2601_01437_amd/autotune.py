"""Launch-shape autotuner with a JSON cache.

The library exposes launch shapes that may be chosen per system (irl_tune_knob in
the C header): the workgroup count of the table-driven D~ v and forward pass, and
the workgroup cap of the enumerating Hamiltonian apply.  Each one only moves rows
between workgroups, so the choice never changes a result bit; it changes the cost
of one matrix-vector product of the operator (Methods, "Practical Matrix-Free
Implementation").

For every knob that a system's kernels use, `tune_system` times the knob's
candidate values on the system's own operator apply with the library's kernel
events, keeps the fastest, and records it in a JSON cache keyed by the device name,
the knob and the shape that decides the kernel's work (orbitals, electrons, rows,
hidden width, Hamiltonian kernel).  A later call with the same key sets the cached
value without timing.  The timing runs through the C entry points only; this module
holds no arithmetic of the method.
"""
from __future__ import annotations

import json
import os
import tempfile

from . import binding as B

# knob -> (name, kernel class timed by irl_stats, candidate values; 0 is the built-in default)
KNOBS = {
    B.IRL_TUNE_LUT_BLOCKS: ("lut_blocks", "gemv", (0, 128, 512, 1024, 2048)),
    B.IRL_TUNE_PULL_BLOCKS: ("pull_blocks", "ham_apply", (0, 8192, 32768, 131072)),
    B.IRL_TUNE_PULL_WAVES: ("pull_waves", "ham_apply", (0, 1, 2, 4)),
}


def shape_key(device, knob, n, na, nb, ns, ham_kernel, hidden=None):
    """Cache key of one knob on one shape (hidden width only where it shapes the kernel)."""
    name = KNOBS[knob][0]
    parts = [str(device), name, f"n={n}", f"na={na}", f"nb={nb}", f"ns={ns}", f"ham={ham_kernel}"]
    if knob == B.IRL_TUNE_LUT_BLOCKS:
        parts.append(f"H={hidden}")
    return "|".join(parts)


def pick_best(timings):
    """timings: [(value, ms per launch)] in candidate order.  The fastest value; a
    candidate must beat the earlier best by more than 1% to replace it, so the
    default (listed first) is kept when the shapes tie within noise."""
    best_v, best_t = None, None
    for v, t in timings:
        if best_t is None or t < best_t * 0.99:
            best_v, best_t = v, t
    return best_v, best_t


class TuneCache:
    """A JSON file of {key: {"value": v, "ms": t, "timings": [[v, t], ...]}}."""

    def __init__(self, path=None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if not isinstance(data, dict):
                raise ValueError(f"{path}: tuning cache is not a JSON object")
            self.entries = data

    def get(self, key):
        e = self.entries.get(key)
        return None if e is None else int(e["value"])

    def put(self, key, value, ms, timings):
        self.entries[key] = {"value": int(value), "ms": float(ms),
                             "timings": [[int(v), float(t)] for v, t in timings]}

    def save(self):
        if not self.path:
            return
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _time_applies(system, v, kind, reps):
    """Mean kernel time (ms) per launch of `kind` over `reps` operator applies."""
    h = system.handle
    system.apply(v)                       # untimed: first launch at this shape
    B.irl_stats_select(h, [kind])
    B.irl_stats_enable(h, True)
    for _ in range(reps):
        system.apply(v)
    st = B.irl_stats_get(h)[kind]
    B.irl_stats_enable(h, False)
    B.irl_stats_select(h, None)
    return st[0] / max(1, st[1])


def tune_system(system, hidden, cache=None, reps=5, seed=0, device_name=None):
    """Choose every applicable knob of `system` (a System whose workspace holds an
    evaluation of a network with `hidden` units).  Returns {knob name: {"value",
    "cached", "timings"}}; knobs the system's kernels do not use are left unset.
    Timing uses the system's kernel statistics: they are cleared, and left off and
    selecting every kind, when the call returns."""
    import torch

    cache = cache if cache is not None else TuneCache(None)
    if device_name is None:
        props = torch.cuda.get_device_properties(system.device)
        device_name = f"{props.name} {getattr(props, 'gcnArchName', '')}".strip()
    dev = device_name
    info = B.irl_system_info_get(system.handle)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(system.ncols, generator=gen, dtype=torch.float64).to(system.device)
    out = {}
    for knob, (name, kind, cands) in KNOBS.items():
        _, applies = B.irl_tune_get(system.handle, knob, hidden)
        if not applies:
            continue
        key = shape_key(dev, knob, system.n, system.na, system.nb, system.ns, info.ham_kernel,
                        hidden)
        hit = cache.get(key)
        if hit is not None:
            B.irl_tune_set(system.handle, knob, hit)
            out[name] = {"value": hit, "cached": True}
            continue
        timings = []
        for c in cands:
            B.irl_tune_set(system.handle, knob, c)
            timings.append((c, _time_applies(system, v, kind, reps)))
        best, ms = pick_best(timings)
        B.irl_tune_set(system.handle, knob, best)
        cache.put(key, best, ms, timings)
        out[name] = {"value": best, "cached": False, "timings": timings}
    cache.save()
    return out
