"""Seeded synthetic inputs for the IRL / linear-method operator library.

This module generates *inputs only*: one- and two-electron integrals, NQS
parameters, and determinant sets selected by a seeded sampler.  It holds none of
the method's arithmetic (no Slater-Condon rules, no NQS evaluation, no Lanczos),
so both the oracle and the GPU path can take their inputs from it without
sharing any computation.

Random draws (all with ``numpy.random.default_rng``; sigma is a standard
deviation):

* integrals, seed ``s``: ``default_rng(s)``.  First ``h[p, q]`` for ``p <= q`` in
  row-major order, each ``N(0, 1) * exp(-|p - q| / 2)``, mirrored.  Then one
  draw per 8-fold symmetry class of the chemists' two-electron integral
  ``(pq|rs)``: compound pair index ``PQ = p(p+1)/2 + q`` (``p >= q``) ascending,
  and for each ``PQ`` the index ``RS <= PQ`` ascending; each draw is
  ``N(0, 0.1) * exp(-(|p - q| + |r - s|) / 2)`` and is written to all eight
  index permutations.
* NQS parameters, seed ``s``: ``default_rng([s, 1]).normal(0, 0.05, P)`` in the
  parameter order ``[a (V), b (H), W (H x V, row-major)]``.
* selected determinant sets (sampler), seed ``s``: ``default_rng([s, 2])``.

Determinant keys: alpha orbital ``p`` is bit ``p`` and beta orbital ``p`` is bit
``32 + p`` of a ``uint64``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "integrals",
    "nqs_theta",
    "n_params",
    "probe_vector",
    "cisd_like_selected_set",
    "capped_set",
    "Workload",
    "WORKLOADS",
    "batch_workloads",
    "serving_arrivals",
    "key_of",
]


def key_of(alpha: int, beta: int) -> int:
    """Pack an alpha and a beta occupation bit string into one uint64 key."""
    return int(alpha) | (int(beta) << 32)


def integrals(n: int, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Random molecule-like integrals: symmetric ``h`` (n x n) and 8-fold
    symmetric chemists' ``g[p, q, r, s] = (pq|rs)`` (n^4), both float64."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    for p in range(n):
        for q in range(p, n):
            val = rng.normal(0.0, 1.0) * math.exp(-abs(p - q) / 2.0)
            h[p, q] = val
            h[q, p] = val
    pairs = [(p, q) for p in range(n) for q in range(p + 1)]  # PQ order
    g = np.zeros((n, n, n, n))
    for PQ, (p, q) in enumerate(pairs):
        for RS in range(PQ + 1):
            r, s = pairs[RS]
            val = rng.normal(0.0, 0.1) * math.exp(-(abs(p - q) + abs(r - s)) / 2.0)
            for (a, b) in ((p, q), (q, p)):
                for (c, d) in ((r, s), (s, r)):
                    g[a, b, c, d] = val
                    g[c, d, a, b] = val
    return h, g


def n_params(V: int, H: int) -> int:
    """Parameter count of the one-hidden-layer network: a (V) + b (H) + W (H*V)."""
    return V * H + H + V


def nqs_theta(V: int, H: int, seed: int = 0, scale: float = 0.05) -> np.ndarray:
    """Random NQS parameters ``theta`` in the order ``[a, b, W]``."""
    rng = np.random.default_rng([seed, 1])
    return rng.normal(0.0, scale, size=n_params(V, H))


def probe_vector(ncols: int, seed: int = 0) -> np.ndarray:
    """A seeded N(0, 1) vector of length ncols (operator-apply test input)."""
    return np.random.default_rng([seed, 7]).normal(size=ncols)


def _strings_by_rank(n: int, ne: int, max_rank: int):
    """Occupation strings of ``ne`` electrons in ``n`` orbitals reachable from the
    aufbau string (orbitals ``0..ne-1``) by moving at most ``max_rank`` electrons.

    Returns arrays (bits, rank, d) with ``d = sum(particle indices) - sum(hole
    indices)``."""
    occ = list(range(ne))
    vir = list(range(ne, n))
    bits, rank, dsum = [], [], []
    aufbau = (1 << ne) - 1
    for r in range(0, min(max_rank, ne, n - ne) + 1):
        for holes in itertools.combinations(occ, r):
            hmask = sum(1 << i for i in holes)
            for parts in itertools.combinations(vir, r):
                pmask = sum(1 << a for a in parts)
                bits.append((aufbau & ~hmask) | pmask)
                rank.append(r)
                dsum.append(sum(parts) - sum(holes))
    return (np.array(bits, dtype=np.uint64), np.array(rank, dtype=np.int64),
            np.array(dsum, dtype=np.int64))


def _pairs_up_to_rank(n, na, nb, max_rank):
    """All (alpha, beta) pairs with total excitation rank <= max_rank from the
    aufbau determinant.  Returns keys, rank, d (unsorted)."""
    ab, ar, ad = _strings_by_rank(n, na, max_rank)
    bb, br, bd = _strings_by_rank(n, nb, max_rank)
    keys, rank, dsum = [], [], []
    for ra in range(max_rank + 1):
        ia = np.nonzero(ar == ra)[0]
        if ia.size == 0:
            continue
        ib = np.nonzero(br <= max_rank - ra)[0]
        if ib.size == 0:
            continue
        A, B = np.meshgrid(ia, ib, indexing="ij")
        A = A.ravel()
        B = B.ravel()
        keys.append(ab[A] | (bb[B] << np.uint64(32)))
        rank.append(ar[A] + br[B])
        dsum.append(ad[A] + bd[B])
    return np.concatenate(keys), np.concatenate(rank), np.concatenate(dsum)


def cisd_like_selected_set(n: int, na: int, nb: int, n_keep: int, seed: int = 0,
                           max_rank: int = 4) -> np.ndarray:
    """Seeded CISD-like selection of ``n_keep`` determinants, ascending keys.

    Candidates are all determinants within ``max_rank`` excitations of the
    aufbau determinant.  Each gets a model coefficient with
    ``log|c| = -r ln 10 - d / 4 + ln|z|`` (``z ~ N(0, 1)`` drawn in ascending
    key order); the ``n_keep`` largest ``|c|`` are kept, ties broken by key."""
    keys, rank, dsum = _pairs_up_to_rank(n, na, nb, max_rank)
    order = np.argsort(keys, kind="stable")
    keys, rank, dsum = keys[order], rank[order], dsum[order]
    if n_keep >= keys.size:
        return keys.copy()
    rng = np.random.default_rng([seed, 2])
    z = rng.normal(0.0, 1.0, size=keys.size)
    with np.errstate(divide="ignore"):
        logc = -rank * math.log(10.0) - dsum / 4.0 + np.log(np.abs(z))
    # primary: larger log|c| first; secondary: smaller key first
    sel = np.lexsort((keys, -logc))[:n_keep]
    return np.sort(keys[sel])


def capped_set(n: int, na: int, nb: int, cap: int) -> np.ndarray:
    """Full (na, nb) space if it has at most ``cap`` determinants, else the
    ``cap`` determinants smallest in (excitation rank, d, key); ascending keys."""
    full = math.comb(n, na) * math.comb(n, nb)
    max_rank = min(na, n - na) + min(nb, n - nb)
    if full <= cap:
        keys, _, _ = _pairs_up_to_rank(n, na, nb, max_rank)
        return np.sort(keys)
    # grow the rank cut until enough candidates exist
    for r_cut in range(0, max_rank + 1):
        keys, rank, dsum = _pairs_up_to_rank(n, na, nb, r_cut)
        if keys.size >= cap:
            break
    sel = np.lexsort((keys, dsum, rank))[:cap]
    return np.sort(keys[sel])


@dataclass
class Workload:
    """One synthetic problem: system, network, and solver settings."""
    name: str
    n: int
    na: int
    nb: int
    V: int
    H: int
    seed: int = 0
    m: int = 20
    k: int = 1
    steps: int = 1
    n_dets: int | None = None   # None: full space
    selection: str = "full"      # "full" | "cisd" | "capped"
    precision: str = "fp64"      # operator precision: "fp64" | "fp32"
    extra: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return n_params(self.V, self.H)

    def full_size(self) -> int:
        return math.comb(self.n, self.na) * math.comb(self.n, self.nb)

    def size(self) -> int:
        if self.selection == "full":
            return self.full_size()
        return min(self.full_size(), int(self.n_dets))

    def integrals(self):
        return integrals(self.n, self.seed)

    def theta(self) -> np.ndarray:
        return nqs_theta(self.V, self.H, self.seed)

    def dets(self) -> np.ndarray | None:
        """Explicit determinant set, or None for the full space (enumerated by
        the code under test)."""
        if self.selection == "full":
            return None
        if self.selection == "cisd":
            return cisd_like_selected_set(self.n, self.na, self.nb, int(self.n_dets),
                                          seed=self.seed)
        if self.selection == "capped":
            return capped_set(self.n, self.na, self.nb, int(self.n_dets))
        raise ValueError(self.selection)


WORKLOADS: dict[str, Workload] = {
    # 8 spatial orbitals, 4a+4b, all 4900 determinants, V=16, H=16, P=288
    "c1": Workload("c1", n=8, na=4, nb=4, V=16, H=16, seed=0, m=20, k=1, steps=1),
    # 12 spatial orbitals, 6a+6b, 853,776 determinants, V=24, H=64, P=1624
    "c2": Workload("c2", n=12, na=6, nb=6, V=24, H=64, seed=0, m=40, k=10, steps=5),
    # 20 spatial orbitals, 10a+10b, 2^20 selected determinants, V=40, H=256
    "c3": Workload("c3", n=20, na=10, nb=10, V=40, H=256, seed=0, m=20, k=1, steps=1,
                   n_dets=1 << 20, selection="cisd", precision="fp32"),
    # scaled-down c3: same orbitals and network, 2^14 selected determinants
    "c3s": Workload("c3s", n=20, na=10, nb=10, V=40, H=256, seed=0, m=20, k=1,
                    steps=1, n_dets=1 << 14, selection="cisd", precision="fp32"),
}


def batch_workloads(count: int = 64, cap: int = 1 << 18, seed: int = 0):
    """Independent small solves with uneven sizes: n ~ U{8..16}, half filled,
    hidden width ~ U{16..128}; determinant set = full space capped at ``cap``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(8, 17))
        H = int(rng.integers(16, 129))
        na, nb = (n + 1) // 2, n // 2
        full = math.comb(n, na) * math.comb(n, nb)
        sel = "full" if full <= cap else "capped"
        out.append(Workload(f"b{i}", n=n, na=na, nb=nb, V=2 * n, H=H, seed=i, m=20,
                            k=1, steps=1, n_dets=None if sel == "full" else cap,
                            selection=sel))
    return out


def serving_arrivals(n_requests: int, rate: float, mix: dict[str, float], seed: int = 0):
    """Poisson arrival times (rate per second) and workload names drawn from
    ``mix`` (name -> weight)."""
    rng = np.random.default_rng([seed, 3])
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    names = list(mix)
    w = np.array([mix[k] for k in names], dtype=float)
    picks = rng.choice(len(names), size=n_requests, p=w / w.sum())
    return np.cumsum(gaps), [names[i] for i in picks]
