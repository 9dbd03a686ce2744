"""Brute-force second-quantised Hamiltonian on a fixed-particle Fock sector.

Independent of oracle/hamiltonian.py: every term h_pq a+_p a_q and
1/2 (pq|rs) a+_p a+_r a_s a_q (spin-orbital operators, Jordan-Wigner signs) is
applied literally to each occupation string.  No Slater-Condon rule is used.
Spin-orbital k < n is alpha orbital k, k >= n is beta orbital k - n; a state is
a^+_{k1} a^+_{k2} ... |0> with k1 < k2 < ..., so operator k picks up
(-1)^(number of occupied spin-orbitals below k).
"""
from __future__ import annotations

import itertools

import numpy as np


def _apply(ops, state):
    """Apply an operator product (rightmost acts first).  ops: [(is_create, k)]."""
    sign = 1
    for create, k in reversed(ops):
        occ = (state >> k) & 1
        if create == bool(occ):
            return 0, 0
        if bin(state & ((1 << k) - 1)).count("1") & 1:
            sign = -sign
        state ^= 1 << k
    return sign, state


def sector_states(n, na, nb):
    out = []
    for A in itertools.combinations(range(n), na):
        for B in itertools.combinations(range(n), nb):
            s = sum(1 << p for p in A) | sum(1 << (n + p) for p in B)
            out.append(s)
    return sorted(out)


def to_key(state, n):
    alpha = state & ((1 << n) - 1)
    beta = state >> n
    return alpha | (beta << 32)


def hamiltonian_dense(n, na, nb, h, g):
    """Dense H over the (na, nb) sector; rows/cols ordered by ascending key."""
    states = sector_states(n, na, nb)
    keys = [to_key(s, n) for s in states]
    order = np.argsort(np.array(keys, dtype=np.uint64))
    states = [states[i] for i in order]
    index = {s: i for i, s in enumerate(states)}
    N = len(states)
    M = 2 * n
    Hd = np.zeros((N, N))
    spin = lambda k: k // n
    orb = lambda k: k % n
    terms = []
    for p in range(M):
        for q in range(M):
            if spin(p) == spin(q) and h[orb(p), orb(q)] != 0.0:
                terms.append((h[orb(p), orb(q)], [(True, p), (False, q)]))
    for p, q, r, s in itertools.product(range(M), repeat=4):
        if spin(p) != spin(q) or spin(r) != spin(s):
            continue
        v = g[orb(p), orb(q), orb(r), orb(s)]
        if v == 0.0:
            continue
        terms.append((0.5 * v, [(True, p), (True, r), (False, s), (False, q)]))
    for col, st in enumerate(states):
        for coef, ops in terms:
            sg, out = _apply(ops, st)
            if sg:
                Hd[index[out], col] += sg * coef
    keys_sorted = np.array([to_key(s, n) for s in states], dtype=np.uint64)
    return Hd, keys_sorted
