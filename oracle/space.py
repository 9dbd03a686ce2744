"""Determinant space with fixed (N_alpha, N_beta).

Methods, "Wave Function Ansatz": the wavefunction is expanded over occupation
number vectors n_i in {0, 1} of M spin-orbitals.  Methods, "Autoregressive
Modeling and Physical Constraints" (Eq. constraint): only configurations with
the prescribed spin-up and spin-down electron counts are valid.

Key layout: alpha orbital p is bit p, beta orbital p is bit 32 + p of a
uint64.  Sets are ordered by ascending key (beta string major).

Pins: counts C(n, Na) C(n, Nb) and the PVC column of Table 1
(tests/test_oracle_space.py).
"""
from __future__ import annotations

import itertools

import numpy as np

ALPHA_MASK = (1 << 32) - 1


def strings(n: int, ne: int) -> list[int]:
    """All bit strings with ``ne`` of the low ``n`` bits set, ascending."""
    out = [sum(1 << p for p in occ) for occ in itertools.combinations(range(n), ne)]
    return sorted(out)


def full_space(n: int, na: int, nb: int) -> np.ndarray:
    """Every determinant with ``na`` alpha and ``nb`` beta electrons in ``n``
    spatial orbitals, as ascending uint64 keys."""
    A = strings(n, na)
    B = strings(n, nb)
    keys = [a | (b << 32) for b in B for a in A]   # beta-major == ascending key
    return np.array(keys, dtype=np.uint64)


def split(key: int) -> tuple[int, int]:
    """(alpha bits, beta bits) of a key."""
    key = int(key)
    return key & ALPHA_MASK, key >> 32


def validate(n: int, na: int, nb: int, keys: np.ndarray) -> np.ndarray:
    """Sort, check popcounts and range, and reject duplicates.  Returns the
    sorted key array."""
    keys = np.sort(np.asarray(keys, dtype=np.uint64))
    if keys.size and np.any(keys[1:] == keys[:-1]):
        raise ValueError("duplicate determinant keys")
    for k in keys.tolist():
        a, b = split(k)
        if a >> n or b >> n:
            raise ValueError("orbital index out of range")
        if bin(a).count("1") != na or bin(b).count("1") != nb:
            raise ValueError("wrong electron count")
    return keys
