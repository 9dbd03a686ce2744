"""Second-quantised electronic Hamiltonian on a determinant set (Slater-Condon).

Methods, "Wave Function Ansatz", Hamiltonian equation: one-body integrals h_pq
and two-body integrals g_pqrs over spin-orbitals.  Reading adopted here (the
paper does not fix the index convention): g is the chemists' integral (pq|rs)
over spatial orbitals and

    H = sum_{pq,s} h_pq a+_{p s} a_{q s}
        + 1/2 sum_{pqrs, s t} (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s}.

Determinant |D> = a+_{i1} a+_{i2} ... |0> with spin-orbitals in ascending
order, alpha orbitals before beta orbitals.  Applying a+_a a_i to D gives
(-1)^(number of occupied spin-orbitals strictly between i and a) times the
canonical determinant.  Matrix elements <D'|H|D> (textbook Slater-Condon rules,
spin-orbital integrals [pq|rs] = (pq|rs) delta(spin p, spin q) delta(spin r, spin s)):

* D' = D:      sum_i h_ii + 1/2 sum_{i,j} ([ii|jj] - [ij|ji])
* single i->a: sign * (h_ia + sum_{j in D} ([ia|jj] - [ij|ja]))
* double i->a then j->b: sign_1 * sign_2 * ([ia|jb] - [ib|ja]), each sign taken
  on the determinant it acts on.

Excitations that leave the determinant set are dropped (Hamiltonian projected
onto the set).

Pins: brute-force second quantisation on the Fock space (independent operator
algebra), one-body closed form, Hermiticity (tests/test_oracle_hamiltonian.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .space import split


def _occ(bits: int, n: int) -> list[int]:
    return [p for p in range(n) if (bits >> p) & 1]


def _between_parity(bits: int, i: int, a: int) -> int:
    """+1 or -1: parity of occupied bits strictly between positions i and a."""
    lo, hi = (i, a) if i < a else (a, i)
    mask = ((1 << hi) - 1) & ~((1 << (lo + 1)) - 1)
    return -1 if bin(bits & mask).count("1") & 1 else 1


def _excite(bits: int, i: int, a: int) -> tuple[int, int]:
    """a+_a a_i on one spin string: (sign, new bits)."""
    s = _between_parity(bits, i, a)
    return s, (bits & ~(1 << i)) | (1 << a)


def diagonal_element(alpha: int, beta: int, n: int, h, g) -> float:
    """<D|H|D>.  ``h`` and ``g`` are nested lists (fast scalar indexing)."""
    oa, ob = _occ(alpha, n), _occ(beta, n)
    e = 0.0
    for i in oa + ob:
        e += h[i][i]
    for occ in (oa, ob):                       # same spin: Coulomb - exchange
        for i in occ:
            for j in occ:
                e += 0.5 * (g[i][i][j][j] - g[i][j][j][i])
    for i in oa:                               # opposite spin: Coulomb only
        for j in ob:
            e += g[i][i][j][j]
    return e


def row_elements(key: int, n: int, h, g) -> list[tuple[int, float]]:
    """All (target key, <target|H|D>) for determinant ``key``, including the
    diagonal, over the full space reachable by one- and two-electron moves.
    ``h`` and ``g`` are nested lists."""
    alpha, beta = split(key)
    oa, ob = _occ(alpha, n), _occ(beta, n)
    va = [p for p in range(n) if not (alpha >> p) & 1]
    vb = [p for p in range(n) if not (beta >> p) & 1]
    out = [(int(key), diagonal_element(alpha, beta, n, h, g))]

    # singles
    for spin in (0, 1):
        same, other = (oa, ob) if spin == 0 else (ob, oa)
        virt = va if spin == 0 else vb
        bits = alpha if spin == 0 else beta
        for i in same:
            for a in virt:
                s, nb_ = _excite(bits, i, a)
                v = h[i][a]
                for j in same:
                    v += g[i][a][j][j] - g[i][j][j][a]
                for j in other:
                    v += g[i][a][j][j]
                tgt = (nb_ | (beta << 32)) if spin == 0 else (alpha | (nb_ << 32))
                out.append((tgt, s * v))

    # same-spin doubles: i < j -> a < b, i->a first then j->b
    for spin in (0, 1):
        occ = oa if spin == 0 else ob
        virt = va if spin == 0 else vb
        bits = alpha if spin == 0 else beta
        for x in range(len(occ)):
            for y in range(x + 1, len(occ)):
                i, j = occ[x], occ[y]
                for u in range(len(virt)):
                    for w in range(u + 1, len(virt)):
                        a, b = virt[u], virt[w]
                        s1, b1 = _excite(bits, i, a)
                        s2, b2 = _excite(b1, j, b)
                        v = s1 * s2 * (g[i][a][j][b] - g[i][b][j][a])
                        tgt = (b2 | (beta << 32)) if spin == 0 else (alpha | (b2 << 32))
                        out.append((tgt, v))

    # opposite-spin doubles: alpha i->a, beta j->b
    for i in oa:
        for a in va:
            s1, a1 = _excite(alpha, i, a)
            for j in ob:
                for b in vb:
                    s2, b1 = _excite(beta, j, b)
                    out.append((a1 | (b1 << 32), s1 * s2 * g[i][a][j][b]))
    return out


def build(keys: np.ndarray, n: int, h: np.ndarray, g: np.ndarray,
          rows: np.ndarray | None = None) -> sp.csr_matrix:
    """Hamiltonian projected on the set ``keys`` as CSR (N_s x N_s), or only the
    listed ``rows`` (len(rows) x N_s) when given.  Columns follow ``keys``."""
    keys = np.asarray(keys, dtype=np.uint64)
    index = {int(k): r for r, k in enumerate(keys.tolist())}
    hl, gl = h.tolist(), g.tolist()
    sel = range(keys.size) if rows is None else [int(r) for r in rows]
    indptr, indices, data = [0], [], []
    for r in sel:
        entries = {}
        for tgt, v in row_elements(int(keys[r]), n, hl, gl):
            c = index.get(tgt)
            if c is not None:
                entries[c] = entries.get(c, 0.0) + v
        cols = sorted(entries)
        indices.extend(cols)
        data.extend(entries[c] for c in cols)
        indptr.append(len(indices))
    shape = (len(indptr) - 1, keys.size)
    return sp.csr_matrix((np.array(data, dtype=np.float64),
                          np.array(indices, dtype=np.int64),
                          np.array(indptr, dtype=np.int64)), shape=shape)


def excitation_list(key: int, keys: np.ndarray, n: int, h: np.ndarray, g: np.ndarray):
    """Off-diagonal connections of one determinant inside the set, sorted by
    target row: (rows int32, signs int8, kinds uint8, values float64).

    kind: 1 alpha single, 2 beta single, 3 alpha-alpha double, 4 beta-beta
    double, 5 alpha-beta double.  ``sign`` is the fermionic sign of the
    excitation operator string (values already include it)."""
    keys = np.asarray(keys, dtype=np.uint64)
    index = {int(k): r for r, k in enumerate(keys.tolist())}
    alpha, beta = split(key)
    hl, gl = h.tolist(), g.tolist()
    out = []
    elems = row_elements(int(key), n, hl, gl)[1:]
    # recover kind and sign from the bit difference (independent of the loop above)
    for tgt, v in elems:
        r = index.get(tgt)
        if r is None:
            continue
        ta, tb = split(tgt)
        da = bin(ta ^ alpha).count("1") // 2
        db = bin(tb ^ beta).count("1") // 2
        kind = {(1, 0): 1, (0, 1): 2, (2, 0): 3, (0, 2): 4, (1, 1): 5}[(da, db)]
        out.append((r, _string_sign(alpha, beta, ta, tb, n), kind, v))
    out.sort()
    rows = np.array([o[0] for o in out], dtype=np.int32)
    signs = np.array([o[1] for o in out], dtype=np.int8)
    kinds = np.array([o[2] for o in out], dtype=np.uint8)
    vals = np.array([o[3] for o in out], dtype=np.float64)
    return rows, signs, kinds, vals


def _string_sign(alpha, beta, ta, tb, n) -> int:
    """Sign of the excitation taking (alpha, beta) to (ta, tb): holes and
    particles paired in ascending order, applied alpha first, lower hole first."""
    s = 1
    for bits, tbits, spin in ((alpha, ta, 0), (beta, tb, 1)):
        holes = [p for p in range(n) if (bits >> p) & 1 and not (tbits >> p) & 1]
        parts = [p for p in range(n) if (tbits >> p) & 1 and not (bits >> p) & 1]
        cur = bits
        for i, a in zip(holes, parts):
            si, cur = _excite(cur, i, a)
            s *= si
    return s
