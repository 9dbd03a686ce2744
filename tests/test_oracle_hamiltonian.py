"""Pins for the oracle's Slater-Condon Hamiltonian.

* brute-force second quantisation (tests/fock_bruteforce.py) fixes every element,
  sign and sparsity pattern for small n;
* the one-body special case g = 0 has the closed-form ground state
  sum of the lowest N_alpha plus lowest N_beta eigenvalues of h;
* Hermiticity;
* the C apply equals the Python rows;
* planted mistakes in the oracle (wrong sign rule, dropped exchange term) are
  caught by the brute-force pin.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import capply, hamiltonian, space
from tests.fock_bruteforce import hamiltonian_dense


@pytest.mark.parametrize("n,na,nb,seed", [(4, 2, 2, 3), (5, 3, 2, 4), (5, 1, 3, 5), (6, 2, 2, 6)])
def test_slater_condon_equals_bruteforce(n, na, nb, seed):
    h, g = synth.integrals(n, seed)
    Hb, kb = hamiltonian_dense(n, na, nb, h, g)
    keys = space.full_space(n, na, nb)
    assert np.array_equal(keys, kb)
    Hs = hamiltonian.build(keys, n, h, g).toarray()
    # pattern and signs bit-exact (random integrals: no accidental zeros)
    assert np.array_equal(np.abs(Hb) > 1e-13, np.abs(Hs) > 1e-13)
    nz = np.abs(Hb) > 1e-13
    assert np.array_equal(np.sign(Hb[nz]), np.sign(Hs[nz]))
    assert np.max(np.abs(Hb - Hs)) <= 1e-12 * max(1.0, np.abs(Hb).max())


def test_c_apply_equals_bruteforce_small():
    n, na, nb = 5, 2, 3
    h, g = synth.integrals(n, 11)
    Hb, keys = hamiltonian_dense(n, na, nb, h, g)
    w = np.random.default_rng(0).normal(size=keys.size)
    u = capply.apply(n, h, g, keys, w)
    assert np.max(np.abs(u - Hb @ w)) <= 1e-12 * np.abs(Hb @ w).max()


def test_hermitian_c1(c1_problem):
    Hm = c1_problem["H"]
    assert abs(Hm - Hm.T).max() == 0.0
    # connections per row of the full space: 1 + singles + doubles
    n, na, nb = 8, 4, 4
    per_row = 1 + na * (n - na) + nb * (n - nb) + 36 + 36 + 16 * 16
    assert Hm.nnz <= Hm.shape[0] * per_row


def test_one_body_closed_form():
    n, na, nb = 6, 3, 2
    h, _ = synth.integrals(n, 7)
    g = np.zeros((n, n, n, n))
    Hm = hamiltonian.build(space.full_space(n, na, nb), n, h, g).toarray()
    e_exact = np.linalg.eigvalsh(Hm)[0]
    eh = np.linalg.eigvalsh(h)
    assert abs(e_exact - (eh[:na].sum() + eh[:nb].sum())) < 1e-11


def test_c_apply_equals_python_c1_and_selected(c1_problem):
    p = c1_problem
    w = np.random.default_rng(1).normal(size=p["keys"].size)
    u = capply.apply(p["w"].n, p["h"], p["g"], p["keys"], w)
    assert np.max(np.abs(u - p["H"] @ w)) <= 1e-13 * np.abs(u).max()
    # projected Hamiltonian on a selected set (excitations that leave are dropped)
    n = 10
    keys = synth.cisd_like_selected_set(n, 5, 5, 3000, seed=0)
    h, g = synth.integrals(n, 2)
    Hs = hamiltonian.build(keys, n, h, g)
    w = np.random.default_rng(2).normal(size=keys.size)
    u = capply.apply(n, h, g, keys, w)
    assert np.max(np.abs(u - Hs @ w)) <= 1e-13 * np.abs(u).max()
    rows = np.array([0, 7, 2999, 1500])
    assert np.allclose(capply.apply(n, h, g, keys, w, rows=rows), (Hs @ w)[rows],
                       rtol=0, atol=1e-13 * np.abs(u).max())


def test_excitation_list_consistent(c1_problem):
    p = c1_problem
    keys, Hm = p["keys"], p["H"]
    for r in (0, 17, 2450, 4899):
        rows, signs, kinds, vals = hamiltonian.excitation_list(int(keys[r]), keys, 8, p["h"], p["g"])
        assert np.all(np.diff(rows) > 0)
        row = Hm.getrow(r).toarray().ravel()
        off = np.nonzero(row)[0]
        off = off[off != r]
        assert np.array_equal(rows, off)
        assert np.allclose(vals, row[rows], rtol=0, atol=1e-14)
        assert set(kinds.tolist()) <= {1, 2, 3, 4, 5}
        assert np.count_nonzero(kinds == 1) == 16 and np.count_nonzero(kinds == 5) == 256


def _assert_bruteforce_fails(monkeypatch, attr, fake):
    monkeypatch.setattr(hamiltonian, attr, fake)
    n, na, nb = 4, 2, 2
    h, g = synth.integrals(n, 3)
    Hb, _ = hamiltonian_dense(n, na, nb, h, g)
    Hs = hamiltonian.build(space.full_space(n, na, nb), n, h, g).toarray()
    assert np.max(np.abs(Hb - Hs)) > 1e-6


def test_planted_sign_mistake_is_caught(monkeypatch):
    _assert_bruteforce_fails(monkeypatch, "_between_parity", lambda bits, i, a: 1)


def test_planted_same_spin_double_sign_is_caught(monkeypatch):
    orig = hamiltonian.row_elements

    def flipped(key, n, h, g):
        alpha, beta = space.split(key)
        out = []
        for tgt, v in orig(key, n, h, g):
            ta, tb = space.split(tgt)
            if bin(ta ^ alpha).count("1") == 4:     # alpha-alpha double
                v = -v
            out.append((tgt, v))
        return out

    _assert_bruteforce_fails(monkeypatch, "row_elements", flipped)


def test_planted_dropped_diagonal_exchange_is_caught(monkeypatch):
    def coulomb_only(alpha, beta, n, h, g):
        occ = [p for p in range(n) if alpha >> p & 1] + [n + p for p in range(n) if beta >> p & 1]
        e = sum(h[q % n][q % n] for q in occ)
        for x in occ:
            for y in occ:
                e += 0.5 * g[x % n][x % n][y % n][y % n]
        return e

    _assert_bruteforce_fails(monkeypatch, "diagonal_element", coulomb_only)


def test_dense_ed_small_c1_like():
    """Exact diagonalisation through the oracle Hamiltonian matches scipy's
    sparse eigensolver on the same matrix (ground-state energy)."""
    n, na, nb = 6, 3, 3
    h, g = synth.integrals(n, 0)
    Hm = hamiltonian.build(space.full_space(n, na, nb), n, h, g)
    e_dense = sla.eigh(Hm.toarray(), eigvals_only=True)[0]
    import scipy.sparse.linalg as spla
    e_sp = spla.eigsh(Hm, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(e_dense - e_sp) < 1e-10
