"""Pins for the oracle's row-by-row Slater-Condon CSR (``capply.csr``, the C
function ``oracle_sc_row``), the reference matrix of several GPU tests and of
the stored expected values under tests/golden/.

* every element, sign and the sparsity pattern equal the brute-force
  second-quantised Hamiltonian (tests/fock_bruteforce.py) on small sectors,
  including unequal electron counts;
* the matrix equals ``hamiltonian.build`` (the Python Slater-Condon rows) on the
  c1 full space and on a CISD-like selected set, where excitations leaving the
  set are dropped (Methods, "Wave Function Ansatz", Hamiltonian equation);
* ``csr @ w`` equals the matrix-free ``capply.apply``;
* mistakes planted in a copy of the C source (a dropped sign of each excitation
  kind, a dropped exchange term of the singles) are caught by the brute-force
  comparison.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import capply, hamiltonian, space
from tests.fock_bruteforce import hamiltonian_dense

SECTORS = [(4, 2, 2, 3), (5, 3, 2, 4), (5, 1, 3, 5), (6, 2, 2, 6), (6, 3, 3, 8)]


def _bruteforce_mismatch(n, na, nb, seed):
    """Largest |H_csr - H_bruteforce| over the sector, plus pattern and sign checks."""
    h, g = synth.integrals(n, seed)
    Hb, kb = hamiltonian_dense(n, na, nb, h, g)
    keys = space.full_space(n, na, nb)
    assert np.array_equal(keys, kb)
    Hc = capply.csr(n, h, g, keys).toarray()
    nzb = np.abs(Hb) > 1e-13
    nzc = np.abs(Hc) > 1e-13
    pattern_ok = np.array_equal(nzb, nzc)
    signs_ok = pattern_ok and np.array_equal(np.sign(Hb[nzb]), np.sign(Hc[nzb]))
    return float(np.max(np.abs(Hb - Hc))), pattern_ok, signs_ok, float(np.abs(Hb).max())


@pytest.mark.parametrize("n,na,nb,seed", SECTORS)
def test_csr_equals_bruteforce(n, na, nb, seed):
    err, pattern_ok, signs_ok, scale = _bruteforce_mismatch(n, na, nb, seed)
    assert pattern_ok and signs_ok
    assert err <= 1e-12 * max(1.0, scale)


def test_csr_rows_have_no_duplicates_and_diagonal_first():
    n, na, nb = 6, 3, 2
    h, g = synth.integrals(n, 9)
    keys = space.full_space(n, na, nb)
    Hc = capply.csr(n, h, g, keys)
    for r in range(keys.size):
        cols = Hc.indices[Hc.indptr[r]:Hc.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
        assert r in cols


def test_csr_equals_python_rows_c1(c1_problem):
    p = c1_problem
    w = p["w"]
    Hc = capply.csr(w.n, p["h"], p["g"], p["keys"])
    Hp = p["H"].tocsr()
    Hp.sort_indices()
    assert np.array_equal(Hc.indptr, Hp.indptr)
    assert np.array_equal(Hc.indices, Hp.indices)
    assert np.max(np.abs(Hc.data - Hp.data)) <= 1e-13 * np.abs(Hp.data).max()
    x = np.random.default_rng(4).normal(size=p["keys"].size)
    u = capply.apply(w.n, p["h"], p["g"], p["keys"], x)
    assert np.max(np.abs(Hc @ x - u)) <= 1e-13 * np.abs(u).max()


@pytest.mark.parametrize("n,na,nb,count,seed", [(10, 5, 5, 3000, 0), (12, 4, 3, 2500, 5)])
def test_csr_equals_python_rows_selected(n, na, nb, count, seed):
    keys = synth.cisd_like_selected_set(n, na, nb, count, seed=seed)
    h, g = synth.integrals(n, seed + 1)
    Hc = capply.csr(n, h, g, keys)
    Hp = hamiltonian.build(keys, n, h, g).tocsr()
    Hp.sort_indices()
    assert np.array_equal(Hc.indptr, Hp.indptr)
    assert np.array_equal(Hc.indices, Hp.indices)
    assert np.max(np.abs(Hc.data - Hp.data)) <= 1e-13 * np.abs(Hp.data).max()
    assert abs(Hc - Hc.T).max() <= 1e-14 * np.abs(Hc.data).max()
    x = np.random.default_rng(seed).normal(size=keys.size)
    u = capply.apply(n, h, g, keys, x)
    assert np.max(np.abs(Hc @ x - u)) <= 1e-13 * np.abs(u).max()


# ---- planted mistakes: a modified copy of the C file must fail the pin ----

PLANTS = {
    # same-spin double: drop the second annihilation/creation sign
    "same_spin_sign": ("if (r >= 0) EMIT(r, s1 * s2 * (G(i, a, j, b) - G(i, b, j, a)));",
                       "if (r >= 0) EMIT(r, s1 * (G(i, a, j, b) - G(i, b, j, a)));"),
    # opposite-spin double: drop the beta string's sign
    "opposite_spin_sign": ("if (r >= 0) EMIT(r, s1 * s2 * G(i, a, j, b));",
                           "if (r >= 0) EMIT(r, s1 * G(i, a, j, b));"),
    # single: drop the exchange with the same-spin occupied orbitals
    "single_exchange": ("if (r < 0) continue;\n"
                        "                double v = h[i * n + a];\n"
                        "                for (int y = 0; y < nos; ++y) v += G(i, a, os[y], os[y]) - G(i, os[y], os[y], a);",
                        "if (r < 0) continue;\n"
                        "                double v = h[i * n + a];\n"
                        "                for (int y = 0; y < nos; ++y) v += G(i, a, os[y], os[y]);"),
    # single: a sign that ignores the occupied orbitals in between
    "single_sign": ("EMIT(r, parity_between(bits, i, a) * v);", "EMIT(r, v);"),
}


def _planted_library(tmp_path, name):
    src = open(os.path.join(os.path.dirname(capply.__file__), "sc_apply.c")).read()
    old, new = PLANTS[name]
    assert src.count(old) == 1, f"plant {name}: anchor text not found once"
    path = tmp_path / f"sc_{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"libsc_{name}.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", str(so), str(path)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_sc_apply.restype = None
    lib.oracle_sc_apply.argtypes = [
        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    return lib


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_row_mistake_is_caught(tmp_path, monkeypatch, name):
    lib = _planted_library(tmp_path, name)
    monkeypatch.setattr(capply, "_lib", lib)
    caught = False
    for n, na, nb, seed in SECTORS:
        err, pattern_ok, signs_ok, scale = _bruteforce_mismatch(n, na, nb, seed)
        if not (pattern_ok and signs_ok) or err > 1e-6 * max(1.0, scale):
            caught = True
            break
    assert caught, f"planted mistake {name} passed the brute-force pin"
