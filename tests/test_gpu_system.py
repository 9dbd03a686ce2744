"""Bit-exact parity of the determinant set, lookup, diagonal and excitation
lists (GPU through the C ABI) against the oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import hamiltonian, space
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def make_system(n, na, nb, seed=0, dets=None, flags=0):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets, flags=flags), h, g


@pytest.mark.parametrize("n,na,nb", [(8, 4, 4), (12, 6, 6), (5, 3, 2), (6, 0, 3), (7, 7, 1)])
def test_full_space_keys_bit_exact(n, na, nb):
    announce(f"keys n={n} na={na} nb={nb}")
    s, _, _ = make_system(n, na, nb)
    assert s.info.full_space == 1
    assert np.array_equal(s.keys(), space.full_space(n, na, nb))


def test_table1_space_sizes():
    """Every consistent row of Table 1 enumerates C(N_o/2, N_e/2)^2 sorted keys."""
    rows = [(2, 1), (6, 2), (7, 5), (11, 9), (8, 5), (10, 7), (10, 6), (14, 10), (15, 7)]
    for n, k in rows:
        announce(f"table1 n={n} k={k}")
        s, _, _ = make_system(n, k, k)
        assert s.ns == math.comb(n, k) ** 2
        if s.ns <= 2_000_000:
            keys = s.keys()
            assert np.all(keys[1:] > keys[:-1])
            if s.ns <= 50_000:
                assert np.array_equal(keys, space.full_space(n, k, k))
        s.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_lookup_full_and_hashed(flags):
    s, _, _ = make_system(8, 4, 4, flags=flags)
    keys = space.full_space(8, 4, 4)
    rows = s.lookup(keys)
    assert np.array_equal(rows, np.arange(keys.size, dtype=np.int32))
    absent = np.array([synth.key_of(0b111, 0b1111), synth.key_of(0b11110000, 0b111000001)], dtype=np.uint64)
    assert np.array_equal(s.lookup(absent), [-1, -1])


def test_selected_set_keys_and_lookup():
    n = 20
    keys = synth.cisd_like_selected_set(n, 10, 10, 1 << 14, seed=0)
    rng = np.random.default_rng(0)
    s, _, _ = make_system(n, 10, 10, dets=keys[rng.permutation(keys.size)])
    assert s.info.full_space == 0
    assert np.array_equal(s.keys(), keys)
    assert np.array_equal(s.lookup(keys), np.arange(keys.size, dtype=np.int32))
    others = synth.cisd_like_selected_set(n, 10, 10, 1 << 15, seed=1)
    missing = np.setdiff1d(others, keys)[:1000]
    assert np.all(s.lookup(missing) == -1)


@pytest.mark.parametrize("flags", [0, 1])
def test_diagonal_c1(c1_problem, flags):
    s, _, _ = make_system(8, 4, 4, flags=flags)
    ref = c1_problem["H"].diagonal()
    assert np.max(np.abs(s.diagonal() - ref)) <= 1e-12


@pytest.mark.parametrize("flags", [0, 1])
def test_excitation_lists_bit_exact_c1(c1_problem, flags):
    p = c1_problem
    s, h, g = make_system(8, 4, 4, flags=flags)
    for r in list(range(0, 4900, 97)) + [4899]:
        rows, signs, kinds, vals = s.excitations(r)
        orow, osig, okind, oval = hamiltonian.excitation_list(int(p["keys"][r]), p["keys"], 8, h, g)
        assert np.array_equal(rows, orow), r
        assert np.array_equal(signs, osig), r
        assert np.array_equal(kinds, okind), r
        assert np.max(np.abs(vals - oval)) <= 1e-12, r


@pytest.mark.parametrize("flags", [0, 1])
def test_excitation_lists_selected_set(flags):
    n = 10
    keys = synth.cisd_like_selected_set(n, 5, 5, 3000, seed=0)
    s, h, g = make_system(n, 5, 5, seed=2, dets=keys, flags=flags)
    for r in (0, 1, 77, 1500, 2999):
        rows, signs, kinds, vals = s.excitations(r)
        orow, osig, okind, oval = hamiltonian.excitation_list(int(keys[r]), keys, n, h, g)
        assert np.array_equal(rows, orow) and np.array_equal(signs, osig)
        assert np.array_equal(kinds, okind)
        assert np.max(np.abs(vals - oval)) <= 1e-12


def test_invalid_inputs_rejected():
    from paper_2601_01437_amd import IrlError, System
    h, g = synth.integrals(4, 0)
    keys = space.full_space(4, 2, 2)
    with pytest.raises(IrlError):
        System(4, 2, 2, h, g, dets=np.concatenate([keys, keys[:1]]))        # duplicate
    bad = keys.copy()
    bad[3] = np.uint64(0b111)
    with pytest.raises(IrlError):
        System(4, 2, 2, h, g, dets=bad)                                      # wrong popcount
    h2 = h.copy()
    h2[0, 1] += 1e-3
    with pytest.raises(IrlError):
        System(4, 2, 2, h2, g)                                               # asymmetric h
    with pytest.raises(IrlError):
        System(33, 2, 2, np.zeros((33, 33)), np.zeros((33,) * 4))            # n > 32
