"""Pins for the oracle's determinant space (fixed N_alpha, N_beta).

Counts are fixed by combinatorics and by the PVC column of Table 1."""
import math
import os

import numpy as np
import pytest

from oracle import space

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_pvc.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        mol, no, ne, pvc = line.split()
        rows.append((mol, int(no), int(ne), float(pvc)))
    return rows


@pytest.mark.parametrize("n,na,nb", [(8, 4, 4), (12, 6, 6), (5, 3, 2), (6, 1, 4), (4, 0, 2)])
def test_full_space_count_order_popcount(n, na, nb):
    keys = space.full_space(n, na, nb)
    assert keys.size == math.comb(n, na) * math.comb(n, nb)
    assert np.all(keys[1:] > keys[:-1])                   # strictly ascending
    for k in keys[:: max(1, keys.size // 500)].tolist():
        a, b = space.split(k)
        assert bin(a).count("1") == na and bin(b).count("1") == nb
        assert a >> n == 0 and b >> n == 0


def test_c1_c2_counts():
    assert space.full_space(8, 4, 4).size == 4900
    assert len(space.strings(12, 6)) ** 2 == 853776


def test_table1_pvc_counts():
    """Table 1: PVC = C(N_o/2, N_e/2)^2 for every row but CH4 (printed values are
    rounded to two significant digits)."""
    checked = 0
    for mol, no, ne, pvc in _table1():
        if mol == "CH4":
            continue
        n, ns = no // 2, ne // 2
        count = len(space.strings(n, ns)) ** 2     # enumerated alpha x beta strings
        if count < 2_000_000:
            assert space.full_space(n, ns, ns).size == count
        assert count == math.comb(n, ns) ** 2
        # printed to two significant digits (H2 exactly): within half a unit
        half_unit = 0.5 * 10 ** (math.floor(math.log10(pvc)) - 1) if pvc >= 10 else 0.0
        assert abs(count - pvc) <= half_unit, mol
        checked += 1
    assert checked == 9


def test_validate_rejects_bad_sets():
    good = space.full_space(4, 2, 1)
    assert np.array_equal(space.validate(4, 2, 1, good[::-1]), good)
    with pytest.raises(ValueError):
        space.validate(4, 2, 1, np.concatenate([good, good[:1]]))
    bad = good.copy()
    bad[0] = np.uint64(0b111)
    with pytest.raises(ValueError):
        space.validate(4, 2, 1, bad)
