"""irl_lookup_noalloc (fixed device scratch, no allocation) against
irl_debug_lookup through the C ABI: bit-identical rows on two calls in a row,
the second with fewer keys, on a hashed selected set and on a full space
(string ranks), including keys absent from the set; sizes past the fixed
maximum are rejected."""
import numpy as np
import pytest

import synth
from oracle import space
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _queries(keys, count, n, seed):
    rng = np.random.default_rng(seed)
    present = keys[rng.integers(0, keys.size, count // 2)]
    # absent keys: random strings of the right popcounts (some collide with the set)
    absent = np.array([synth.key_of(int(a), int(b)) for a, b in zip(
        [sum(1 << int(i) for i in rng.choice(n, n // 2, replace=False)) for _ in range(count - count // 2)],
        [sum(1 << int(i) for i in rng.choice(n, n // 2, replace=False)) for _ in range(count - count // 2)])],
        dtype=np.uint64)
    q = np.concatenate([present, absent, np.array([~np.uint64(0), np.uint64(0)], dtype=np.uint64)])
    return q[rng.permutation(q.size)]


@pytest.mark.parametrize("kind", ["selected", "full"])
def test_lookup_noalloc_matches_lookup(kind):
    from paper_2601_01437_amd import System
    from paper_2601_01437_amd import binding as B
    announce(f"lookup noalloc {kind}")
    n = 12
    h, g = synth.integrals(n, 0)
    if kind == "selected":
        keys = synth.cisd_like_selected_set(n, 6, 6, 50_000, seed=1)
        s = System(n, 6, 6, h, g, dets=keys)
    else:
        keys = space.full_space(n, 6, 6)
        s = System(n, 6, 6, h, g)
    sorted_keys = np.sort(keys)
    for count, seed in ((200_000, 3), (1_000, 4)):
        q = _queries(sorted_keys, count, n, seed)
        got = B.irl_lookup_noalloc(s.handle, q)
        ref = B.irl_debug_lookup(s.handle, q)
        assert np.array_equal(got, ref)
        hit = got >= 0
        assert np.array_equal(sorted_keys[got[hit]], q[hit])
        assert not np.isin(q[~hit], sorted_keys).any()
    with pytest.raises(B.IrlError):
        B.irl_lookup_noalloc(s.handle, np.zeros((1 << 18) + 1, dtype=np.uint64))
    assert B.irl_lookup_noalloc(s.handle, np.zeros(0, dtype=np.uint64)).size == 0
    s.close()
