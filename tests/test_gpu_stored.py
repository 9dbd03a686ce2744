"""Stored Hamiltonian rows (irl_system_store_hamiltonian) through the C ABI.

The number of stored elements is an integer fixed by the set: it must equal the
oracle's count of off-diagonal connections inside the set (bit-exact, through
the reported byte size).  Applies and whole steps that stream the stored rows
are compared with the oracle at the FP64 tolerances of the enumerating kernels
(||u - u_ref|| <= 1e-12 ||u_ref||; energies 1e-12 Ha)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import capply, space
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3s_step.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(n, na, nb, seed, dets, flags=0):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets, flags=flags), h, g


CASES = [  # (n, na, nb, selected count or None, seed, system flags)
    (8, 4, 4, None, 0, 2),          # full space, rank lookup
    (10, 5, 5, 3000, 2, 0),         # selected, beta-blocked lookup
    (10, 5, 5, 3000, 2, 1),         # selected, hashed lookup
    (20, 10, 10, 1 << 14, 0, 0),    # selected, 20 orbitals
    (24, 4, 3, 5000, 1, 0),         # selected, 24 orbitals
    (9, 5, 4, 1, 5, 0),             # one determinant: no off-diagonal elements
]


@pytest.mark.parametrize("n,na,nb,count,seed,flags", CASES)
def test_stored_rows_count_and_apply(n, na, nb, count, seed, flags):
    """L2-blocked layout (IRL_SYS_STORE_BLOCKS): the byte size is exact and the
    apply matches the oracle."""
    from paper_2601_01437_amd import IRL_SYS_STORE_BLOCKS
    announce(f"stored rows n={n} count={count} flags={flags}")
    keys = (space.full_space(n, na, nb) if count is None
            else synth.cisd_like_selected_set(n, na, nb, count, seed=seed))
    s, h, g = _system(n, na, nb, seed, None if count is None else keys, flags | IRL_SYS_STORE_BLOCKS)
    Href = capply.csr(n, h, g, keys)
    nnz_off = Href.nnz - keys.size        # the oracle emits the diagonal once per row
    stored, need = s.store_hamiltonian(1 << 40)
    assert stored and s.info.ham_kernel == 4
    nb = s.info.stored_col_blocks
    assert 1 <= nb <= 8 and nb == max(1, -(-keys.size // (1 << 18)))    # 2 MiB slices of w
    assert need == nb * (keys.size + 1) * 8 + 12 * nnz_off
    assert s.info.stored_elements == nnz_off
    w = np.random.default_rng(4).normal(size=keys.size)
    u = host(s.apply_hamiltonian(dev(w)))
    assert rel_err(u, Href @ w) <= 1e-12
    again, need2 = s.store_hamiltonian(0)   # already stored: no-op
    assert again and need2 == need


def _sliced_fixed_bytes(nsl, ns):
    """Bytes of the LDS-sliced layout besides the 10-byte slots: per slice and group
    of 64 rows the slot offset and length, per group lane its row, per slice the
    base, and the per-(slice, row) partial sums."""
    groups = -(-ns // 64)
    return groups * nsl * 6 + groups * 64 * nsl * 2 + nsl * 8 + nsl * ns * 8


SLICED_CASES = [  # (n, na, nb, selected count or None, seed, system flags)
    (10, 5, 5, None, 0, 2),         # full space (63,504 rows): 4 slices, the last ragged
    (10, 5, 5, 20000, 2, 0),        # selected, beta-blocked lookup: 2 slices
    (10, 5, 5, 16384, 2, 1),        # selected, hashed lookup: exactly one slice
    (9, 5, 4, 1, 5, 0),             # one determinant: no off-diagonal elements
]


@pytest.mark.parametrize("n,na,nb,count,seed,flags", SLICED_CASES)
def test_stored_rows_lds_slices_count_and_apply(n, na, nb, count, seed, flags):
    """LDS-sliced layout (slices of 2^14 target rows, the default; also requested
    with IRL_SYS_STORE_SLICED): the number of stored elements must
    equal the oracle's number of connections inside the set (the byte size then
    counts the padded slots of the 64-row groups);
    the apply matches the oracle to FP64 rounding, repeats bitwise, and a second
    system built from the same set stores the same rows (each segment in the
    fixed lane-major enumeration order)."""
    from paper_2601_01437_amd import IRL_SYS_STORE_SLICED
    announce(f"stored rows, LDS slices: n={n} count={count} flags={flags}")
    keys = (space.full_space(n, na, nb) if count is None
            else synth.cisd_like_selected_set(n, na, nb, count, seed=seed))
    fl = flags | IRL_SYS_STORE_SLICED
    s, h, g = _system(n, na, nb, seed, None if count is None else keys, fl)
    Href = capply.csr(n, h, g, np.sort(keys))
    nnz_off = Href.nnz - keys.size
    stored, need = s.store_hamiltonian(1 << 40)
    nsl = -(-keys.size // (1 << 14))
    assert stored and s.info.ham_kernel == 4 and s.info.stored_col_blocks == nsl
    assert s.info.stored_elements == nnz_off
    slots, rem = divmod(need - _sliced_fixed_bytes(nsl, keys.size), 10)
    assert rem == 0 and slots >= nnz_off
    w_h = np.random.default_rng(4).normal(size=keys.size)
    w = dev(w_h)
    u1 = host(s.apply_hamiltonian(w))
    assert rel_err(u1, Href @ w_h) <= 1e-12
    assert np.array_equal(host(s.apply_hamiltonian(w)), u1)
    s2, _, _ = _system(n, na, nb, seed, None if count is None else keys, fl)
    assert s2.store_hamiltonian(1 << 40) == (True, need)
    assert np.array_equal(host(s2.apply_hamiltonian(w)), u1)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("count", [300000, (1 << 18) + 1])
def test_stored_rows_lds_slices_large(count):
    """Sets above 2^18 determinants (the old L2-block range) in the LDS-sliced layout: 300,000
    rows give 19 slices (the last ragged), 2^18 + 1 rows 17 (the last holds one
    row).  The apply equals the enumerating kernel of the same system (pinned to
    the oracle) to FP64 rounding and the oracle's rows on a sample, and is
    bitwise reproducible across two systems built from the same set."""
    announce(f"stored rows: LDS slices, {count} rows")
    keys = synth.cisd_like_selected_set(14, 7, 7, count, seed=3)
    s, h, g = _system(14, 7, 7, 3, keys)
    w_h = np.random.default_rng(7).normal(size=keys.size)
    w = dev(w_h)
    u_enum = host(s.apply_hamiltonian(w))
    stored, need = s.store_hamiltonian(1 << 40)
    nsl = -(-keys.size // (1 << 14))
    assert stored and s.info.ham_kernel == 4 and s.info.stored_col_blocks == nsl
    slots, rem = divmod(need - _sliced_fixed_bytes(nsl, keys.size), 10)
    assert rem == 0 and slots >= s.info.stored_elements
    u1 = host(s.apply_hamiltonian(w))
    assert rel_err(u1, u_enum) <= 1e-12
    sk = np.sort(keys)
    rows = np.concatenate([np.random.default_rng(8).choice(keys.size, 400, replace=False),
                           [0, keys.size - 1, (1 << 14) - 1, 1 << 14]])
    ref = capply.apply(14, h, g, sk, w_h, rows=rows)
    assert np.max(np.abs(u1[rows] - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(host(s.apply_hamiltonian(w)), u1)
    s2, _, _ = _system(14, 7, 7, 3, keys)
    assert s2.store_hamiltonian(1 << 40) == (True, need)
    assert np.array_equal(host(s2.apply_hamiltonian(w)), u1)


def test_stored_rows_largest_l2_block_set():
    """2^18 determinants exactly (the largest set of one 2 MiB column block in the
    L2-blocked layout): one column block of 2^18 target rows; apply against the
    enumerating kernel."""
    from paper_2601_01437_amd import IRL_SYS_STORE_BLOCKS
    announce("stored rows: L2 column block at 2^18 rows")
    keys = synth.cisd_like_selected_set(14, 7, 7, 1 << 18, seed=3)
    s, _, _ = _system(14, 7, 7, 3, keys, IRL_SYS_STORE_BLOCKS)
    w = dev(np.random.default_rng(7).normal(size=keys.size))
    u_enum = host(s.apply_hamiltonian(w))
    stored, need = s.store_hamiltonian(1 << 40)
    assert stored and s.info.ham_kernel == 4 and s.info.stored_col_blocks == 1
    u1 = host(s.apply_hamiltonian(w))
    assert rel_err(u1, u_enum) <= 1e-12
    assert np.array_equal(host(s.apply_hamiltonian(w)), u1)


def test_stored_rows_over_budget_leaves_system_unchanged():
    announce("stored rows over budget")
    keys = synth.cisd_like_selected_set(10, 5, 5, 2000, seed=3)
    s, h, g = _system(10, 5, 5, 3, keys)
    kernel, nbytes = s.info.ham_kernel, s.info.device_bytes
    stored, need = s.store_hamiltonian(1000)
    assert not stored and need > 1000
    assert s.info.ham_kernel == kernel and s.info.device_bytes == nbytes
    w = np.random.default_rng(5).normal(size=keys.size)
    u = host(s.apply_hamiltonian(dev(w)))
    assert rel_err(u, capply.apply(10, h, g, keys, w)) <= 1e-12
    stored, need3 = s.store_hamiltonian(need)  # exactly the size needed fits
    assert stored and need3 == need
    assert s.info.device_bytes == nbytes + need
    u2 = host(s.apply_hamiltonian(dev(w)))
    assert rel_err(u2, u) <= 1e-13


def test_stored_rows_apply_is_bitwise_reproducible():
    keys = synth.cisd_like_selected_set(12, 6, 6, 20000, seed=1)
    s, _, _ = _system(12, 6, 6, 1, keys)
    assert s.store_hamiltonian(1 << 32)[0]
    w = dev(np.random.default_rng(6).normal(size=keys.size))
    u1 = host(s.apply_hamiltonian(w))
    u2 = host(s.apply_hamiltonian(w))
    assert np.array_equal(u1, u2)
    # two systems built from the same set store identical rows
    s2, _, _ = _system(12, 6, 6, 1, keys)
    assert s2.store_hamiltonian(1 << 32)[0]
    assert np.array_equal(host(s2.apply_hamiltonian(w)), u1)


def test_stored_rows_c3s_step_matches_oracle():
    """One FP64 step on the 2^14-determinant, 20-orbital selected set with V = 40,
    H = 256 (P = 10,536), the Hamiltonian streamed from stored rows."""
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c3s_step.json not generated")
    from paper_2601_01437_amd import IRL_FP64, IRL_WS_FP64, System
    announce("stored rows c3s step")
    G = json.load(open(GOLDEN))
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    s = System(w.n, w.na, w.nb, h, g, dets=w.dets())
    assert s.store_hamiltonian(1 << 34)[0]
    rc, r, dth, _ = s.step(dev(w.theta()), w.V, w.H, m=w.m, k_keep=w.k, precision=IRL_FP64,
                           ws_flags=IRL_WS_FP64)
    assert r.converged == 1
    assert abs(r.E_before - G["E"]) <= 1e-12
    assert abs(r.lambda_min - G["lambda_min"]) <= 1e-10 * max(abs(G["lambda_min"]), G["norm_Hp"])
    assert abs(r.E_after - G["E_after"]) <= 1e-12
    d = host(dth)
    assert abs(np.linalg.norm(d) - G["dtheta_norm"]) <= 1e-8 * G["dtheta_norm"]
