"""Batched solves (grouped kernels, lockstep members) through the C ABI: every
member's result equals the solo irl_step result on a system that uses the same
Hamiltonian kernel (per-determinant, string-product or stored rows), bit for
bit, and matches the oracle."""
import numpy as np
import pytest

import synth
from oracle import hamiltonian, space, step
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


# (n, na, nb, H, seed, selected-set size or None)
MEMBERS = [(6, 3, 3, 8, 1, None), (8, 4, 4, 16, 0, None), (7, 4, 3, 12, 2, None),
           (10, 5, 5, 6, 3, 2000), (9, 5, 4, 10, 4, 777), (8, 4, 4, 24, 5, 3000)]


def _build(flags_full, store=False, flags_sel=0):
    from paper_2601_01437_amd import System
    out = []
    for n, na, nb, H, seed, sel in MEMBERS:
        h, g = synth.integrals(n, seed)
        dets = None if sel is None else synth.cisd_like_selected_set(n, na, nb, sel, seed=seed)
        s = System(n, na, nb, h, g, dets=dets, flags=flags_full if dets is None else flags_sel)
        if store:
            assert s.store_hamiltonian(1 << 32)[0]
        theta = synth.nqs_theta(2 * n, H, seed, scale=0.2)
        out.append((s, theta, 2 * n, H, h, g, dets))
    return out


def _fields(r):
    return (r.E_before, r.lambda_min, r.E_after, r.c0, r.residual_est, r.residual_explicit,
            r.n_apply, r.n_restart, r.converged)


# (flags for full spaces, store rows, flags for selected sets)
KERNELS = {"pull": (2, False, 0), "default": (0, False, 0), "stored": (2, True, 0),
           "hash": (1, False, 1)}


@pytest.mark.parametrize("kernels", ["pull", "default", "stored", "hash"])
@pytest.mark.parametrize("m,k", [(20, 1), (12, 4)])
def test_batch_equals_solo_bitwise(m, k, kernels):
    """pull: per-determinant kernels (string ranks, beta blocks); default:
    string-product for full spaces and beta-blocked for selected sets; stored:
    every member's rows stored; hash: hashed lookup for every member."""
    from paper_2601_01437_amd import Batch
    announce(f"batch vs solo m={m} k={k} kernels={kernels}")
    flags_full, store, flags_sel = KERNELS[kernels]
    solo = _build(flags_full, store, flags_sel)
    ref = []
    for s, theta, V, H, *_ in solo:
        th = dev(theta)
        rc, r, dth, _ = s.step(th, V, H, m=m, k_keep=k)
        ref.append((rc, r, host(dth), host(th)))
    batch_sys = _build(flags_full, store, flags_sel)
    kinds = [x[0].info.ham_kernel for x in batch_sys]
    assert kinds == [x[0].info.ham_kernel for x in solo]
    if kernels == "stored":
        assert set(kinds) == {4}
    elif kernels == "default":
        assert 2 in kinds and 3 in kinds
    elif kernels == "hash":
        assert set(kinds) == {0}
    thetas = [dev(t) for _, t, *_ in batch_sys]
    bt = Batch([x[0] for x in batch_sys], thetas, [x[2] for x in batch_sys], [x[3] for x in batch_sys])
    res, status, dth = bt.step(m=m, k_keep=k, want_dtheta=True)
    for i, (rc, r, d_ref, th_ref) in enumerate(ref):
        assert status[i] == rc, i
        assert _fields(res[i]) == _fields(r), (i, _fields(res[i]), _fields(r))
        assert np.array_equal(host(dth[i]), d_ref), i
        assert np.array_equal(host(thetas[i]), th_ref), i
    bt.close()


@pytest.mark.parametrize("kernels", ["default", "stored"])
def test_batch_factored_equals_solo_bitwise(kernels):
    """Factored-Jacobian workspaces: each member's forward and backward products
    are its solo launches inside the lockstep batch, so every member equals its
    solo factored step bit for bit (string-product, beta-blocked and stored-row
    Hamiltonians)."""
    from paper_2601_01437_amd import IRL_WS_FACTORED, Batch
    announce(f"batch factored vs solo kernels={kernels}")
    flags_full, store, flags_sel = KERNELS[kernels]
    solo = _build(flags_full, store, flags_sel)
    ref = []
    for s, theta, V, H, *_ in solo:
        th = dev(theta)
        rc, r, dth, _ = s.step(th, V, H, m=20, k_keep=2, ws_flags=IRL_WS_FACTORED)
        ref.append((rc, r, host(dth), host(th)))
    batch_sys = _build(flags_full, store, flags_sel)
    thetas = [dev(t) for _, t, *_ in batch_sys]
    bt = Batch([x[0] for x in batch_sys], thetas, [x[2] for x in batch_sys], [x[3] for x in batch_sys],
               ws_flags=IRL_WS_FACTORED)
    for step_no in range(2):
        res, status, dth = bt.step(m=20, k_keep=2, want_dtheta=True)
        if step_no == 0:
            for i, (rc, r, d_ref, th_ref) in enumerate(ref):
                assert status[i] == rc, i
                assert _fields(res[i]) == _fields(r), (i, _fields(res[i]), _fields(r))
                assert np.array_equal(host(dth[i]), d_ref), i
                assert np.array_equal(host(thetas[i]), th_ref), i
    # a second step of each solo system matches the batch's second step
    for i, (s, theta, V, H, *_) in enumerate(solo):
        th = dev(ref[i][3])
        rc, r, _, _ = s.step(th, V, H, m=20, k_keep=2, ws_flags=IRL_WS_FACTORED)
        assert _fields(res[i]) == _fields(r), i
    bt.close()


def test_batch_factored_rejects_mixed_flags():
    from paper_2601_01437_amd import IRL_WS_FACTORED, IRL_WS_FP64, IrlError, Batch
    mem = _build(0)[:2]
    with pytest.raises(IrlError):
        Batch([x[0] for x in mem], [dev(t) for _, t, *_ in mem], [x[2] for x in mem], [x[3] for x in mem],
              ws_flags=IRL_WS_FACTORED | IRL_WS_FP64)


def test_batch_matches_oracle():
    from paper_2601_01437_amd import Batch
    announce("batch vs oracle")
    mem = _build(0)
    thetas = [dev(t) for _, t, *_ in mem]
    bt = Batch([x[0] for x in mem], thetas, [x[2] for x in mem], [x[3] for x in mem])
    res, status, _ = bt.step(m=20, k_keep=2)
    for i, (s, theta, V, H, h, g, dets) in enumerate(mem):
        n = s.n
        keys = space.full_space(n, s.na, s.nb) if dets is None else dets
        Hm = hamiltonian.build(keys, n, h, g)
        o, th_new, E_after = step.lm_step(keys, n, V, H, theta, Hm)
        normH = np.linalg.norm(o.Hp, 2)
        assert res[i].converged == 1
        assert abs(res[i].E_before - o.E) <= 1e-12
        assert abs(res[i].lambda_min - o.lam) <= 1e-10 * max(abs(o.lam), normH)
        assert abs(res[i].E_after - E_after) <= 1e-12
    bt.close()


def test_batch_three_steps_equal_solo():
    from paper_2601_01437_amd import IRL_SYS_FORCE_PULL, Batch
    announce("batch 3 steps")
    solo = _build(IRL_SYS_FORCE_PULL)
    ref = []
    for s, theta, V, H, *_ in solo:
        th = dev(theta)
        Es = []
        for _ in range(3):
            rc, r, _, _ = s.step(th, V, H, m=16, k_keep=2)
            Es.append((r.E_before, r.E_after, r.lambda_min))
        ref.append(Es)
    mem = _build(IRL_SYS_FORCE_PULL)
    thetas = [dev(t) for _, t, *_ in mem]
    bt = Batch([x[0] for x in mem], thetas, [x[2] for x in mem], [x[3] for x in mem])
    got = [[] for _ in mem]
    for _ in range(3):
        res, status, _ = bt.step(m=16, k_keep=2)
        for i, r in enumerate(res):
            got[i].append((r.E_before, r.E_after, r.lambda_min))
    assert got == ref
    bt.close()


def test_batch_fp32_only_equals_solo_bitwise():
    """FP32 copy of D~ only (FP32 products, gradient recomputed from theta in
    FP64): batched members equal their solo steps bit for bit."""
    from paper_2601_01437_amd import IRL_FP32, IRL_WS_FP32, Batch
    announce("batch fp32-only vs solo")
    solo = _build(0)
    ref = []
    for s, theta, V, H, *_ in solo:
        th = dev(theta)
        rc, r, dth, _ = s.step(th, V, H, m=20, k_keep=1, precision=IRL_FP32, ws_flags=IRL_WS_FP32)
        ref.append((rc, r, host(dth)))
    mem = _build(0)
    thetas = [dev(t) for _, t, *_ in mem]
    bt = Batch([x[0] for x in mem], thetas, [x[2] for x in mem], [x[3] for x in mem], ws_flags=IRL_WS_FP32)
    res, status, dth = bt.step(m=20, k_keep=1, precision=IRL_FP32, want_dtheta=True)
    for i, (rc, r, d_ref) in enumerate(ref):
        assert status[i] == rc, i
        assert _fields(res[i]) == _fields(r), (i, _fields(res[i]), _fields(r))
        assert np.array_equal(host(dth[i]), d_ref), i
    bt.close()
