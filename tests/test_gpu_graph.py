"""Captured Lanczos cycles (IRL_STEP_GRAPH) through the C ABI: every step with
graph replay equals the same step with launched kernels, bit for bit (eigenvalue,
energies, residuals, apply and restart counts, update), over several consecutive
steps (each replays the cached graphs with eager work and synchronisations in
between), for the Hamiltonian kernels (string product with the dense same-spin
DGEMMs, beta-blocked pull, stored rows), dense and factored Jacobians, modes A,
P and C, the FP32 operator with its FP64 polish (two cached precisions), the
sampled estimators, and after the workspace changes (the graphs are rebuilt)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(n, na, nb, seed, dets=None, flags=0, store=False):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    s = System(n, na, nb, h, g, dets=dets, flags=flags)
    if store:
        assert s.store_hamiltonian(1 << 32)[0]
    return s


def _fields(r):
    # repr: exact for floats and equal for NaN (mode P reports no energy after)
    return tuple(repr(x) for x in (r.E_before, r.lambda_min, r.E_after, r.c0, r.residual_est,
                                   r.residual_explicit, r.n_apply, r.n_restart, r.converged, r.norm_T))


def _last_error(s):
    from paper_2601_01437_amd import binding as B
    msg = B._lib.irl_last_error(s.handle)
    return msg.decode() if msg else ""


def _run(s, theta, V, H, steps, graph, **kw):
    from paper_2601_01437_amd import IRL_STEP_GRAPH
    flags = kw.pop("flags", 0) | (IRL_STEP_GRAPH if graph else 0)
    th = dev(theta)
    out = []
    for _ in range(steps):
        rc, r, dth, _ = s.step(th, V, H, flags=flags, **kw)
        # the replay is really used (not the launched fallback), and only when asked for
        assert (r.n_graph_cycles > 0) == graph, (r.n_graph_cycles, _last_error(s))
        out.append((rc, _fields(r), None if dth is None else host(dth).tobytes(), host(th).tobytes()))
    return out


CASES = {
    # name: (n, na, nb, H, seed, selected size, system flags, store rows)
    "product": (8, 4, 4, 16, 0, None, 0, False),
    "pull": (10, 5, 4, 12, 5, 2047, 0, False),
    "stored": (10, 5, 4, 12, 5, 2047, 0, True),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("jac", ["dense", "factored"])
@pytest.mark.parametrize("m,k", [(20, 1), (8, 2)])
def test_graph_steps_equal_launched(case, jac, m, k):
    from paper_2601_01437_amd import IRL_WS_FACTORED, IRL_WS_FP64
    announce(f"graph vs launched {case} {jac} m={m} k={k}")
    n, na, nb, H, seed, sel, sflags, store = CASES[case]
    dets = None if sel is None else synth.cisd_like_selected_set(n, na, nb, sel, seed=seed)
    theta = synth.nqs_theta(2 * n, H, seed, scale=0.2)
    fl = IRL_WS_FACTORED if jac == "factored" else IRL_WS_FP64
    ref = _run(_system(n, na, nb, seed, dets, sflags, store), theta, 2 * n, H, 3, False,
               m=m, k_keep=k, ws_flags=fl)
    got = _run(_system(n, na, nb, seed, dets, sflags, store), theta, 2 * n, H, 3, True,
               m=m, k_keep=k, ws_flags=fl)
    assert got == ref
    if (m, k) == (8, 2):
        assert sum(int(x[1][7]) for x in ref) > 0     # restarts were replayed


@pytest.mark.parametrize("mode", ["P", "C"])
def test_graph_modes(mode):
    from paper_2601_01437_amd import IRL_MODE_C, IRL_MODE_P, IRL_WS_FACTORED
    announce(f"graph mode {mode}")
    theta = synth.nqs_theta(16, 16, 3, scale=0.2)
    kw = dict(m=10, k_keep=3, ws_flags=IRL_WS_FACTORED, mode=IRL_MODE_P if mode == "P" else IRL_MODE_C,
              want_dtheta=mode == "C")
    ref = _run(_system(8, 4, 4, 3), theta, 16, 16, 2, False, **kw)
    got = _run(_system(8, 4, 4, 3), theta, 16, 16, 2, True, **kw)
    assert got == ref


def test_graph_fp32_with_polish():
    from paper_2601_01437_amd import IRL_FP32, IRL_WS_FP32, IRL_WS_FP64
    announce("graph fp32 + polish")
    n, na, nb, H, seed, sel = 10, 5, 4, 12, 5, 2047
    dets = synth.cisd_like_selected_set(n, na, nb, sel, seed=seed)
    theta = synth.nqs_theta(2 * n, H, seed, scale=0.2)
    kw = dict(m=12, k_keep=3, precision=IRL_FP32, ws_flags=IRL_WS_FP32 | IRL_WS_FP64)
    ref = _run(_system(n, na, nb, seed, dets), theta, 2 * n, H, 3, False, **kw)
    got = _run(_system(n, na, nb, seed, dets), theta, 2 * n, H, 3, True, **kw)
    assert got == ref


def test_graph_sampled_estimators_and_workspace_change():
    """Sampled (gathered) estimators, then exact steps on a new workspace: the
    graphs follow every change of the key."""
    from paper_2601_01437_amd import (IRL_STEP_GRAPH, IRL_STEP_WS_CURRENT, IRL_WS_FACTORED, IRL_WS_FP64,
                                      IRL_WS_SAMPLED)
    announce("graph sampled + workspace change")
    theta = synth.nqs_theta(16, 16, 4, scale=0.2)
    results = []
    for graph in (False, True):
        s = _system(8, 4, 4, 4)
        th = dev(theta)
        extra = IRL_STEP_GRAPH if graph else 0
        out = []
        fl = IRL_WS_FACTORED | IRL_WS_SAMPLED
        for it in range(3):
            s.evaluate(16, 16, th, ws_flags=fl)
            s.vmc_sample(dev(np.random.default_rng(10 + it).random(3000)))
            rc, r, dth, _ = s.step(th, 16, 16, m=12, k_keep=2, ws_flags=fl, flags=IRL_STEP_WS_CURRENT | extra)
            assert (r.n_graph_cycles > 0) == graph, _last_error(s)
            out.append((rc, _fields(r), host(dth).tobytes()))
        for fl2 in (IRL_WS_FP64, IRL_WS_FACTORED):
            rc, r, dth, _ = s.step(th, 16, 16, m=12, k_keep=2, ws_flags=fl2, flags=extra)
            out.append((rc, _fields(r), host(dth).tobytes()))
        results.append(out)
    assert results[0] == results[1]
