"""Serving lanes (continuous admission into resident slots, one host thread and
stream per class) through the C ABI: every request completes, requests of one
class are admitted together when they queue up, and each result in the mix is
bit-for-bit the result of the same request run alone."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _pools(precision, factored=False):
    from paper_2601_01437_amd.serving import ClassPool, ClassSpec
    specs = {}
    for name, (n, na, nb, H, sel) in {"a": (6, 3, 3, 8, None), "b": (8, 4, 4, 16, None),
                                      "s": (10, 5, 5, 12, 2000)}.items():
        h, g = synth.integrals(n, 7)
        dets = None if sel is None else synth.cisd_like_selected_set(n, na, nb, sel, seed=7)
        specs[name] = ClassPool(ClassSpec(name, n, na, nb, 2 * n, H, h, g, dets=dets, m=20, k_keep=1,
                                          precision=precision, slots=4,
                                          store_rows_bytes=(1 << 30) if name == "s" else 0,
                                          factored=factored))
    return specs


@pytest.mark.parametrize("fp32,factored", [(False, False), (True, False), (False, True)])
def test_serving_results_equal_alone(fp32, factored):
    from paper_2601_01437_amd import IRL_FP32, IRL_FP64
    from paper_2601_01437_amd.serving import Request, Server
    announce(f"serving lanes fp32={fp32} factored={factored}")
    pools = _pools(IRL_FP32 if fp32 else IRL_FP64, factored)
    arr, picks = synth.serving_arrivals(60, 120.0, {"a": 0.5, "b": 0.3, "s": 0.2}, seed=1)
    reqs = [Request(i, picks[i], float(arr[i]),
                    synth.nqs_theta(pools[picks[i]].spec.V, pools[picks[i]].spec.H, 50 + i, scale=0.2))
            for i in range(len(arr))]
    makespan = Server(pools).run(reqs)
    assert makespan >= arr[-1]
    assert all(np.isfinite(r.end) and r.end >= r.arrival for r in reqs)
    assert all(r.status in (0, 2) for r in reqs)
    for r in reqs:
        alone = Request(r.rid, r.cls, 0.0, r.theta)
        pools[r.cls].step([alone])
        assert (alone.lambda_min, alone.E_after, alone.n_apply, alone.status) == \
            (r.lambda_min, r.E_after, r.n_apply, r.status), r.rid
    for p in pools.values():
        p.close()


def test_serving_admits_queued_requests_together():
    from paper_2601_01437_amd import IRL_FP64
    from paper_2601_01437_amd.serving import Request, Server
    pools = _pools(IRL_FP64)
    # ten requests of one class, all arrived at t = 0: admitted 4, 4, 2
    reqs = [Request(i, "b", 0.0, synth.nqs_theta(16, 16, 80 + i, scale=0.2)) for i in range(10)]
    Server({"b": pools["b"]}).run(reqs)
    assert sorted(r.batch_size for r in reqs) == [2, 2] + [4] * 8
    for p in pools.values():
        p.close()


def _varied_specs(precision, factored):
    """Request classes that no pool holds in advance (full spaces and selected sets
    of several sizes and network widths)."""
    from paper_2601_01437_amd.serving import ClassSpec
    out = []
    for i, (n, na, nb, H, sel) in enumerate([(6, 3, 3, 8, None), (8, 4, 4, 16, None), (7, 3, 4, 12, None),
                                             (10, 5, 5, 12, 2000), (12, 6, 6, 24, 5000)]):
        h, g = synth.integrals(n, 11 + i)
        dets = None if sel is None else synth.cisd_like_selected_set(n, na, nb, sel, seed=11 + i)
        out.append(ClassSpec(f"v{i}", n, na, nb, 2 * n, H, h, g, dets=dets, m=20, k_keep=1,
                             precision=precision, slots=1, store_rows_bytes=(1 << 30) if sel else 0,
                             factored=factored))
    return out


def _alone(spec, theta):
    """The same step alone, on a fresh system and workspace."""
    import torch
    from paper_2601_01437_amd import System
    s = System(spec.n, spec.na, spec.nb, spec.h, spec.g, dets=spec.dets)
    try:
        if spec.store_rows_bytes and not s.info.full_space:
            s.store_hamiltonian(spec.store_rows_bytes)
        s.workspace(spec.P + 1, spec.ws_flags)
        th = torch.tensor(theta, dtype=torch.float64, device="cuda")
        rc, res, _, _ = s.step(th, spec.V, spec.H, m=spec.m, k_keep=spec.k_keep, tol=spec.tol,
                               precision=spec.precision, ws_flags=spec.ws_flags, want_dtheta=False)
        return rc, res
    finally:
        s.close()


@pytest.mark.parametrize("factored", [False, True])
def test_footprint_admission_any_class(factored):
    """Requests of classes not built in advance are admitted when their slot's bytes
    (system, stored rows, workspace from irl_workspace_query) fit the budget; the
    budget holds about two slots, so requests wait and idle slots of other classes
    are evicted; every result equals the same request alone, bit for bit."""
    from paper_2601_01437_amd import IRL_FP64
    from paper_2601_01437_amd.serving import FootprintServer, Request, latency_summary
    announce(f"footprint admission factored={factored}")
    specs = _varied_specs(IRL_FP64, factored)
    # each class's slot bytes, measured once with room to spare
    probe = FootprintServer(1 << 40, lanes=1)
    sizes = []
    for sp in specs:
        sl = probe._create(sp, 1 << 40)
        sizes.append(sl.nbytes)
        probe._destroy(sl)
    budget = sorted(sizes)[-1] + sorted(sizes)[-2] + (1 << 20)
    rng = np.random.default_rng(5)
    picks = rng.integers(0, len(specs), size=40)
    arr = np.cumsum(rng.exponential(1 / 200.0, size=40))
    reqs = [Request(i, specs[p].name, float(arr[i]),
                    synth.nqs_theta(specs[p].V, specs[p].H, 300 + i, scale=0.2), spec=specs[p])
            for i, p in enumerate(picks)]
    srv = FootprintServer(budget, lanes=3, max_batch=4)
    try:
        makespan = srv.run(reqs)
        adm = srv.adm
        assert adm.peak <= budget
        assert adm.evicted >= 1 and adm.reused >= 1
    finally:
        srv.close()
    lat = latency_summary(reqs)
    print(f"[footprint] makespan {makespan:.2f} s p50 {lat['p50_ms']:.1f} ms p99 {lat['p99_ms']:.1f} ms "
          f"created {adm.created} evicted {adm.evicted} reused {adm.reused} peak {adm.peak} / {budget}")
    assert all(np.isfinite(r.end) and r.end >= r.arrival for r in reqs)
    assert all(r.status in (0, 2) for r in reqs)
    for r in reqs:
        rc, res = _alone(r.spec, r.theta)
        assert (res.lambda_min, res.E_after, res.n_apply, rc) == \
            (r.lambda_min, r.E_after, r.n_apply, r.status), r.rid


def test_footprint_admission_refuses_what_never_fits():
    from paper_2601_01437_amd import IRL_FP64
    from paper_2601_01437_amd.serving import FootprintServer, Request
    sp = _varied_specs(IRL_FP64, True)[4]
    srv = FootprintServer(1 << 20, lanes=1)
    try:
        with pytest.raises(RuntimeError, match="does not fit"):
            srv.run([Request(0, sp.name, 0.0, synth.nqs_theta(sp.V, sp.H, 1, scale=0.2), spec=sp)])
    finally:
        srv.close()


def test_system_bytes_estimate_bounds_the_created_system():
    from paper_2601_01437_amd import System
    from paper_2601_01437_amd.serving import estimate_system_bytes
    for n, na, nb, sel in [(6, 3, 3, None), (8, 4, 4, None), (12, 6, 6, None), (10, 5, 5, 2000),
                           (16, 8, 8, 100000)]:
        h, g = synth.integrals(n, 3)
        dets = None if sel is None else synth.cisd_like_selected_set(n, na, nb, sel, seed=3)
        s = System(n, na, nb, h, g, dets=dets)
        try:
            est = estimate_system_bytes(n, na, nb, None if dets is None else len(dets))
            assert est >= s.info.device_bytes, (n, sel, est, s.info.device_bytes)
        finally:
            s.close()
