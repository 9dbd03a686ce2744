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
