"""Launch-shape tuning through the C ABI: every value of every knob leaves the
operator apply and a whole step bit for bit unchanged (the knobs only move rows
between workgroups), and the autotuner picks a value, records it in its JSON
cache and sets the cached value on a second call without timing."""
import json

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _selected(n_dets=1 << 14, H=256):
    """c3s-shaped selected set (20 orbitals, 10a+10b, CISD-like selection), no
    stored rows, so D~ v is table-driven and H w enumerates excitations."""
    from paper_2601_01437_amd import IRL_WS_FACTORED, System
    w = synth.WORKLOADS["c3s"]
    h, g = synth.integrals(w.n, w.seed)
    dets = synth.cisd_like_selected_set(w.n, w.na, w.nb, n_dets, seed=w.seed)
    s = System(w.n, w.na, w.nb, h, g, dets=dets)
    V = w.V
    P = V * H + H + V
    rng = np.random.default_rng(5)
    theta = dev(rng.normal(scale=0.05, size=P))
    s.evaluate(V, H, theta, ws_flags=IRL_WS_FACTORED)
    return s, V, H, theta


def test_knobs_are_bit_neutral():
    from paper_2601_01437_amd import autotune
    from paper_2601_01437_amd import binding as B
    s, V, H, theta = _selected(n_dets=20000, H=100)
    for knob in autotune.KNOBS:
        assert B.irl_tune_get(s.handle, knob, H)[1], knob
    rng = np.random.default_rng(11)
    v = dev(rng.normal(size=s.ncols))
    Z0, E0, g0 = s.evaluate(V, H, theta, ws_flags=B.IRL_WS_FACTORED)
    g0 = host(g0)
    yH0, yS0 = (host(t) for t in s.apply(v))
    for knob, (name, _, cands) in autotune.KNOBS.items():
        extra = () if knob == B.IRL_TUNE_PULL_WAVES else (1, 7, 157)
        for c in cands + extra:
            announce(f"knob {name} = {c}")
            B.irl_tune_set(s.handle, knob, c)
            assert B.irl_tune_get(s.handle, knob, H)[0] == c
            Z, E, g = s.evaluate(V, H, theta, ws_flags=B.IRL_WS_FACTORED)
            assert Z == Z0 and E == E0 and np.array_equal(host(g), g0), (name, c)
            yH, yS = (host(t) for t in s.apply(v))
            assert np.array_equal(yH, yH0) and np.array_equal(yS, yS0), (name, c)
        B.irl_tune_set(s.handle, knob, 0)
    with pytest.raises(B.IrlError):
        B.irl_tune_set(s.handle, 99, 1)
    with pytest.raises(B.IrlError):
        B.irl_tune_set(s.handle, B.IRL_TUNE_LUT_BLOCKS, -1)
    with pytest.raises(B.IrlError):
        B.irl_tune_set(s.handle, B.IRL_TUNE_PULL_WAVES, 3)


def test_tuned_step_equals_default_step():
    from paper_2601_01437_amd import binding as B
    s, V, H, theta = _selected(n_dets=1 << 14, H=256)
    res = []
    full, graph = B.IRL_STEP_FULL_CYCLES, B.IRL_STEP_FULL_CYCLES | B.IRL_STEP_GRAPH
    for lut, pull, waves, flags in [(0, 0, 0, full), (1024, 8192, 1, full), (0, 0, 0, graph),
                                    (128, 262144, 2, graph), (0, 0, 0, graph)]:
        announce(f"step lut={lut} pull={pull} waves={waves} flags={flags}")
        B.irl_tune_set(s.handle, B.IRL_TUNE_LUT_BLOCKS, lut)
        B.irl_tune_set(s.handle, B.IRL_TUNE_PULL_BLOCKS, pull)
        B.irl_tune_set(s.handle, B.IRL_TUNE_PULL_WAVES, waves)
        rc, r, dth, _ = s.step(theta.clone(), V, H, ws_flags=B.IRL_WS_FACTORED, flags=flags)
        res.append((rc, r.lambda_min, r.E_after, r.n_apply, host(dth)))
        if flags & B.IRL_STEP_GRAPH:
            assert r.n_graph_cycles >= 1
    for x in res[1:]:
        assert x[:4] == res[0][:4]
        assert np.array_equal(x[4], res[0][4])


def test_autotune_cache(tmp_path):
    from paper_2601_01437_amd import autotune
    from paper_2601_01437_amd import binding as B
    s, V, H, theta = _selected(n_dets=1 << 14, H=256)
    path = str(tmp_path / "tune.json")
    cache = autotune.TuneCache(path)
    first = autotune.tune_system(s, H, cache=cache, reps=3)
    announce(f"tuned {first}")
    names = (("lut_blocks", B.IRL_TUNE_LUT_BLOCKS), ("pull_blocks", B.IRL_TUNE_PULL_BLOCKS),
             ("pull_waves", B.IRL_TUNE_PULL_WAVES))
    assert set(first) == {n for n, _ in names}
    data = json.load(open(path))
    assert len(data) == 3
    for name, knob in names:
        assert not first[name]["cached"]
        assert B.irl_tune_get(s.handle, knob, H)[0] == first[name]["value"]
        cands = autotune.KNOBS[knob][2]
        assert [t[0] for t in first[name]["timings"]] == list(cands)
        assert all(t[1] > 0 for t in first[name]["timings"])
    # second system of the same shape: values from the cache, no timing
    s2, _, _, _ = _selected(n_dets=1 << 14, H=256)
    again = autotune.tune_system(s2, H, cache=autotune.TuneCache(path), reps=3)
    for name, knob in names:
        assert again[name]["cached"] and again[name]["value"] == first[name]["value"]
        assert B.irl_tune_get(s2.handle, knob, H)[0] == first[name]["value"]
    # stored rows: the pull knob no longer applies and is not tuned
    s2.store_hamiltonian(1 << 34)
    assert not B.irl_tune_get(s2.handle, B.IRL_TUNE_PULL_BLOCKS)[1]
    assert not B.irl_tune_get(s2.handle, B.IRL_TUNE_PULL_WAVES)[1]
    assert set(autotune.tune_system(s2, H, cache=autotune.TuneCache(path), reps=3)) == {"lut_blocks"}
