"""Factored Jacobian (IRL_WS_FACTORED) through the C ABI: the operator, the
gradient and whole steps computed from psi, d = 1 - t^2 and the occupations
(forward and backward products of the network) match the oracle at the FP64
tolerances of the dense path (operator 1e-10 relative, eigenvalue 1e-10
max(|lambda|, ||H~'||), energies 1e-12 Ha), and the dense FP64 path to rounding."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import capply, lm, nqs, step
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3s_step.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _fl():
    from paper_2601_01437_amd import IRL_WS_FACTORED
    return IRL_WS_FACTORED


def _system(n, na, nb, seed=0, dets=None):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets), h, g


def test_factored_evaluate_and_apply_c1(c1_problem):
    announce("factored evaluate/apply c1")
    p = c1_problem
    w = p["w"]
    Dt = nqs.dtilde(p["keys"], w.n, w.V, w.H, p["theta"])
    Z, E_el, E = lm.energy(Dt[:, 0], p["H"])
    g = lm.gradient(Dt, p["H"])
    s, _, _ = _system(8, 4, 4)
    Zg, Eg, grad = s.evaluate(w.V, w.H, dev(p["theta"]), ws_flags=_fl())
    assert abs(Zg - Z) <= 1e-12 * Z and abs(Eg - E) <= 1e-12
    assert rel_err(host(grad), g) <= 1e-10
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.normal(size=w.P + 1)
        yH, yS = s.apply(dev(v))
        rH, rS = lm.apply_lm_operator(Dt, p["H"], v)
        assert rel_err(host(yH), rH) <= 1e-10 and rel_err(host(yS), rS) <= 1e-10


@pytest.mark.parametrize("n,na,nb,V,H,count,seed", [(32, 3, 2, 64, 70, 3000, 1), (12, 6, 6, 24, 100, 20000, 2),
                                                     (20, 10, 10, 40, 256, 1 << 14, 0)])
def test_factored_matches_dense_fp64(n, na, nb, V, H, count, seed):
    """V = 64, hidden widths not multiples of 64 and several row blocks: the
    factored operator and gradient equal the dense FP64 ones to rounding."""
    from paper_2601_01437_amd import IRL_WS_FP64
    announce(f"factored vs dense n={n} H={H}")
    keys = synth.cisd_like_selected_set(n, na, nb, count, seed=seed)
    s, _, _ = _system(n, na, nb, seed=seed, dets=keys)
    theta = dev(synth.nqs_theta(V, H, seed, scale=0.2))
    v = dev(np.random.default_rng(seed).normal(size=V * H + H + V + 1))
    Z1, E1, g1 = s.evaluate(V, H, theta, ws_flags=IRL_WS_FP64)
    yH1, yS1 = s.apply(v)
    Z2, E2, g2 = s.evaluate(V, H, theta, ws_flags=_fl())
    yH2, yS2 = s.apply(v)
    assert abs(Z2 - Z1) <= 1e-13 * Z1 and abs(E2 - E1) <= 1e-12
    assert rel_err(host(g2), host(g1)) <= 1e-12
    assert rel_err(host(yH2), host(yH1)) <= 1e-12 and rel_err(host(yS2), host(yS1)) <= 1e-12


@pytest.mark.parametrize("n,na,nb,H,seed", [
    (10, 5, 5, 64, 3),    # 63,504 rows: 252 x 252 strings, one hidden tile
    (10, 5, 4, 100, 4),   # 252 x 210 strings, a ragged second hidden tile
    (10, 4, 5, 16, 5),    # 210 x 252, a quarter of the lanes per tile
    (13, 6, 5, 8, 6),     # 1716 x 1287 strings (2.2 M rows), 13 alpha orbitals
    (14, 1, 6, 24, 7),    # 14 x 3003 strings: one alpha range, 188 tiles of beta strings
    (14, 6, 1, 24, 8),    # 3003 x 14 strings: one partial tile, 188 alpha ranges
])
def test_factored_full_space_string_split(n, na, nb, H, seed):
    """Full spaces of 32,768 rows or more take the string-split backward product
    (alpha/beta partial sums, no matrix-core work): the gradient, the operator pair,
    the connected-basis sigma and a whole step equal the dense FP64 path to rounding."""
    from paper_2601_01437_amd import IRL_MODE_C, IRL_WS_FP64
    announce(f"factored full space n={n} {na}+{nb} H={H}")
    V = 2 * n
    theta = synth.nqs_theta(V, H, seed, scale=0.2)
    out = {}
    for fl in (IRL_WS_FP64, _fl()):
        s, _, _ = _system(n, na, nb, seed=seed)
        assert s.info.full_space
        Z, E, g = s.evaluate(V, H, dev(theta), ws_flags=fl)
        v = dev(np.random.default_rng(seed).normal(size=V * H + H + V + 1))
        yH, yS = s.apply(v)
        rc, r, dth, _ = s.step(dev(theta), V, H, m=12, k_keep=2, ws_flags=fl, mode=IRL_MODE_C)
        out[fl] = (Z, E, host(g), host(yH), host(yS), r.lambda_min, r.E_after, r.norm_T, host(dth))
    a, b = out[IRL_WS_FP64], out[_fl()]
    assert abs(b[0] - a[0]) <= 1e-13 * a[0] and abs(b[1] - a[1]) <= 1e-12
    for k in (2, 3, 4):
        assert rel_err(b[k], a[k]) <= 1e-12, k
    assert abs(b[5] - a[5]) <= 1e-10 * max(abs(a[5]), a[7])
    assert abs(b[6] - a[6]) <= 1e-12 * max(1.0, abs(a[6]))
    assert rel_err(b[8], a[8]) <= 1e-8


def test_factored_full_space_string_split_vs_oracle():
    """The string-split product on 63,504 rows against the oracle's dense D~ and
    Slater-Condon rows: Z, E, the gradient and the operator pair."""
    announce("factored full space vs oracle n=10 5+5 H=12")
    from oracle import space
    n, na, nb, H, seed = 10, 5, 5, 12, 8
    V = 2 * n
    s, h, g = _system(n, na, nb, seed=seed)
    keys = space.full_space(n, na, nb)
    Hm = capply.csr(n, h, g, keys)
    th = synth.nqs_theta(V, H, seed, scale=0.3)
    Dt = nqs.dtilde(keys, n, V, H, th)
    Z, _, E = lm.energy(Dt[:, 0], Hm)
    Zg, Eg, grad = s.evaluate(V, H, dev(th), ws_flags=_fl())
    assert abs(Zg - Z) <= 1e-12 * Z and abs(Eg - E) <= 1e-12 * max(1.0, abs(E))
    assert rel_err(host(grad), lm.gradient(Dt, Hm)) <= 1e-10
    v = np.random.default_rng(seed).normal(size=V * H + H + V + 1)
    yH, yS = s.apply(dev(v))
    rH, rS = lm.apply_lm_operator(Dt, Hm, v)
    assert rel_err(host(yH), rH) <= 1e-10 and rel_err(host(yS), rS) <= 1e-10


@pytest.mark.parametrize("n,na,nb,H,count,seed", [
    (6, 3, 2, 5, 151, 3),       # V = 12 (one column tile, two k-steps padded), H = 5 (unaligned d rows)
    (8, 4, 3, 64, 1001, 4),     # V = 16, exactly one hidden chunk, ragged 16-row tail
    (10, 5, 4, 130, 2047, 5),   # three hidden chunks (the last one 2 wide), H % 4 != 0
    (11, 3, 3, 33, 17, 6),      # 17 rows: one full tile plus one row
    (9, 5, 4, 7, 1, 7),         # one determinant
    # the table-driven D~ v (H a multiple of 64): one group of 4 orbitals per spin
    # with two hidden chunks, six groups (n = 24), three chunks with a ragged batch
    (3, 2, 1, 128, 9, 8),
    (24, 3, 3, 64, 3001, 9),
    (12, 4, 4, 192, 4097, 10),
    (5, 2, 2, 64, 1, 11),       # one determinant through the table-driven kernels
])
def test_factored_shapes_vs_oracle(n, na, nb, H, count, seed):
    """Tile edges of the matrix-core kernels against the oracle's dense D~:
    psi (through Z and E), the gradient and the operator pair."""
    announce(f"factored shapes n={n} H={H} rows={count}")
    V = 2 * n
    keys = synth.cisd_like_selected_set(n, na, nb, count, seed=seed)
    s, h, g = _system(n, na, nb, seed=seed, dets=keys)
    Hm = capply.csr(n, h, g, keys)
    th = synth.nqs_theta(V, H, seed, scale=0.3)
    Dt = nqs.dtilde(keys, n, V, H, th)
    Z, _, E = lm.energy(Dt[:, 0], Hm)
    Zg, Eg, grad = s.evaluate(V, H, dev(th), ws_flags=_fl())
    assert abs(Zg - Z) <= 1e-12 * Z and abs(Eg - E) <= 1e-12 * max(1.0, abs(E))
    g_ref = lm.gradient(Dt, Hm)
    if keys.size == 1:                      # psi is an eigenvector: the gradient vanishes
        assert np.max(np.abs(host(grad))) <= 1e-12 * max(1.0, abs(E))
    else:
        assert rel_err(host(grad), g_ref) <= 1e-10
    rng = np.random.default_rng(seed)
    for zero_v0 in (False, True):
        v = rng.normal(size=V * H + H + V + 1)
        if zero_v0:
            v[0] = 0.0
        yH, yS = s.apply(dev(v))
        rH, rS = lm.apply_lm_operator(Dt, Hm, v)
        assert rel_err(host(yH), rH) <= 1e-10 and rel_err(host(yS), rS) <= 1e-10


@pytest.mark.parametrize("m,k", [(20, 1), (12, 3)])
def test_factored_step_c1(c1_problem, m, k):
    announce(f"factored step c1 m={m} k={k}")
    p = c1_problem
    w = p["w"]
    res, th_new, E_after = step.lm_step(p["keys"], w.n, w.V, w.H, p["theta"], p["H"])
    s, _, _ = _system(8, 4, 4)
    theta = dev(p["theta"])
    rc, r, dth, _ = s.step(theta, w.V, w.H, m=m, k_keep=k, ws_flags=_fl())
    normH = np.linalg.norm(res.Hp, 2)
    assert rc == 0 and r.converged == 1
    assert abs(r.E_before - res.E) <= 1e-12
    assert abs(r.lambda_min - res.lam) <= 1e-10 * max(abs(res.lam), normH)
    assert rel_err(host(dth), res.dtheta) <= 1e-8
    assert abs(r.E_after - E_after) <= 1e-12
    assert rel_err(host(theta), th_new) <= 1e-10


@pytest.fixture(scope="module")
def c3s_golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c3s_step.json not generated")
    return json.load(open(GOLDEN))


@pytest.mark.parametrize("fp32", [False, True])
def test_factored_c3s_step(c3s_golden, fp32):
    """2^14-determinant 20-orbital set, P = 10,536: FP64 step on the factored
    Jacobian, or FP32 D~ products polished in FP64 through the factored form."""
    from paper_2601_01437_amd import IRL_FP32, IRL_FP64, IRL_WS_FP32, System
    announce(f"factored c3s step fp32={fp32}")
    G = c3s_golden
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    s = System(w.n, w.na, w.nb, h, g, dets=w.dets())
    fl = _fl() | (IRL_WS_FP32 if fp32 else 0)
    rc, r, dth, _ = s.step(dev(w.theta()), w.V, w.H, m=w.m, k_keep=w.k, ws_flags=fl,
                           precision=IRL_FP32 if fp32 else IRL_FP64)
    assert r.converged == 1
    assert abs(r.E_before - G["E"]) <= 1e-12
    assert abs(r.lambda_min - G["lambda_min"]) <= 1e-10 * max(abs(G["lambda_min"]), G["norm_Hp"])
    assert abs(r.E_after - G["E_after"]) <= 1e-12
    d = host(dth)
    assert abs(np.linalg.norm(d) - G["dtheta_norm"]) <= 1e-8 * G["dtheta_norm"]


def test_factored_errors():
    from paper_2601_01437_amd import IrlError, Batch
    announce("factored errors")
    s, _, _ = _system(5, 2, 2, seed=1)
    with pytest.raises(IrlError):                   # a caller-set D~ has no factored form
        s.set_dtilde(dev(np.eye(100)[:, :7]), ws_flags=_fl())
    theta = dev(synth.nqs_theta(10, 4, 1))
    s.evaluate(10, 4, theta, ws_flags=_fl())
    with pytest.raises(IrlError):                   # multi-vector applies need a D~ copy
        s.apply_block(dev(np.ones((2, 55))))
    with pytest.raises(IrlError):                   # a batch holds D~ copies or the factored Jacobian
        from paper_2601_01437_amd import IRL_WS_FP64
        Batch([s], [theta], [10], [4], ws_flags=_fl() | IRL_WS_FP64)
