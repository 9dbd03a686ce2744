"""Multi-vector operator and thick-restart block Lanczos (GPU through the C ABI).

The multi-vector apply returns, per column, the same raw operator pair as the
oracle's matrix-free apply (||y - y_ref|| <= 1e-10 ||y_ref||, FP64).  The block
solve converges to the oracle's lowest eigenpair of the centred matrix with the
same tolerances as the single-vector step (eigenvalue 1e-10 max(|lambda|,
||H~'||), energies 1e-12 Ha), with an FP64 D~ copy and with the factored
Jacobian; the pins that do not depend on the Krylov method (D~ = I is exact
diagonalisation, an exact psi gives a zero update) hold too."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import hamiltonian, lm, nqs, space, step
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3s_step.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _flags(fp32=False, factored=False):
    from paper_2601_01437_amd import IRL_WS_BLOCK, IRL_WS_FACTORED, IRL_WS_FP32, IRL_WS_FP64
    if factored:
        return IRL_WS_FACTORED | IRL_WS_BLOCK
    return IRL_WS_FP64 | IRL_WS_BLOCK | (IRL_WS_FP32 if fp32 else 0)


def _system(n, na, nb, seed=0, dets=None, flags=0):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets, flags=flags), h, g


@pytest.fixture(scope="module")
def c1_oracle(c1_problem):
    p = c1_problem
    w = p["w"]
    Dt = nqs.dtilde(p["keys"], w.n, w.V, w.H, p["theta"])
    res, th_new, E_after = step.lm_step(p["keys"], w.n, w.V, w.H, p["theta"], p["H"])
    return Dt, res, th_new, E_after


@pytest.mark.parametrize("factored", [False, True])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 8])
def test_multi_vector_apply_c1(c1_problem, c1_oracle, nb, factored):
    """Per column: the oracle's operator pair; the single-vector apply to
    rounding with a D~ copy, bit for bit with the factored Jacobian (whose block
    apply is one single-vector apply per column)."""
    announce(f"multi-vector apply c1 nb={nb} factored={factored}")
    p = c1_problem
    w = p["w"]
    Dt = c1_oracle[0]
    s, _, _ = _system(8, 4, 4)
    s.evaluate(w.V, w.H, dev(p["theta"]), ws_flags=_flags(factored=factored))
    V = np.random.default_rng(10 + nb).normal(size=(nb, w.P + 1))
    YH, YS = s.apply_block(dev(V))
    YH, YS = host(YH), host(YS)
    for q in range(nb):
        yH, yS = lm.apply_lm_operator(Dt, p["H"], V[q])
        assert rel_err(YH[q], yH) <= 1e-10, q
        assert rel_err(YS[q], yS) <= 1e-10, q
        # the same column through the single-vector apply
        y1H, y1S = s.apply(dev(V[q]))
        assert rel_err(YH[q], host(y1H)) <= 1e-13 and rel_err(YS[q], host(y1S)) <= 1e-13
        if factored:
            assert np.array_equal(YH[q], host(y1H)) and np.array_equal(YS[q], host(y1S))


@pytest.mark.parametrize("nb", [2, 4, 8])
def test_multi_vector_apply_selected_fp32(nb):
    """Selected set, row length not a multiple of the tile (P + 1 = 10,537), FP32
    copy: every column equals the single-vector FP32 apply to FP32 rounding."""
    from paper_2601_01437_amd import IRL_FP32
    announce(f"multi-vector apply c3s fp32 nb={nb}")
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    from paper_2601_01437_amd import System
    s = System(w.n, w.na, w.nb, h, g, dets=w.dets())
    s.evaluate(w.V, w.H, dev(w.theta()), ws_flags=_flags(fp32=True))
    V = np.random.default_rng(20 + nb).normal(size=(nb, w.P + 1))
    YH, YS = s.apply_block(dev(V), precision=IRL_FP32)
    YH64, YS64 = s.apply_block(dev(V))
    for q in range(nb):
        y1H, y1S = s.apply(dev(V[q]), precision=IRL_FP32)
        assert rel_err(host(YH[q]), host(y1H)) <= 1e-6 and rel_err(host(YS[q]), host(y1S)) <= 1e-6
        y1H, y1S = s.apply(dev(V[q]))
        assert rel_err(host(YH64[q]), host(y1H)) <= 1e-13 and rel_err(host(YS64[q]), host(y1S)) <= 1e-13


@pytest.mark.parametrize("factored", [False, True])
@pytest.mark.parametrize("nb,m,k", [(2, 20, 4), (4, 20, 4), (4, 40, 10), (2, 8, 2), (8, 24, 8)])
def test_block_step_c1(c1_problem, c1_oracle, nb, m, k, factored):
    announce(f"block step c1 nb={nb} m={m} k={k} factored={factored}")
    p = c1_problem
    w = p["w"]
    _, res, th_new, E_after = c1_oracle
    s, _, _ = _system(8, 4, 4)
    theta = dev(p["theta"])
    rc, r, dth, ritz = s.step(theta, w.V, w.H, m=m, k_keep=k, want_ritz=True, block=nb,
                              ws_flags=_flags(factored=factored))
    normH = np.linalg.norm(res.Hp, 2)
    announce(f"block nb={nb}: applies {r.n_apply} restarts {r.n_restart} "
             f"dlambda {r.lambda_min - res.lam:.2e}")
    assert rc == 0 and r.converged == 1
    assert abs(r.E_before - res.E) <= 1e-12
    assert abs(r.lambda_min - res.lam) <= 1e-10 * max(abs(res.lam), normH)
    assert rel_err(host(dth), res.dtheta) <= 1e-8
    assert abs(r.E_after - E_after) <= 1e-12
    assert rel_err(host(theta), th_new) <= 1e-10
    assert abs(abs(host(ritz) @ res.c) - 1.0) <= 1e-10
    assert r.residual_explicit <= max(1e-12, 1024 * 2.2e-16 * normH)


def test_block_step_mode_p(c1_problem, c1_oracle):
    from paper_2601_01437_amd import IRL_MODE_P
    announce("block step c1 mode P")
    p = c1_problem
    w = p["w"]
    Dt = c1_oracle[0]
    resP = lm.solve(Dt, p["H"], mode="P")
    s, _, _ = _system(8, 4, 4)
    s.evaluate(w.V, w.H, dev(p["theta"]), ws_flags=_flags())
    rc, r, _, ritz = s.step(None, m=24, k_keep=4, mode=IRL_MODE_P, flags=1, want_ritz=True,
                            want_dtheta=False, block=4)
    normH = np.linalg.norm(resP.Hp[1:, 1:], 2)
    assert r.converged == 1
    assert abs(r.lambda_min - resP.lam) <= 1e-10 * max(abs(resP.lam), normH)
    assert abs(abs(host(ritz) @ resP.c) - 1.0) <= 1e-9


def test_block_identity_dtilde_is_exact_diagonalisation():
    announce("block: dtilde = I")
    n, na, nb = 5, 2, 2
    s, h, g = _system(n, na, nb, seed=3)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    e_exact = np.linalg.eigvalsh(Hm)[0]
    s.set_dtilde(dev(np.eye(keys.size)), ws_flags=_flags())
    rc, r, _, _ = s.step(None, m=40, k_keep=8, flags=1, block=4)
    assert r.converged == 1
    assert abs(r.lambda_min + r.E_before - e_exact) <= 1e-10


def test_block_exact_psi_gives_zero_update():
    announce("block: exact psi")
    n, na, nb = 5, 3, 2
    s, h, g = _system(n, na, nb, seed=4)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    psi0 = np.linalg.eigh(Hm)[1][:, 0]
    J = np.random.default_rng(5).normal(size=(keys.size, 30))
    s.set_dtilde(dev(np.concatenate([psi0[:, None], J], axis=1)), ws_flags=_flags())
    rc, r, dth, _ = s.step(None, m=20, k_keep=4, flags=1, block=4)
    assert abs(r.lambda_min) <= 1e-12
    assert np.max(np.abs(host(dth))) <= 1e-10


def test_block_invariant_subspace_breakdown():
    """A 6-dimensional problem with block 2: the Krylov space is the whole space
    after three block steps (m is clamped to 6), the next block is numerically
    zero and is replaced by fresh directions, and the step still returns the
    exact lowest eigenpair."""
    announce("block: breakdown")
    rng = np.random.default_rng(8)
    n, na, nb = 4, 1, 1
    s, h, g = _system(n, na, nb, seed=6)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    D = np.concatenate([rng.normal(size=(keys.size, 1)), rng.normal(size=(keys.size, 5))], axis=1)
    s.set_dtilde(dev(D), ws_flags=_flags())
    Z = D[:, 0] @ D[:, 0]
    E = D[:, 0] @ Hm @ D[:, 0] / Z
    Hp = (D.T @ Hm @ D - E * D.T @ D) / Z
    lam_ref = np.linalg.eigvalsh(Hp)[0]
    rc, r, _, _ = s.step(None, m=16, k_keep=4, flags=1 | 2, block=2, want_dtheta=False)
    assert r.converged == 1
    assert abs(r.lambda_min - lam_ref) <= 1e-10 * max(1.0, np.abs(np.linalg.eigvalsh(Hp)).max())


@pytest.mark.parametrize("factored", [False, True])
def test_block_c3s_step_matches_oracle(factored):
    """2^14-determinant, 20-orbital selected set with P = 10,536, FP64, block 4,
    with the FP64 D~ copy and with the factored Jacobian."""
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c3s_step.json not generated")
    from paper_2601_01437_amd import System
    announce(f"block c3s step factored={factored}")
    G = json.load(open(GOLDEN))
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    s = System(w.n, w.na, w.nb, h, g, dets=w.dets())
    rc, r, dth, _ = s.step(dev(w.theta()), w.V, w.H, m=40, k_keep=8, block=4,
                           ws_flags=_flags(factored=factored))
    announce(f"block c3s: applies {r.n_apply} restarts {r.n_restart}")
    assert r.converged == 1
    assert abs(r.E_before - G["E"]) <= 1e-12
    assert abs(r.lambda_min - G["lambda_min"]) <= 1e-10 * max(abs(G["lambda_min"]), G["norm_Hp"])
    assert abs(r.E_after - G["E_after"]) <= 1e-12
    d = host(dth)
    assert abs(np.linalg.norm(d) - G["dtheta_norm"]) <= 1e-8 * G["dtheta_norm"]


def test_block_option_errors():
    from paper_2601_01437_amd import IRL_WS_FP64, IrlError
    p_n = 5
    s, _, _ = _system(p_n, 2, 2, seed=1)
    theta = dev(synth.nqs_theta(10, 4, 1))
    with pytest.raises(IrlError):                       # no IRL_WS_BLOCK
        s.step(theta, 10, 4, m=16, k_keep=2, block=4, ws_flags=IRL_WS_FP64)
    with pytest.raises(IrlError):                       # block > 8
        s.step(theta, 10, 4, m=32, k_keep=2, block=9, ws_flags=_flags())
    with pytest.raises(IrlError):                       # m < 2 * block
        s.step(theta, 10, 4, m=6, k_keep=2, block=4, ws_flags=_flags())
