"""Reduced-precision operator (FP32 D~ products with FP32 accumulation inside a
row block; energy, gradient, Lanczos and QR in FP64).

The centred matrix is assembled in split form: its psi row and column come from
the FP64 gradient, so an exact wavefunction (g = 0) is still a fixed point with
lambda = 0 and a zero update.  FP32 results are compared with the FP64 oracle
at tolerances stated in each test (a precision report, not FP64 parity); the
FP64 path on the same workloads is held to the FP64 tolerances."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import hamiltonian, lm, space, step
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3s_step.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def flags():
    from paper_2601_01437_amd import IRL_WS_FP32, IRL_WS_FP64
    return IRL_WS_FP64 | IRL_WS_FP32


@pytest.mark.parametrize("polish", [True, False])
def test_fp32_step_c1(c1_problem, polish):
    """FP32 solve + FP64 polish meets the FP64 tolerances; the FP32 solve alone
    is reported against the FP64 oracle."""
    from paper_2601_01437_amd import IRL_FP32, IRL_STEP_NO_POLISH, System
    announce(f"fp32 step c1 polish={polish}")
    p = c1_problem
    w = p["w"]
    res, th_new, E_after = step.lm_step(p["keys"], w.n, w.V, w.H, p["theta"], p["H"])
    s = System(8, 4, 4, p["h"], p["g"])
    rc, r, dth, _ = s.step(dev(p["theta"]), w.V, w.H, m=20, k_keep=1, precision=IRL_FP32,
                           ws_flags=flags(), flags=0 if polish else IRL_STEP_NO_POLISH)
    normH = np.linalg.norm(res.Hp, 2)
    assert r.converged == 1
    assert abs(r.E_before - res.E) <= 1e-12          # energy is FP64
    announce(f"fp32 c1 polish={polish}: dlambda={r.lambda_min - res.lam:.3e} "
             f"dE_after={r.E_after - E_after:.3e} applies={r.n_apply} (fp32 {r.n_apply_lo})")
    if polish:
        assert abs(r.lambda_min - res.lam) <= 1e-10 * max(abs(res.lam), normH)
        assert abs(r.E_after - E_after) <= 1e-12
    else:
        assert abs(r.lambda_min - res.lam) <= 1e-5 * normH
        assert abs(r.E_after - E_after) <= 1e-6


@pytest.mark.parametrize("polish", [True, False])
def test_fp32_exact_psi_is_fixed_point(polish):
    """g = 0 in FP64 => the split-form matrix is [[0, 0], [0, H_eff]]: e_0 is an
    exact eigenvector for eigenvalue 0 although H_eff comes from FP32 products.
    With the FP64 polish the solve reaches it to FP64 accuracy; the FP32 solve
    alone stops at its precision floor (tolerance tol_used)."""
    from paper_2601_01437_amd import IRL_FP32, IRL_STEP_NO_POLISH, System
    announce(f"fp32 fixed point polish={polish}")
    n, na, nb = 5, 3, 2
    h, g = synth.integrals(n, 4)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    psi0 = np.linalg.eigh(Hm)[1][:, 0]
    J = np.random.default_rng(5).normal(size=(keys.size, 30))
    s = System(n, na, nb, h, g)
    s.set_dtilde(dev(np.concatenate([psi0[:, None], J], axis=1)), ws_flags=flags())
    rc, r, dth, _ = s.step(None, m=20, k_keep=2, precision=IRL_FP32,
                           flags=1 | (0 if polish else IRL_STEP_NO_POLISH))
    assert r.converged == 1
    if polish:
        assert abs(r.lambda_min) <= 1e-12
        assert np.max(np.abs(host(dth))) <= 1e-10
    else:
        assert -r.tol_used <= r.lambda_min <= r.tol_used
        announce(f"fp32 only: lambda={r.lambda_min:.3e} tol={r.tol_used:.3e} "
                 f"max|dtheta|={np.max(np.abs(host(dth))):.3e}")


@pytest.fixture(scope="module")
def c3s_golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/c3s_step.json not generated")
    return json.load(open(GOLDEN))


def _c3s_system():
    from paper_2601_01437_amd import System
    w = synth.WORKLOADS["c3s"]
    h, g = w.integrals()
    return w, System(w.n, w.na, w.nb, h, g, dets=w.dets())


def test_c3s_fp64_step_matches_oracle(c3s_golden):
    from paper_2601_01437_amd import IRL_FP64
    announce("c3s fp64 step")
    G = c3s_golden
    w, s = _c3s_system()
    theta = dev(w.theta())
    rc, r, dth, _ = s.step(theta, w.V, w.H, m=w.m, k_keep=w.k, precision=IRL_FP64,
                           ws_flags=flags())
    assert r.converged == 1
    assert abs(r.E_before - G["E"]) <= 1e-12
    assert abs(r.lambda_min - G["lambda_min"]) <= 1e-10 * max(abs(G["lambda_min"]), G["norm_Hp"])
    assert abs(r.E_after - G["E_after"]) <= 1e-12
    d = host(dth)
    assert abs(np.linalg.norm(d) - G["dtheta_norm"]) <= 1e-8 * G["dtheta_norm"]
    assert rel_err(d[:32], np.array(G["dtheta_head"])) <= 1e-8


@pytest.mark.parametrize("polish", [True, False])
def test_c3s_fp32_step(c3s_golden, polish):
    from paper_2601_01437_amd import IRL_FP32, IRL_STEP_NO_POLISH
    announce(f"c3s fp32 step polish={polish}")
    G = c3s_golden
    w, s = _c3s_system()
    theta = dev(w.theta())
    rc, r, dth, _ = s.step(theta, w.V, w.H, m=w.m, k_keep=w.k, precision=IRL_FP32,
                           ws_flags=flags(), flags=0 if polish else IRL_STEP_NO_POLISH)
    assert r.converged == 1
    assert abs(r.E_before - G["E"]) <= 1e-12
    dlam = abs(r.lambda_min - G["lambda_min"])
    dE = abs(r.E_after - G["E_after"])
    announce(f"c3s fp32 polish={polish}: |dlambda|={dlam:.3e} (norm {G['norm_Hp']:.3e}) "
             f"|dE_after|={dE:.3e} applies={r.n_apply} (fp32 {r.n_apply_lo})")
    if polish:
        assert dlam <= 1e-10 * max(abs(G["lambda_min"]), G["norm_Hp"])
        assert dE <= 1e-12
    else:
        assert dlam <= 1e-5 * G["norm_Hp"]
        assert dE <= 1e-5 * max(1.0, abs(G["E_after"]))


def test_c3s_fp32_only_workspace(c3s_golden):
    """FP32 copy of D~ only: energy and gradient stay FP64 (the gradient is
    recomputed from theta), the solve runs on FP32 products without polish."""
    from paper_2601_01437_amd import IRL_FP32, IRL_STEP_NO_POLISH, IRL_WS_FP32
    announce("c3s fp32-only workspace")
    G = c3s_golden
    w, s = _c3s_system()
    theta = dev(w.theta())
    Z, E, grad = s.evaluate(w.V, w.H, theta, ws_flags=IRL_WS_FP32)
    assert abs(E - G["E"]) <= 1e-12
    assert abs(np.linalg.norm(host(grad)) - G["grad_norm"]) <= 1e-10 * G["grad_norm"]
    assert rel_err(host(grad)[:32], np.array(G["grad_head"])) <= 1e-10
    rc, r, dth, _ = s.step(theta, w.V, w.H, m=w.m, k_keep=w.k, precision=IRL_FP32,
                           ws_flags=IRL_WS_FP32, flags=IRL_STEP_NO_POLISH)
    assert r.converged == 1 and r.n_apply_lo == r.n_apply
    dlam = abs(r.lambda_min - G["lambda_min"])
    dE = abs(r.E_after - G["E_after"])
    announce(f"c3s fp32-only: |dlambda|={dlam:.3e} |dE_after|={dE:.3e} applies={r.n_apply}")
    assert dlam <= 1e-5 * G["norm_Hp"]
    assert dE <= 1e-5 * max(1.0, abs(G["E_after"]))
