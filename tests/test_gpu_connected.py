"""Connected tangent basis (IRL_MODE_C) through the C ABI against the oracle's
mode C (explicitly projected D~, dense solve): eigenvalue within 1e-10
max(|lambda|, ||H~'_c||), update within 1e-8 relative, energies within 1e-12 Ha,
on the dense FP64 copy and on the factored Jacobian; plus the properties the
oracle pins (zero update at an exact psi, invariance under adding multiples of
psi to the derivative columns) checked on the GPU path itself."""
import numpy as np
import pytest

import synth
from oracle import capply, hamiltonian, lm, nqs, space, step
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(n, na, nb, seed=0, dets=None):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets), h, g


def _ws(factored):
    from paper_2601_01437_amd import IRL_WS_FACTORED, IRL_WS_FP64
    return IRL_WS_FACTORED if factored else IRL_WS_FP64


def _check(rc, r, dth, theta, res, th_new, E_after):
    normH = np.linalg.norm(res.Hp, 2)
    assert rc == 0 and r.converged == 1
    assert abs(r.E_before - res.E) <= 1e-12 * max(1.0, abs(res.E))
    assert abs(r.lambda_min - res.lam) <= 1e-10 * max(abs(res.lam), normH)
    assert rel_err(host(dth), res.dtheta) <= 1e-8
    assert abs(r.E_after - E_after) <= 1e-12 * max(1.0, abs(E_after))
    assert rel_err(host(theta), th_new) <= 1e-10
    assert r.residual_explicit <= max(1e-12, 1024 * 2.2e-16 * normH)


@pytest.fixture(scope="module")
def c1_oracle_c(c1_problem):
    p = c1_problem
    w = p["w"]
    return step.lm_step(p["keys"], w.n, w.V, w.H, p["theta"], p["H"], mode="C")


@pytest.mark.parametrize("factored", [False, True])
@pytest.mark.parametrize("m,k", [(20, 1), (12, 3)])
def test_connected_step_c1(c1_problem, c1_oracle_c, factored, m, k):
    from paper_2601_01437_amd import IRL_MODE_C
    announce(f"connected step c1 factored={factored} m={m} k={k}")
    p = c1_problem
    w = p["w"]
    res, th_new, E_after = c1_oracle_c
    s, _, _ = _system(8, 4, 4)
    theta = dev(p["theta"])
    rc, r, dth, ritz = s.step(theta, w.V, w.H, m=m, k_keep=k, mode=IRL_MODE_C, ws_flags=_ws(factored),
                              want_ritz=True)
    _check(rc, r, dth, theta, res, th_new, E_after)
    c = host(ritz)
    assert abs(abs(c @ res.c) - 1.0) <= 1e-10
    # the reported c0 is the coefficient of psi, c_0 - sigma . c[1:] (sign of the Ritz vector)
    _, sigma = lm.connected_basis(nqs.dtilde(p["keys"], w.n, w.V, w.H, p["theta"]))
    den = c[0] - sigma @ c[1:]
    assert abs(r.c0 - den) <= 1e-10 * max(1.0, abs(den))


@pytest.mark.parametrize("n,na,nb,H,count,seed", [(10, 5, 4, 13, 2047, 5), (12, 4, 4, 40, 3001, 8)])
def test_connected_step_selected_set(n, na, nb, H, count, seed):
    """Selected sets with several row tiles and a ragged tail, factored Jacobian."""
    from paper_2601_01437_amd import IRL_MODE_C
    announce(f"connected step selected n={n} H={H} rows={count}")
    V = 2 * n
    keys = synth.cisd_like_selected_set(n, na, nb, count, seed=seed)
    s, h, g = _system(n, na, nb, seed=seed, dets=keys)
    Hm = capply.csr(n, h, g, keys)
    th = synth.nqs_theta(V, H, seed, scale=0.3)
    res, th_new, E_after = step.lm_step(keys, n, V, H, th, Hm, mode="C")
    theta = dev(th)
    rc, r, dth, _ = s.step(theta, V, H, m=20, k_keep=4, mode=IRL_MODE_C, ws_flags=_ws(True))
    _check(rc, r, dth, theta, res, th_new, E_after)


def test_connected_exact_psi_gives_zero_update():
    from paper_2601_01437_amd import IRL_MODE_C
    announce("connected: exact psi")
    n, na, nb = 5, 3, 2
    s, h, g = _system(n, na, nb, seed=4)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    psi0 = np.linalg.eigh(Hm)[1][:, 0]
    J = np.random.default_rng(5).normal(size=(keys.size, 30))
    s.set_dtilde(dev(np.concatenate([psi0[:, None], J], axis=1)))
    rc, r, dth, _ = s.step(None, m=20, k_keep=4, flags=1, mode=IRL_MODE_C)
    assert abs(r.lambda_min) <= 1e-12
    assert np.max(np.abs(host(dth))) <= 1e-10


def test_connected_invariant_under_psi_shift():
    """D~ and D~ + psi a^T (derivative columns) give the same eigenvalue and the
    same linearised wavefunction in mode C."""
    from paper_2601_01437_amd import IRL_MODE_C
    announce("connected: psi-shift invariance")
    n, na, nb = 6, 3, 3
    s, h, g = _system(n, na, nb, seed=2)
    keys = space.full_space(n, na, nb)
    V, H = 2 * n, 8
    D = nqs.dtilde(keys, n, V, H, synth.nqs_theta(V, H, 2, scale=0.3))
    psi = D[:, 0]
    D2 = D.copy()
    D2[:, 1:] += np.outer(psi, np.random.default_rng(6).normal(size=D.shape[1] - 1))
    out = []
    for M in (D, D2):
        s.set_dtilde(dev(M))
        rc, r, dth, _ = s.step(None, m=40, k_keep=8, flags=1, mode=IRL_MODE_C)
        assert r.converged == 1
        phi = psi + M[:, 1:] @ host(dth)
        phi /= np.linalg.norm(phi)
        out.append((r.lambda_min, phi * np.sign(phi[np.argmax(np.abs(phi))])))
    Hm = hamiltonian.build(keys, n, h, g)
    normH = np.linalg.norm(lm.solve(D, Hm, mode="C").Hp, 2)
    assert abs(out[0][0] - out[1][0]) <= 1e-10 * normH
    assert np.linalg.norm(out[0][1] - out[1][1]) <= 1e-8


def test_connected_option_errors():
    from paper_2601_01437_amd import IRL_FP32, IRL_MODE_C, IRL_WS_BLOCK, IRL_WS_FP32, IRL_WS_FP64, IrlError
    announce("connected: option errors")
    s, _, _ = _system(5, 2, 2, seed=1)
    theta = dev(synth.nqs_theta(10, 4, 1))
    with pytest.raises(IrlError):                       # FP32 solve
        s.step(theta, 10, 4, m=16, k_keep=2, mode=IRL_MODE_C, precision=IRL_FP32,
               ws_flags=IRL_WS_FP32 | IRL_WS_FP64)
    with pytest.raises(IrlError):                       # block solve
        s.step(theta, 10, 4, m=16, k_keep=2, mode=IRL_MODE_C, block=4,
               ws_flags=IRL_WS_FP64 | IRL_WS_BLOCK)
