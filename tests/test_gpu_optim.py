"""Optimiser comparison baselines through the C ABI (GPU).

Adam (irl_adam_step): each step evaluates the FP64 gradient and applies the
published update; three steps on c1 match the oracle's gradient + Adam step
(theta within 1e-9 relative: the update divides by sqrt(v), so a gradient
component near zero turns the gradient's 1e-12 relative error into an absolute
update error of about lr * 1e-12 / eps) and the energies before each step
within 1e-12 Ha.

Standard Lanczos (irl_step with no restarts and full cycles, Algorithm 2): the
lowest Ritz value of an m-step Krylov space bounds the exact lowest eigenvalue
from above, does not increase with m, and equals it once the space is the whole
(P + 1)-dimensional space."""
import numpy as np
import pytest

import synth
from oracle import hamiltonian, lm, nqs, optim, space
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(n, na, nb, seed=0):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g), h, g


@pytest.mark.parametrize("factored", [False, True])
def test_adam_matches_oracle_c1(c1_problem, factored):
    import torch
    from paper_2601_01437_amd import IRL_WS_FACTORED, IRL_WS_FP64
    announce(f"adam c1 factored={factored}")
    p = c1_problem
    w = p["w"]
    s, _, _ = _system(8, 4, 4)
    fl = IRL_WS_FACTORED if factored else IRL_WS_FP64
    th_ref = p["theta"].copy()
    m_ref = np.zeros(w.P)
    v_ref = np.zeros(w.P)
    th = dev(th_ref)
    m = torch.zeros(w.P, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    opts = dict(lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    for t in range(1, 4):
        Dt = nqs.dtilde(p["keys"], w.n, w.V, w.H, th_ref)
        _, _, E_ref = lm.energy(Dt[:, 0], p["H"])
        g_ref = lm.gradient(Dt, p["H"])
        _, E = s.adam_step(w.V, w.H, th, m, v, t, ws_flags=fl, **opts)
        th_ref, m_ref, v_ref = optim.adam_step(th_ref, g_ref, m_ref, v_ref, t, **opts)
        assert abs(E - E_ref) <= 1e-12
        assert rel_err(host(th), th_ref) <= 1e-9
        assert rel_err(host(m), m_ref) <= 1e-10


def test_adam_argument_errors():
    import torch
    from paper_2601_01437_amd import IrlError
    s, _, _ = _system(5, 2, 2, seed=1)
    th = dev(synth.nqs_theta(10, 4, 1))
    m = torch.zeros(54, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    with pytest.raises(IrlError):
        s.adam_step(10, 4, th, m, v, 0)                 # step count starts at 1
    with pytest.raises(IrlError):
        s.adam_step(10, 4, th, m, v, 1, beta1=1.0)      # beta in [0, 1)
    with pytest.raises(IrlError):
        s.adam_step(10, 4, th, m, v, 1, eps=0.0)        # eps > 0


def test_standard_lanczos_ritz_bounds():
    """n = 4, 2 + 2 electrons (36 determinants), V = 8, H = 4: P + 1 = 45."""
    from paper_2601_01437_amd import IRL_STEP_FULL_CYCLES, IRL_STEP_NO_UPDATE, IRL_WS_FP64
    announce("standard Lanczos Ritz bounds")
    n, na, nb, V, H = 4, 2, 2, 8, 4
    s, h, g = _system(n, na, nb, seed=2)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    th0 = synth.nqs_theta(V, H, 2, scale=0.3)
    Dt = nqs.dtilde(keys, n, V, H, th0)
    ref = lm.solve(Dt, Hm)
    normH = np.linalg.norm(ref.Hp, 2)
    lams = []
    for m in (8, 16, 32, 45):
        rc, r, _, _ = s.step(dev(th0), V, H, m=m, k_keep=1, max_restarts=0,
                             flags=IRL_STEP_FULL_CYCLES | IRL_STEP_NO_UPDATE, ws_flags=IRL_WS_FP64,
                             want_dtheta=False)
        assert r.n_restart == 0 and r.n_apply <= m + 1
        lams.append(r.lambda_min)
    assert all(lam >= ref.lam - 1e-10 * normH for lam in lams)
    assert all(a >= b - 1e-10 * normH for a, b in zip(lams, lams[1:]))
    assert abs(lams[-1] - ref.lam) <= 1e-10 * max(abs(ref.lam), normH)
