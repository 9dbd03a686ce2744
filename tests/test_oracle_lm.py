"""Pins for the oracle's LM matrices, centring, eigenproblem and update.

* operator identities of the raw pair (y_H, y_S);
* D~ = I reduces H~ to the Hamiltonian: mode A gives lambda + E = E_exact;
* an exact eigenvector as psi gives g = 0, lambda = 0, dtheta = 0;
* a square full-rank D~ makes the generalised problem exact: lambda + E = E_exact;
* ARPACK's implicitly restarted Lanczos (scipy eigsh) on H~' gives the same
  lowest eigenvalue as the dense solver;
* g = 2 H~'[1:, 0] equals a central finite difference of E(theta);
* mode G's lambda equals E_new - E for the linearised wavefunction;
* planted mistakes (no centring) are caught.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import hamiltonian, lm, nqs, space, step


@pytest.fixture(scope="module")
def small():
    n, na, nb, V, H = 6, 3, 3, 12, 8
    h, g = synth.integrals(n, 1)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    theta = synth.nqs_theta(V, H, 1, scale=0.3)
    Dt = nqs.dtilde(keys, n, V, H, theta)
    e_exact, psi0 = np.linalg.eigh(Hm.toarray())
    return dict(n=n, V=V, H=H, keys=keys, Hm=Hm, theta=theta, Dt=Dt, e=e_exact, psi0=psi0[:, 0])


def test_operator_identities(small):
    Dt, Hm = small["Dt"], small["Hm"]
    rng = np.random.default_rng(0)
    v, u = rng.normal(size=Dt.shape[1]), rng.normal(size=Dt.shape[1])
    yH, yS = lm.apply_lm_operator(Dt, Hm, v)
    uH, uS = lm.apply_lm_operator(Dt, Hm, u)
    assert abs(v @ yS - np.linalg.norm(Dt @ v) ** 2) < 1e-10 * abs(v @ yS)
    assert abs(u @ yH - v @ uH) < 1e-10 * abs(u @ yH)
    e0 = np.zeros(Dt.shape[1])
    e0[0] = 1.0
    yH, yS = lm.apply_lm_operator(Dt, Hm, e0)
    Z, E_el, _ = lm.energy(Dt[:, 0], Hm)
    assert abs(yS[0] - Z) < 1e-12 * Z
    assert abs(yH[0] / yS[0] - E_el) < 1e-12


def test_identity_dtilde_reduces_to_ed(small):
    Hm, e = small["Hm"], small["e"]
    N = Hm.shape[0]
    Dt = np.eye(N)
    Ht, St = lm.dense_matrices(Dt, Hm)
    assert np.array_equal(St, np.eye(N))
    assert np.max(np.abs(Ht - Hm.toarray())) < 1e-14
    res = lm.solve(Dt, Hm, mode="A")
    assert abs(res.E - Hm[0, 0]) < 1e-14
    assert abs(res.lam + res.E - e[0]) < 1e-11


def test_exact_psi_gives_zero_update(small):
    Hm, psi0 = small["Hm"], small["psi0"]
    rng = np.random.default_rng(3)
    Dt = np.concatenate([psi0[:, None], rng.normal(size=(psi0.size, 40))], axis=1)
    Ht, St = lm.dense_matrices(Dt, Hm)
    Z, E_el, _ = lm.energy(psi0, Hm)
    g = 2.0 * lm.centred(Ht, St, E_el)[1:, 0]
    assert np.max(np.abs(g)) < 1e-12
    assert np.max(np.abs(lm.gradient(Dt, Hm))) < 1e-12
    res = lm.solve(Dt, Hm, mode="A")
    assert abs(res.lam) < 1e-12
    assert np.max(np.abs(res.dtheta)) < 1e-12


def test_planted_missing_centring_is_caught(small, monkeypatch):
    monkeypatch.setattr(lm, "centred", lambda Ht, St, E: 0.5 * (Ht + Ht.T))
    Hm, psi0 = small["Hm"], small["psi0"]
    rng = np.random.default_rng(3)
    Dt = np.concatenate([psi0[:, None], rng.normal(size=(psi0.size, 40))], axis=1)
    res = lm.solve(Dt, Hm, mode="A")
    assert abs(res.lam) > 1e-3


def test_square_full_rank_generalised_is_exact(small):
    Hm, e = small["Hm"], small["e"]
    N = Hm.shape[0]
    rng = np.random.default_rng(4)
    Dt = rng.normal(size=(N, N))
    res = lm.solve(Dt, Hm, mode="G")
    assert abs(res.lam + res.E - e[0]) < 1e-9


def test_arpack_irl_agrees_with_dense(small):
    res = lm.solve(small["Dt"], small["Hm"], mode="A")
    Hp = res.Hp
    op = spla.LinearOperator(Hp.shape, matvec=lambda x: Hp @ x, dtype=np.float64)
    lam = spla.eigsh(op, k=1, which="SA", ncv=20, tol=1e-13)[0][0]
    assert abs(lam - res.lam) <= 1e-10 * max(abs(res.lam), np.linalg.norm(Hp, 2))


def test_gradient_matches_finite_difference(small):
    n, V, H, keys, Hm, theta = (small[k] for k in ("n", "V", "H", "keys", "Hm", "theta"))
    res = lm.solve(small["Dt"], Hm, mode="A")
    g = 2.0 * res.Hp[1:, 0]
    assert np.allclose(g, lm.gradient(small["Dt"], Hm), rtol=0, atol=1e-12 * np.abs(g).max())

    def E(t):
        psi, _ = nqs.psi_and_jacobian(keys, n, V, H, t)
        return lm.energy(psi, Hm)[2]

    hstep = 1e-5
    for i in list(range(0, theta.size, 7)) + [theta.size - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += hstep
        tm[i] -= hstep
        fd = (E(tp) - E(tm)) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, np.abs(g).max())


def test_generalised_lambda_is_predicted_decrease(small):
    Dt, Hm = small["Dt"], small["Hm"]
    res = lm.solve(Dt, Hm, mode="G")
    psi_new = Dt[:, 0] + Dt[:, 1:] @ res.dtheta
    _, E_new, _ = lm.energy(psi_new, Hm)
    assert abs(res.lam - (E_new - res.E)) < 1e-9


def test_mode_a_is_augmented_hessian_step(small):
    res = lm.solve(small["Dt"], small["Hm"], mode="A")
    Heff, g = res.Hp[1:, 1:], 2.0 * res.Hp[1:, 0]
    v = res.dtheta
    assert abs(res.lam - 0.5 * g @ v) < 1e-9 * max(1.0, abs(res.lam))
    r = Heff @ v - res.lam * v + 0.5 * g
    assert np.linalg.norm(r) < 1e-8 * max(1.0, np.linalg.norm(Heff @ v))
    assert res.lam <= 1e-14                   # c = e_0 gives 0, so the minimum is <= 0


def test_mode_p_is_heff_lowest(small):
    res = lm.solve(small["Dt"], small["Hm"], mode="P")
    resA = lm.solve(small["Dt"], small["Hm"], mode="A")
    assert abs(res.lam - np.linalg.eigvalsh(resA.Hp[1:, 1:])[0]) < 1e-12 * np.linalg.norm(resA.Hp)
    # interlacing: the bordered matrix's lowest eigenvalue is below H_eff's
    assert resA.lam <= res.lam + 1e-12


def test_c1_step_runs(c1_problem):
    p = c1_problem
    w = p["w"]
    res, th_new, E_after = step.lm_step(p["keys"], w.n, w.V, w.H, p["theta"], p["H"])
    assert res.Hp.shape == (w.P + 1, w.P + 1)
    assert np.max(np.abs(res.Hp - res.Hp.T)) == 0.0
    s = np.linalg.eigvalsh(res.St)
    assert s[0] >= -1e-12 * s[-1]                  # S~ is positive semidefinite
    assert np.isfinite(E_after)


def test_trajectory_towards_fci_small():
    """End-to-end report on a tiny system (4 orbitals, 2+2 electrons, 36
    determinants, V = 8, H = 8): consecutive mode-A steps lower the energy
    towards the exact ground state.  Reported, gated only on a decrease; a
    shallow network may stop short of E_FCI at a local minimum."""
    import scipy.sparse.linalg  # noqa: F401
    from oracle import hamiltonian, space, step
    import synth
    n, na, nb, V, H = 4, 2, 2, 8, 8
    h, g = synth.integrals(n, 11)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    e_fci = np.linalg.eigvalsh(Hm.toarray())[0]
    theta = synth.nqs_theta(V, H, 11, scale=0.3)
    energies, lams, _ = step.trajectory(keys, n, V, H, theta, Hm, steps=12)
    print(f"E - E_FCI per step: {np.array2string(energies - e_fci, precision=3)}")
    assert np.all(energies >= e_fci - 1e-10)          # variational
    assert energies[-1] < energies[0]
    assert energies[-1] - e_fci < 0.5 * (energies[0] - e_fci)
    assert np.all(lams <= 1e-12)                       # mode A: predicted decrease is never positive


@pytest.mark.parametrize("chunk", [7, 333, 100_000])
def test_streamed_evaluation_equals_dense(c1_problem, chunk):
    """The row-chunked evaluation (used for sets whose D~ does not fit in host
    memory) gives the dense definitions' Z, E, gradient and operator pairs on
    c1, including chunk sizes that leave a ragged last chunk and one chunk."""
    from oracle import capply
    p = c1_problem
    w = p["w"]
    Dt = nqs.dtilde(p["keys"], w.n, w.V, w.H, p["theta"])
    rng = np.random.default_rng(8)
    vs = [rng.normal(size=w.P + 1) for _ in range(2)]
    happ = lambda x: capply.apply(w.n, p["h"], p["g"], p["keys"], x)
    Z, E_el, g, pairs = lm.streamed_evaluation(p["keys"], w.n, w.V, w.H, p["theta"], happ, vs,
                                               chunk=chunk)
    Zd, Ed, _ = lm.energy(Dt[:, 0], p["H"])
    gd = lm.gradient(Dt, p["H"])
    assert abs(Z - Zd) <= 1e-13 * Zd and abs(E_el - Ed) <= 1e-13
    assert np.linalg.norm(g - gd) <= 1e-12 * np.linalg.norm(gd)
    for v, (yH, yS) in zip(vs, pairs):
        rH, rS = lm.apply_lm_operator(Dt, p["H"], v)
        assert np.linalg.norm(yH - rH) <= 1e-12 * np.linalg.norm(rH)
        assert np.linalg.norm(yS - rS) <= 1e-12 * np.linalg.norm(rS)


def test_streamed_evaluation_identities_and_fd(small):
    """Independent of the dense functions: v = e_0 gives y_S[0] = Z and
    y_H[0] / y_S[0] = E; the gradient matches a central finite difference of
    E(theta); v^T y_S = |D~ v|^2."""
    n, V, H, keys, Hm, theta = (small[k] for k in ("n", "V", "H", "keys", "Hm", "theta"))
    P = V * H + H + V
    e0 = np.zeros(P + 1)
    e0[0] = 1.0
    v = np.random.default_rng(3).normal(size=P + 1)
    Z, E_el, g, pairs = lm.streamed_evaluation(keys, n, V, H, theta, lambda x: Hm @ x, [e0, v], chunk=50)
    (yH0, yS0), (yH, yS) = pairs
    assert abs(yS0[0] - Z) <= 1e-13 * Z and abs(yH0[0] / yS0[0] - E_el) <= 1e-12
    assert abs(v @ yS - np.linalg.norm(small["Dt"] @ v) ** 2) <= 1e-11 * abs(v @ yS)

    def E(t):
        return lm.streamed_evaluation(keys, n, V, H, t, lambda x: Hm @ x, [], chunk=50)[1]

    hstep = 1e-5
    for i in list(range(0, P, 11)) + [P - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += hstep
        tm[i] -= hstep
        assert abs((E(tp) - E(tm)) / (2 * hstep) - g[i]) <= 1e-7 * max(1.0, np.abs(g).max())
