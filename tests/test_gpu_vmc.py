"""Sampled (VMC) estimators through the C ABI against the oracle's sampler and
sample means (oracle/vmc.py), on the oracle's own psi and draws:

* the drawn rows equal the orbital-by-orbital sampler's, except where u falls
  within rounding of an interval boundary of the cumulative |psi|^2;
* sampled energy (1e-12 relative), local-energy variance (1e-10), distinct rows
  (exact) and the sampled gradient (1e-10 relative);
* the sampled operator pair, (y_H, y_S) / Z = (<O E_loc O^T> v, <O O^T> v),
  within 1e-10 relative;
* a step on the sampled centred matrix (modes A and P, FP64 and FP32 with the
  FP64 polish, dense copy and factored Jacobian): eigenvalue within 1e-10
  max(|lambda|, ||M||), update within 1e-8, exact energy after the update
  within 1e-12;
* zero variance at an exact eigenvector, inverse-transform monotonicity and
  the statistical error of the energy at 853,776 determinants."""
import math

import numpy as np
import pytest

import synth
from oracle import capply, hamiltonian, lm, nqs, space, vmc
from tests.gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(n, na, nb, seed=0, dets=None):
    from paper_2601_01437_amd import System
    h, g = synth.integrals(n, seed)
    return System(n, na, nb, h, g, dets=dets), h, g


def _check_rows(rows_gpu, rows_ref, psi, u):
    """Equal rows, except at an interval boundary within rounding."""
    c = np.cumsum(psi ** 2)
    bad = np.nonzero(rows_gpu != rows_ref)[0]
    for s in bad:
        lo = min(rows_gpu[s], rows_ref[s])
        assert abs(u[s] * c[-1] - c[lo]) <= 1e-12 * c[-1], (s, rows_gpu[s], rows_ref[s])
    return bad.size


def _problem(kind):
    if kind == "c1":
        w = synth.WORKLOADS["c1"]
        h, g = w.integrals()
        keys = space.full_space(w.n, w.na, w.nb)
        return dict(n=w.n, na=w.na, nb=w.nb, V=w.V, H=w.H, seed=w.seed, keys=keys, dets=None,
                    Hm=hamiltonian.build(keys, w.n, h, g), theta=w.theta())
    n, na, nb, H, count, seed = 12, 4, 4, 40, 3001, 8
    keys = synth.cisd_like_selected_set(n, na, nb, count, seed=seed)
    h, g = synth.integrals(n, seed)
    return dict(n=n, na=na, nb=nb, V=2 * n, H=H, seed=seed, keys=keys, dets=keys,
                Hm=capply.csr(n, h, g, keys), theta=synth.nqs_theta(2 * n, H, seed, scale=0.3))


@pytest.fixture(scope="module", params=["c1", "selected"])
def vmc_case(request):
    p = _problem(request.param)
    Dt = nqs.dtilde(p["keys"], p["n"], p["V"], p["H"], p["theta"])
    psi = Dt[:, 0]
    u = np.random.default_rng(17).random(800)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi, u)
    p.update(name=request.param, Dt=Dt, psi=psi, u=u, rows=rows,
             Eloc=vmc.local_energy(psi, p["Hm"]), O=vmc.log_derivatives(Dt))
    return p


def _gpu_system(p, ws_flags):
    s, _, _ = _system(p["n"], p["na"], p["nb"], seed=p["seed"], dets=p["dets"])
    theta = dev(p["theta"])
    s.evaluate(p["V"], p["H"], theta, ws_flags=ws_flags)
    return s, theta


def test_vmc_draws_and_estimators(vmc_case):
    from paper_2601_01437_amd import IRL_WS_FACTORED
    p = vmc_case
    announce(f"vmc draws and estimators {p['name']}")
    s, _ = _gpu_system(p, IRL_WS_FACTORED)
    out, rows, F = s.vmc_sample(dev(p["u"]), want_rows=True, want_grad=True)
    rows = host(rows)
    assert _check_rows(rows, p["rows"], p["psi"], p["u"]) == 0
    Eloc, O, r = p["Eloc"], p["O"], p["rows"]
    Es = vmc.sampled_energy(r, Eloc)
    _, E_el, _ = lm.energy(p["psi"], p["Hm"])
    assert abs(out.E_sampled - Es) <= 1e-12 * max(1.0, abs(Es))
    assert abs(out.E_exact - E_el) <= 1e-12 * max(1.0, abs(E_el))
    assert abs(out.E_loc_var - vmc.sampled_variance(r, Eloc)) <= 1e-10 * vmc.sampled_variance(r, Eloc)
    assert out.n_unique == np.unique(r).size and out.n_samples == r.size
    assert rel_err(host(F), vmc.sampled_gradient(r, O, Eloc)) <= 1e-10


@pytest.mark.parametrize("factored", [False, True, "gathered"])
def test_vmc_operator_pair(vmc_case, factored):
    from paper_2601_01437_amd import IRL_WS_FACTORED, IRL_WS_FP64, IRL_WS_SAMPLED
    p = vmc_case
    announce(f"vmc operator pair {p['name']} factored={factored}")
    fl = {False: IRL_WS_FP64, True: IRL_WS_FACTORED, "gathered": IRL_WS_FACTORED | IRL_WS_SAMPLED}[factored]
    s, _ = _gpu_system(p, fl)
    out, _, _ = s.vmc_sample(dev(p["u"]))
    Z, _, _ = lm.energy(p["psi"], p["Hm"])
    rng = np.random.default_rng(3)
    for _ in range(2):
        v = rng.normal(size=p["Dt"].shape[1])
        yH, yS = s.apply(dev(v))
        rH, rS = vmc.sampled_pair(p["rows"], p["O"], p["Eloc"], v)
        assert rel_err(host(yH) / Z, rH) <= 1e-10 and rel_err(host(yS) / Z, rS) <= 1e-10
    # block apply of the sampled operator
    from paper_2601_01437_amd import IRL_WS_BLOCK
    if factored is False:
        s2, _ = _gpu_system(p, IRL_WS_FP64 | IRL_WS_BLOCK)
        s2.vmc_sample(dev(p["u"]))
        Vb = rng.normal(size=(3, p["Dt"].shape[1]))
        YH, YS = s2.apply_block(dev(Vb))
        for q in range(3):
            rH, rS = vmc.sampled_pair(p["rows"], p["O"], p["Eloc"], Vb[q])
            assert rel_err(host(YH[q]) / Z, rH) <= 1e-10 and rel_err(host(YS[q]) / Z, rS) <= 1e-10


@pytest.mark.parametrize("variant", ["fp64", "factored", "gathered", "fp32_polish", "mode_p"])
def test_vmc_step(vmc_case, variant):
    from paper_2601_01437_amd import (IRL_FP32, IRL_FP64, IRL_MODE_A, IRL_MODE_P, IRL_STEP_WS_CURRENT,
                                      IRL_WS_FACTORED, IRL_WS_FP32, IRL_WS_FP64, IRL_WS_SAMPLED)
    p = vmc_case
    announce(f"vmc step {p['name']} {variant}")
    fl = {"fp64": IRL_WS_FP64, "factored": IRL_WS_FACTORED, "gathered": IRL_WS_FACTORED | IRL_WS_SAMPLED,
          "fp32_polish": IRL_WS_FP64 | IRL_WS_FP32, "mode_p": IRL_WS_FACTORED | IRL_WS_SAMPLED}[variant]
    mode = IRL_MODE_P if variant == "mode_p" else IRL_MODE_A
    s, theta = _gpu_system(p, fl)
    s.vmc_sample(dev(p["u"]))
    lam, c, dth_ref, M = vmc.solve_sampled(p["rows"], p["O"], p["Eloc"], "P" if mode == IRL_MODE_P else "A")
    normM = np.linalg.norm(M[1:, 1:] if mode == IRL_MODE_P else M, 2)
    rc, r, dth, ritz = s.step(theta, p["V"], p["H"], m=20, k_keep=4, mode=mode, ws_flags=fl,
                              flags=IRL_STEP_WS_CURRENT, want_ritz=True,
                              want_dtheta=mode == IRL_MODE_A,
                              precision=IRL_FP32 if variant == "fp32_polish" else IRL_FP64)
    assert r.converged == 1
    assert abs(r.E_before - vmc.sampled_energy(p["rows"], p["Eloc"])) <= 1e-12 * max(1.0, abs(r.E_before))
    assert abs(r.lambda_min - lam) <= 1e-10 * max(abs(lam), normM)
    assert abs(abs(host(ritz) @ c) - 1.0) <= 1e-9
    if mode == IRL_MODE_A:
        assert rel_err(host(dth), dth_ref) <= 1e-8
        th_new = p["theta"] + dth_ref
        psi_new = nqs.dtilde(p["keys"], p["n"], p["V"], p["H"], th_new)[:, 0]
        _, E_new, _ = lm.energy(psi_new, p["Hm"])
        assert abs(r.E_after - E_new) <= 1e-12 * max(1.0, abs(E_new))
        assert rel_err(host(theta), th_new) <= 1e-10


def test_vmc_zero_variance_at_exact_eigenvector():
    announce("vmc: exact psi")
    n, na, nb = 5, 3, 2
    s, h, g = _system(n, na, nb, seed=4)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g).toarray()
    e, U = np.linalg.eigh(Hm)
    J = np.random.default_rng(5).normal(size=(keys.size, 30))
    s.set_dtilde(dev(np.concatenate([U[:, :1], J], axis=1)))
    out, _, F = s.vmc_sample(dev(np.random.default_rng(6).random(4000)), want_grad=True)
    assert abs(out.E_sampled - e[0]) <= 1e-10 and out.E_loc_var <= 1e-18
    assert np.max(np.abs(host(F))) <= 1e-9
    # E_loc = E on every drawn row: the sampled centred matrix vanishes (its
    # eigenvector is then arbitrary, so only the eigenvalue is fixed)
    rc, r, _, _ = s.step(None, m=20, k_keep=4, flags=1, want_dtheta=False)
    assert abs(r.lambda_min) <= 1e-9


def test_vmc_c2_scale_properties():
    """853,776 determinants, 2^17 draws: rows are monotone in u (inverse
    transform), the distinct rows match the reported count, the sampled energy is
    within five standard errors of the exact one, and a sampled step converges to
    the same eigenvalue with the products over every row and over the gathered
    drawn rows only."""
    import torch
    from paper_2601_01437_amd import IRL_STEP_WS_CURRENT, IRL_WS_FACTORED, IRL_WS_SAMPLED, System
    announce("vmc c2 scale")
    w = synth.WORKLOADS["c2"]
    h, g = w.integrals()
    s = System(w.n, w.na, w.nb, h, g)
    u = np.random.default_rng(9).random(1 << 17)
    lams = []
    for fl in (IRL_WS_FACTORED, IRL_WS_FACTORED | IRL_WS_SAMPLED):
        theta = dev(w.theta())
        s.evaluate(w.V, w.H, theta, ws_flags=fl)
        out, rows, F = s.vmc_sample(dev(u), want_rows=True, want_grad=True)
        rows = host(rows)
        order = np.argsort(u, kind="stable")
        assert np.all(np.diff(rows[order]) >= 0)
        assert out.n_unique == np.unique(rows).size
        assert abs(out.E_sampled - out.E_exact) <= 5.0 * math.sqrt(out.E_loc_var / u.size)
        assert np.all(np.isfinite(host(F)))
        rc, r, _, _ = s.step(theta, w.V, w.H, m=40, k_keep=10, ws_flags=fl,
                             flags=IRL_STEP_WS_CURRENT, want_dtheta=False)
        assert r.converged == 1 and r.lambda_min <= 0.0 and np.isfinite(r.E_after)
        lams.append((r.lambda_min, r.norm_T))
    assert abs(lams[0][0] - lams[1][0]) <= 1e-10 * max(abs(lams[0][0]), lams[0][1])
    torch.cuda.synchronize()


def test_vmc_errors():
    from paper_2601_01437_amd import IRL_MODE_C, IRL_STEP_WS_CURRENT, IRL_WS_FP32, IRL_WS_FP64, IrlError, System
    import torch
    announce("vmc errors")
    s, _, _ = _system(5, 2, 2, seed=1)
    theta = dev(synth.nqs_theta(10, 4, 1))
    u = dev(np.random.default_rng(1).random(64))
    with pytest.raises(IrlError):                   # nothing evaluated yet
        s.ws = torch.empty(16, dtype=torch.uint8, device="cuda")
        s.vmc_sample(u)
    s.ws = None
    s.evaluate(10, 4, theta, ws_flags=IRL_WS_FP32)
    with pytest.raises(IrlError):                   # no FP64 Jacobian for the gradient
        s.vmc_sample(u)
    s.evaluate(10, 4, theta, ws_flags=IRL_WS_FP64)
    with pytest.raises(IrlError):                   # no samples
        s.vmc_sample(u[:0])
    s.vmc_sample(u)
    with pytest.raises(IrlError):                   # mode C on sampled estimators
        s.step(theta, 10, 4, m=16, k_keep=2, mode=IRL_MODE_C, ws_flags=IRL_WS_FP64, flags=IRL_STEP_WS_CURRENT)


def test_vmc_edge_draws():
    """One draw; u at the ends of [0, 1) and outside it (clamped: below 0 and NaN
    act as 0, 1 and above as the largest u below 1); rows with psi = 0 are never
    drawn, even where u lands exactly on their (empty) interval."""
    from paper_2601_01437_amd import IRL_WS_FP64
    announce("vmc edge draws")
    n, na, nb = 5, 2, 2
    s, h, g = _system(n, na, nb, seed=7)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    rng = np.random.default_rng(8)
    psi = rng.normal(size=keys.size)
    zero = [0, 1, 17, keys.size - 1]          # first, last and interior rows with psi = 0
    psi[zero] = 0.0
    D = np.concatenate([psi[:, None], rng.normal(size=(keys.size, 12))], axis=1)
    s.set_dtilde(dev(D), ws_flags=IRL_WS_FP64)
    nz = np.nonzero(psi)[0]
    below_one = np.nextafter(1.0, 0.0)
    # one draw at u = 0: the first row with psi != 0, and E is its local energy
    out, rows, _ = s.vmc_sample(dev(np.array([0.0])), want_rows=True)
    Eloc = vmc.local_energy(psi, Hm)
    assert host(rows)[0] == nz[0] and out.n_unique == 1
    assert abs(out.E_sampled - Eloc[nz[0]]) <= 1e-12 * max(1.0, abs(Eloc[nz[0]]))
    u = np.array([0.0, below_one, -0.25, np.nan, 1.0, 7.5, -np.inf, np.inf])
    out, rows, _ = s.vmc_sample(dev(u), want_rows=True)
    r = host(rows)
    assert r[0] == nz[0]
    assert r[1] == nz[-1]
    assert r[2] == r[0] and r[3] == r[0] and r[6] == r[0]
    assert r[4] == r[1] and r[5] == r[1] and r[7] == r[1]
    # inner boundaries: u exactly at the cumulative weight of a zero row's start
    c = np.cumsum(psi ** 2)
    ub = np.array([c[16] / c[-1], c[17] / c[-1], 0.5])
    out, rows, _ = s.vmc_sample(dev(ub), want_rows=True)
    r = host(rows)
    assert not np.isin(r, zero).any()
    ref = vmc.sample_autoregressive(keys, n, na, nb, psi, ub)
    assert _check_rows(r, ref, psi, ub) <= 3
