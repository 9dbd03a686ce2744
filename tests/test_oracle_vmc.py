"""Pins for the oracle's sampled (VMC) estimators and its orbital-by-orbital
sampler.

* the sequential sampler with exact conditionals (Eqs.
  autoregressive_factorization, constraint) draws the same rows as inverse
  transform sampling of |psi|^2 in ascending key order (numpy's cumsum and
  searchsorted), except where u lies within rounding of an interval boundary;
* its frequencies pass a chi-square test against |psi|^2 / Z, and rows with
  psi = 0 are never drawn;
* a sample multiset exactly proportional to |psi|^2 gives the exact energy
  psi^T H psi / Z and the exact gradient 2 D~^T (H psi - E psi) / Z;
* an exact eigenvector gives E_loc = E on every row, so the sampled centred
  matrix, the gradient and the eigenvalue vanish (zero-variance principle);
* Eq. matrix_vec_prod summed sample by sample equals the matrix form, and Eq.
  centered_hamiltonian's two terms combine to it;
* the sampled energy lies within five standard errors of the exact one;
* a planted mistake (the orbitals sampled in the opposite order) is caught.
"""
import math

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import hamiltonian, lm, nqs, space, vmc


@pytest.fixture(scope="module")
def sys6():
    n, na, nb, V, H = 6, 3, 2, 12, 6
    h, g = synth.integrals(n, 3)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    theta = synth.nqs_theta(V, H, 3, scale=0.4)
    Dt = nqs.dtilde(keys, n, V, H, theta)
    return dict(n=n, na=na, nb=nb, keys=keys, Hm=Hm, Dt=Dt)


def _inverse_transform(psi, u):
    c = np.cumsum(psi ** 2)
    return np.searchsorted(c, u * c[-1], side="right"), c


def test_sampler_matches_inverse_transform(sys6):
    p = sys6
    psi = p["Dt"][:, 0]
    u = np.random.default_rng(0).random(1500)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi, u)
    ref, c = _inverse_transform(psi, u)
    bad = np.nonzero(rows != ref)[0]
    for s in bad:                       # only at a boundary, within rounding
        lo = min(rows[s], ref[s])
        assert abs(rows[s] - ref[s]) == 1
        assert abs(u[s] * c[-1] - c[lo]) <= 1e-12 * c[-1]
    assert bad.size <= 2


def test_planted_orbital_order_is_caught(sys6):
    """Sampling the orbitals in the opposite order still draws from |psi|^2 but
    maps u to other rows: the inverse-transform comparison catches it."""
    p = sys6
    psi = p["Dt"][:, 0]
    u = np.random.default_rng(0).random(300)
    wrong = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi, u,
                                      order=vmc.spin_orbital_order(p["n"])[::-1])
    ref, _ = _inverse_transform(psi, u)
    assert np.mean(wrong != ref) > 0.5


def test_sampler_frequencies_and_zero_rows():
    n, na, nb = 4, 2, 1
    keys = space.full_space(n, na, nb)
    rng = np.random.default_rng(1)
    psi = rng.normal(size=keys.size)
    psi[[3, 10]] = 0.0
    u = rng.random(6000)
    rows = vmc.sample_autoregressive(keys, n, na, nb, psi, u)
    counts = np.bincount(rows, minlength=keys.size)
    assert counts[3] == 0 and counts[10] == 0
    p = psi ** 2 / np.sum(psi ** 2)
    nz = p > 0
    chi2 = np.sum((counts[nz] - u.size * p[nz]) ** 2 / (u.size * p[nz]))
    assert chi2 <= scipy.stats.chi2.ppf(0.999, nz.sum() - 1)


def test_samples_respect_electron_counts(sys6):
    p = sys6
    u = np.random.default_rng(2).random(200)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], p["Dt"][:, 0], u)
    for k in p["keys"][rows]:
        a, b = space.split(k)
        assert bin(a).count("1") == p["na"] and bin(b).count("1") == p["nb"]


def test_exact_multiset_gives_exact_energy_and_gradient(sys6):
    """psi_r^2 = k_r (small integers) and row r repeated k_r times: the sample
    mean over the multiset is the |psi|^2-weighted sum."""
    p = sys6
    Hm = p["Hm"]
    k = np.random.default_rng(4).integers(1, 5, size=p["keys"].size)
    psi = np.sqrt(k.astype(np.float64))
    J = p["Dt"][:, 1:]
    Dt = np.concatenate([psi[:, None], J], axis=1)
    rows = np.repeat(np.arange(k.size), k)
    Eloc = vmc.local_energy(psi, Hm)
    O = vmc.log_derivatives(Dt)
    Z, E_el, _ = lm.energy(psi, Hm)
    assert abs(vmc.sampled_energy(rows, Eloc) - E_el) <= 1e-12 * max(1.0, abs(E_el))
    g = lm.gradient(Dt, Hm)
    assert np.max(np.abs(vmc.sampled_gradient(rows, O, Eloc) - g)) <= 1e-11 * np.max(np.abs(g))
    M = vmc.sampled_matrix(rows, O, Eloc)
    assert abs(M[0, 0]) <= 1e-12 * np.max(np.abs(M))
    assert np.max(np.abs(2.0 * M[1:, 0] - g)) <= 1e-11 * np.max(np.abs(g))


def test_zero_variance_at_an_exact_eigenvector(sys6):
    p = sys6
    Hm = p["Hm"]
    e, U = np.linalg.eigh(Hm.toarray())
    psi0 = U[:, 0]
    J = p["Dt"][:, 1:]
    Dt = np.concatenate([psi0[:, None], J], axis=1)
    Eloc = vmc.local_energy(psi0, Hm)
    u = np.random.default_rng(5).random(500)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi0, u)
    O = vmc.log_derivatives(Dt)
    assert abs(vmc.sampled_energy(rows, Eloc) - e[0]) <= 1e-10
    assert vmc.sampled_variance(rows, Eloc) <= 1e-18
    lam, c, dth, M = vmc.solve_sampled(rows, O, Eloc)
    scale = np.max(np.abs(O[rows])) ** 2
    assert np.max(np.abs(M)) <= 1e-9 * scale
    assert abs(lam) <= 1e-9 * scale


def test_mvp_sample_by_sample(sys6):
    p = sys6
    Dt, Hm = p["Dt"], p["Hm"]
    psi = Dt[:, 0]
    u = np.random.default_rng(6).random(300)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi, u)
    Eloc = vmc.local_energy(psi, Hm)
    O = vmc.log_derivatives(Dt)
    v = np.random.default_rng(7).normal(size=Dt.shape[1])
    E = vmc.sampled_energy(rows, Eloc)
    acc = [[] for _ in range(Dt.shape[1])]
    for r in rows:                       # Eq. matrix_vec_prod, one sample at a time
        o = Dt[r] / psi[r]
        s = (Eloc[r] - E) * math.fsum((o * v).tolist())
        for i in range(Dt.shape[1]):
            acc[i].append(o[i] * s)
    ref = np.array([math.fsum(a) for a in acc]) / rows.size
    y = vmc.sampled_mvp(rows, O, Eloc, v)
    assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert np.max(np.abs(vmc.sampled_matrix(rows, O, Eloc) @ v - ref)) <= 1e-11 * np.max(np.abs(ref))
    yH, yS = vmc.sampled_pair(rows, O, Eloc, v)
    assert np.max(np.abs(yH - E * yS - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_sampled_energy_statistical_error(sys6):
    p = sys6
    Dt, Hm = p["Dt"], p["Hm"]
    psi = Dt[:, 0]
    u = np.random.default_rng(8).random(3000)
    rows = vmc.sample_autoregressive(p["keys"], p["n"], p["na"], p["nb"], psi, u)
    Eloc = vmc.local_energy(psi, Hm)
    _, E_el, _ = lm.energy(psi, Hm)
    Es = vmc.sampled_energy(rows, Eloc)
    sigma = math.sqrt(vmc.sampled_variance(rows, Eloc) / rows.size)
    assert abs(Es - E_el) <= 5.0 * sigma
