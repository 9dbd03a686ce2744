"""Pins for the oracle's connected-basis mode (mode C).

Mode C is mode A's identity-metric problem in the connected tangent basis: the
derivative columns d_i psi projected against psi (Methods, "From SR to a Stable
Eigenvalue Problem": H_eff in connected-correlation form).  What fixes it:

* the connected columns are orthogonal to psi: S~_c[0, 1:] = 0, S~_c[0, 0] = 1;
* the basis, and therefore lambda and the linearised wavefunction, does not
  change when any multiple of psi is added to any derivative column (mode A's
  does, which the test checks too, so a mode C that silently ran mode A fails);
* derivatives already orthogonal to psi make mode C identical to mode A;
* an exact eigenvector as psi gives lambda = 0 and a zero update;
* the exact generalised problem spans the same space in either basis: its
  lowest eigenvalue and linearised wavefunction agree between the raw and the
  connected basis (with the connected update's psi coefficient c_0 - sigma.c);
* a planted mistake (the projection's sign flipped) breaks the invariance.
"""
import numpy as np
import pytest

import synth
from oracle import hamiltonian, lm, nqs, space


@pytest.fixture(scope="module")
def small():
    n, na, nb, V, H = 6, 3, 3, 12, 8
    h, g = synth.integrals(n, 2)
    keys = space.full_space(n, na, nb)
    Hm = hamiltonian.build(keys, n, h, g)
    theta = synth.nqs_theta(V, H, 2, scale=0.3)
    Dt = nqs.dtilde(keys, n, V, H, theta)
    e_exact, U = np.linalg.eigh(Hm.toarray())
    return dict(Hm=Hm, Dt=Dt, e=e_exact, psi0=U[:, 0])


def _direction(psi, J, dtheta):
    """Unit linearised wavefunction psi + J dtheta, sign fixed by its largest entry."""
    phi = psi + J @ dtheta
    phi = phi / np.linalg.norm(phi)
    return phi * np.sign(phi[np.argmax(np.abs(phi))])


def test_connected_columns_orthogonal_to_psi(small):
    Dc, sigma = lm.connected_basis(small["Dt"])
    _, Sc = lm.dense_matrices(Dc, small["Hm"])
    assert abs(Sc[0, 0] - 1.0) <= 1e-14
    assert np.max(np.abs(Sc[0, 1:])) <= 1e-13 * max(1.0, np.max(np.abs(Sc)))
    psi = small["Dt"][:, 0]
    assert np.allclose(sigma, small["Dt"][:, 1:].T @ psi / (psi @ psi), rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", [0, 1])
def test_invariant_under_adding_psi_to_derivatives(small, seed):
    Dt, Hm = small["Dt"], small["Hm"]
    psi = Dt[:, 0]
    a = np.random.default_rng(seed).normal(size=Dt.shape[1] - 1)
    Dt2 = Dt.copy()
    Dt2[:, 1:] += np.outer(psi, a)
    r1 = lm.solve(Dt, Hm, mode="C")
    r2 = lm.solve(Dt2, Hm, mode="C")
    scale = max(abs(r1.lam), np.linalg.norm(r1.Hp, 2))
    assert abs(r1.lam - r2.lam) <= 1e-11 * scale
    d1 = _direction(psi, Dt[:, 1:], r1.dtheta)
    d2 = _direction(psi, Dt2[:, 1:], r2.dtheta)
    assert np.linalg.norm(d1 - d2) <= 1e-9
    # mode A is not invariant under the same change
    a1 = lm.solve(Dt, Hm, mode="A")
    a2 = lm.solve(Dt2, Hm, mode="A")
    assert abs(a1.lam - a2.lam) > 1e-6 * scale


def test_reduces_to_mode_a_for_orthogonal_derivatives(small):
    Dt, Hm = small["Dt"], small["Hm"]
    Dc, _ = lm.connected_basis(Dt)
    rc = lm.solve(Dc, Hm, mode="C")
    ra = lm.solve(Dc, Hm, mode="A")
    assert abs(rc.lam - ra.lam) <= 1e-13 * max(1.0, abs(ra.lam))
    assert np.max(np.abs(rc.dtheta - ra.dtheta)) <= 1e-9 * max(1.0, np.max(np.abs(ra.dtheta)))


def test_exact_psi_gives_zero_update(small):
    Hm, psi0 = small["Hm"], small["psi0"]
    J = np.random.default_rng(3).normal(size=(psi0.size, 40))
    Dt = np.concatenate([psi0[:, None], J], axis=1)
    r = lm.solve(Dt, Hm, mode="C")
    assert abs(r.lam) <= 1e-12
    assert np.max(np.abs(r.dtheta)) <= 1e-10


def test_exact_metric_same_space_in_either_basis(small):
    """The generalised problem H~' c = lambda S~ c only sees span(D~), which the
    projection does not change.  A random tall J keeps S~ well conditioned."""
    Hm = small["Hm"]
    psi = small["Dt"][:, 0]
    J = np.random.default_rng(4).normal(size=(psi.size, 30))
    Dt = np.concatenate([psi[:, None], J], axis=1)
    rg = lm.solve(Dt, Hm, mode="G")
    Dc, sigma = lm.connected_basis(Dt)
    rgc = lm.solve(Dc, Hm, mode="G")
    assert abs(rg.lam - rgc.lam) <= 1e-11 * max(1.0, abs(rg.lam))
    dth_c = lm.connected_update(rgc.c, sigma)
    assert np.linalg.norm(_direction(psi, J, rg.dtheta) - _direction(psi, J, dth_c)) <= 1e-9


def test_planted_sign_error_breaks_invariance(small):
    Dt, Hm = small["Dt"], small["Hm"]
    psi = Dt[:, 0]
    Z = psi @ psi

    def wrong(D):                      # projection with the sign flipped
        sig = D[:, 1:].T @ psi / Z
        Dw = D.copy()
        Dw[:, 1:] = D[:, 1:] + np.outer(psi, sig)
        return lm.solve(Dw, Hm, mode="A").lam

    Dt2 = Dt.copy()
    Dt2[:, 1:] += np.outer(psi, np.random.default_rng(5).normal(size=Dt.shape[1] - 1))
    assert abs(wrong(Dt) - wrong(Dt2)) > 1e-6 * abs(wrong(Dt))


def test_rank_two_form_equals_projection(small):
    """The connected centred matrix is the raw one with H_eff corrected by
    -(g sigma^T + sigma g^T) / 2 and the psi row and column unchanged (the form a
    matrix-free apply evaluates from the raw operator pair, g and sigma)."""
    Dt, Hm = small["Dt"], small["Hm"]
    ra = lm.solve(Dt, Hm, mode="A")
    rc = lm.solve(Dt, Hm, mode="C")
    _, sigma = lm.connected_basis(Dt)
    half_g = ra.Hp[1:, 0]
    Hc = ra.Hp.copy()
    Hc[1:, 1:] -= np.outer(half_g, sigma) + np.outer(sigma, half_g)
    assert np.max(np.abs(Hc - rc.Hp)) <= 1e-12 * np.max(np.abs(ra.Hp))
