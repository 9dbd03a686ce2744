"""Pins for the oracle network: occupations from keys, a closed-form special
case, the Jacobian against torch.autograd (CPU, float64) and against central
finite differences of the amplitude."""
import numpy as np
import pytest
import torch

import synth
from oracle import nqs, space


def test_occupations_from_key():
    n = 6
    key = synth.key_of(0b000101, 0b110000)
    x = nqs.occupations(np.array([key], dtype=np.uint64), n)[0]
    assert x.tolist() == [1, 0, 1, 0, 0, 0] + [0, 0, 0, 0, 1, 1]


def test_closed_form_special_cases():
    n, V, H = 4, 8, 5
    keys = space.full_space(n, 2, 1)
    x = nqs.occupations(keys, n)
    a = np.arange(1, V + 1, dtype=float)
    theta = np.concatenate([a, np.zeros(H), np.zeros(H * V)])
    psi, J = nqs.psi_and_jacobian(keys, n, V, H, theta)
    assert np.array_equal(psi, x @ a)                     # tanh(0) = 0
    assert np.array_equal(J[:, V:V + H], np.ones((keys.size, H)))
    b = np.full(H, 0.3)
    theta = np.concatenate([np.zeros(V), b, np.zeros(H * V)])
    psi, _ = nqs.psi_and_jacobian(keys, n, V, H, theta)
    assert np.allclose(psi, H * np.tanh(0.3), rtol=0, atol=1e-15)


def _torch_psi(x, theta, V, H):
    a = theta[:V]
    b = theta[V:V + H]
    W = theta[V + H:].reshape(H, V)
    return x @ a + torch.tanh(x @ W.T + b).sum(dim=1)


@pytest.mark.parametrize("n,na,nb,H,seed", [(4, 2, 2, 3, 0), (8, 4, 4, 16, 0)])
def test_jacobian_vs_autograd(n, na, nb, H, seed):
    V = 2 * n
    keys = space.full_space(n, na, nb)[:300]
    theta = synth.nqs_theta(V, H, seed, scale=0.3)
    psi, J = nqs.psi_and_jacobian(keys, n, V, H, theta)
    x = torch.from_numpy(nqs.occupations(keys, n))
    th = torch.from_numpy(theta.copy())
    Jt = torch.autograd.functional.jacobian(lambda t: _torch_psi(x, t, V, H), th)
    assert np.max(np.abs(Jt.numpy() - J)) < 1e-14
    assert np.max(np.abs(_torch_psi(x, th, V, H).numpy() - psi)) < 1e-14


def test_jacobian_vs_finite_differences():
    n, V, H = 5, 10, 4
    keys = space.full_space(n, 2, 3)
    theta = synth.nqs_theta(V, H, 3, scale=0.5)
    _, J = nqs.psi_and_jacobian(keys, n, V, H, theta)
    step = 1e-6
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += step
        tm[i] -= step
        fd = (nqs.psi_and_jacobian(keys, n, V, H, tp)[0] - nqs.psi_and_jacobian(keys, n, V, H, tm)[0]) / (2 * step)
        assert np.max(np.abs(fd - J[:, i])) < 1e-8


def test_planted_transposed_weight_is_caught(monkeypatch):
    """A transposed W block (column-major instead of row-major) fails the
    autograd pin."""
    orig = nqs.unpack

    def transposed(theta, V, H):
        a, b, W = orig(theta, V, H)
        return a, b, np.asarray(theta[V + H:]).reshape(V, H).T

    monkeypatch.setattr(nqs, "unpack", transposed)
    n, H = 4, 3
    V = 2 * n
    keys = space.full_space(n, 2, 2)
    theta = synth.nqs_theta(V, H, 0, scale=0.3)
    psi, _ = nqs.psi_and_jacobian(keys, n, V, H, theta)
    x = torch.from_numpy(nqs.occupations(keys, n))
    assert np.max(np.abs(_torch_psi(x, torch.from_numpy(theta), V, H).numpy() - psi)) > 1e-6
