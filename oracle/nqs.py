"""One-hidden-layer real network: amplitude psi(x) and Jacobian d psi / d theta.

Methods, "From SR to a Stable Eigenvalue Problem": the linearised wavefunction
uses the tangent basis chi = {psi, d psi / d theta_1, ..., d psi / d theta_p}.
The matrix D~ has one row per determinant x and the columns
[psi(x), d psi(x) / d theta_1, ..., d psi(x) / d theta_p].

Architecture (the paper's network is autoregressive and complex but its layers
are not specified; a real one-hidden-layer network with tanh units is used):

    x_v = occupation of spin-orbital v (alpha orbitals v < n, beta v - n >= 0)
    t_h = tanh(b_h + sum_v W_hv x_v)
    psi(x) = sum_v a_v x_v + sum_h t_h

theta = [a (V), b (H), W (H x V, row-major)], V = 2n, P = V H + H + V.

Jacobian: d psi/d a_v = x_v; d psi/d b_h = 1 - t_h^2; d psi/d W_hv = (1 - t_h^2) x_v.

Pins: torch.autograd Jacobian and central finite differences
(tests/test_oracle_nqs.py).
"""
from __future__ import annotations

import numpy as np


def occupations(keys: np.ndarray, n: int) -> np.ndarray:
    """x (N_s x 2n) in {0, 1} from the determinant keys."""
    keys = np.asarray(keys, dtype=np.uint64)
    x = np.zeros((keys.size, 2 * n), dtype=np.float64)
    for v in range(n):
        x[:, v] = ((keys >> np.uint64(v)) & np.uint64(1)).astype(np.float64)
        x[:, n + v] = ((keys >> np.uint64(32 + v)) & np.uint64(1)).astype(np.float64)
    return x


def unpack(theta: np.ndarray, V: int, H: int):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == V * H + H + V
    a = theta[:V]
    b = theta[V:V + H]
    W = theta[V + H:].reshape(H, V)
    return a, b, W


def psi_and_jacobian(keys: np.ndarray, n: int, V: int, H: int, theta: np.ndarray):
    """Return (psi (N_s), J (N_s x P)) in float64."""
    assert V == 2 * n
    x = occupations(keys, n)
    a, b, W = unpack(theta, V, H)
    t = np.tanh(x @ W.T + b)                   # N_s x H
    psi = x @ a + t.sum(axis=1)
    d = 1.0 - t * t                            # d tanh / d z
    JW = (d[:, :, None] * x[:, None, :]).reshape(keys.size, H * V)
    J = np.concatenate([x, d, JW], axis=1)
    return psi, J


def dtilde(keys: np.ndarray, n: int, V: int, H: int, theta: np.ndarray) -> np.ndarray:
    """D~ = [psi, J], N_s x (P + 1), row-major float64."""
    psi, J = psi_and_jacobian(keys, n, V, H, theta)
    return np.concatenate([psi[:, None], J], axis=1)
