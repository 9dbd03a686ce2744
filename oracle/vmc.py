"""Sampled (variational Monte Carlo) estimators of the energy, the gradient and
the effective Hamiltonian's product with a vector.

Test infrastructure: only tests/, the package's smoke check and the benchmark's
CPU baseline use this module; the product path never calls it.

Sources:

* Methods, "Autoregressive Modeling and Physical Constraints": p(n) = |psi(n)|^2
  factorised into conditionals over the spin-orbitals (Eq.
  autoregressive_factorization) and sampled one orbital at a time, with the
  conditionals restricted so that the spin-up and spin-down electron counts
  never exceed N_up and N_down, then renormalised (Eq. constraint).  The
  network here is not autoregressive, so the conditionals are the exact
  marginals of |psi|^2 over the determinant set (the set holds only valid
  configurations, so a branch that breaks the counts has zero weight).  One
  uniform number per sample drives the whole sequence: at each orbital it is
  compared with the probability of an empty orbital and rescaled into the
  chosen branch's interval.  Orbital order: most significant key bit first
  (beta orbital n-1 down to beta 0, then alpha n-1 down to alpha 0), the order
  in which ascending keys are lexicographic.
* Methods, "From SR to a Stable Eigenvalue Problem": the local energy E_loc(x)
  = (H psi)(x) / psi(x), the log-derivatives O_i(x) = d ln psi(x) / d theta_i,
  E = <E_loc>, H_eff = <O E_loc O> - E S with S = <O O> (Eq.
  centered_hamiltonian).
* Methods, "Practical Matrix-Free Implementation": the product H_eff v as the
  sample mean of O_i (E_loc - E) (O . v) (Eq. matrix_vec_prod); the gradient F
  = 2 <O (E_loc - E)> (the cost analysis in the same part).

The augmented problem (mode A) adds O_0 = 1 for the psi direction, so its
centred matrix is the sample mean of O (E_loc - E) O^T over the P + 1
components: entry (0, 0) is <E_loc - E> = 0 and column 0 is F / 2.

Pins: tests/test_oracle_vmc.py.
"""
from __future__ import annotations

import math

import numpy as np


def spin_orbital_order(n: int) -> list[int]:
    """Key bits in sampling order: beta n-1 .. beta 0, then alpha n-1 .. alpha 0."""
    return [32 + p for p in range(n - 1, -1, -1)] + [p for p in range(n - 1, -1, -1)]


def sample_autoregressive(keys: np.ndarray, n: int, na: int, nb: int, psi: np.ndarray,
                          u: np.ndarray, order=None) -> np.ndarray:
    """Row index of each sample, drawn orbital by orbital from the exact
    conditionals of |psi|^2 on the set (Eqs. autoregressive_factorization and
    constraint) with one uniform number u_s in [0, 1) per sample.  order: key
    bits in sampling order (default spin_orbital_order(n))."""
    keys = np.asarray(keys, dtype=np.uint64)
    w = np.asarray(psi, dtype=np.float64) ** 2
    order = spin_orbital_order(n) if order is None else list(order)
    rows = np.empty(len(u), dtype=np.int64)
    for s, us in enumerate(np.asarray(u, dtype=np.float64)):
        match = np.ones(keys.size, dtype=bool)       # configurations with the chosen prefix
        n_up = n_dn = 0
        x = float(us)
        for bit in order:
            is_beta = bit >= 32
            occ = ((keys >> np.uint64(bit)) & np.uint64(1)).astype(bool)
            w0 = math.fsum(w[match & ~occ].tolist())
            w1 = math.fsum(w[match & occ].tolist())
            # Eq. constraint: no branch past the prescribed electron counts
            if (is_beta and n_dn + 1 > nb) or (not is_beta and n_up + 1 > na):
                w1 = 0.0
            p0 = w0 / (w0 + w1)
            if x < p0:
                match &= ~occ
                x = x / p0
            else:
                match &= occ
                x = (x - p0) / (1.0 - p0) if p0 < 1.0 else 0.0
                if is_beta:
                    n_dn += 1
                else:
                    n_up += 1
        idx = np.nonzero(match)[0]
        assert idx.size == 1
        rows[s] = idx[0]
    return rows


def local_energy(psi: np.ndarray, Hmat) -> np.ndarray:
    """E_loc(x) = (H psi)(x) / psi(x) for every row (inf/nan where psi = 0;
    such rows are never sampled)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.asarray(Hmat @ psi) / psi


def log_derivatives(Dt: np.ndarray) -> np.ndarray:
    """O (N x (P+1)): column 0 is psi / psi = 1, columns i >= 1 are
    d psi / d theta_i / psi."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return Dt / Dt[:, :1]


def sampled_energy(rows: np.ndarray, Eloc: np.ndarray) -> float:
    """E = (1 / N) sum_s E_loc(x_s) (correctly rounded sum)."""
    return math.fsum(Eloc[rows].tolist()) / len(rows)


def sampled_variance(rows: np.ndarray, Eloc: np.ndarray) -> float:
    E = sampled_energy(rows, Eloc)
    return math.fsum(((Eloc[rows] - E) ** 2).tolist()) / len(rows)


def sampled_gradient(rows: np.ndarray, O: np.ndarray, Eloc: np.ndarray) -> np.ndarray:
    """F = (2 / N) sum_s O(x_s) (E_loc(x_s) - E) over the P parameters."""
    E = sampled_energy(rows, Eloc)
    Os = O[rows, 1:]
    return 2.0 * (Os.T @ (Eloc[rows] - E)) / len(rows)


def sampled_mvp(rows: np.ndarray, O: np.ndarray, Eloc: np.ndarray, v: np.ndarray) -> np.ndarray:
    """(1 / N) sum_s O(x_s) (E_loc(x_s) - E) (O(x_s) . v) (Eq. matrix_vec_prod) over
    the P + 1 augmented components (O_0 = 1); v has P + 1 entries."""
    E = sampled_energy(rows, Eloc)
    Os = O[rows]
    return Os.T @ ((Eloc[rows] - E) * (Os @ v)) / len(rows)


def sampled_pair(rows: np.ndarray, O: np.ndarray, Eloc: np.ndarray, v: np.ndarray):
    """(<O E_loc O^T> v, <O O^T> v) over the samples: the two terms of Eq.
    centered_hamiltonian applied to v (augmented, P + 1 components)."""
    Os = O[rows]
    Ov = Os @ v
    return Os.T @ (Eloc[rows] * Ov) / len(rows), Os.T @ Ov / len(rows)


def sampled_matrix(rows: np.ndarray, O: np.ndarray, Eloc: np.ndarray) -> np.ndarray:
    """The sampled centred matrix (1 / N) sum_s O (E_loc - E) O^T, (P+1) x (P+1)."""
    E = sampled_energy(rows, Eloc)
    Os = O[rows]
    M = Os.T @ ((Eloc[rows] - E)[:, None] * Os) / len(rows)
    return 0.5 * (M + M.T)


def solve_sampled(rows: np.ndarray, O: np.ndarray, Eloc: np.ndarray, mode: str = "A"):
    """Lowest eigenpair of the sampled centred matrix with identity metric:
    mode A on the P + 1 augmented components (update c[1:] / c[0]), mode P on
    H_eff alone (direction only).  Returns (lambda, c, dtheta or None, matrix)."""
    M = sampled_matrix(rows, O, Eloc)
    if mode == "A":
        w, U = np.linalg.eigh(M)
        c = U[:, 0]
        return w[0], c, c[1:] / c[0], M
    if mode == "P":
        w, U = np.linalg.eigh(M[1:, 1:])
        return w[0], U[:, 0], None, M
    raise ValueError(mode)
