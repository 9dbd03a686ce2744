"""Linear-method matrices, energy centring, eigenproblem and update (dense FP64).

Methods, "From SR to a Stable Eigenvalue Problem":

* tangent basis chi_0 = psi, chi_i = d psi / d theta_i; H~_ij = <chi_i|H|chi_j>,
  S~_ij = <chi_i|chi_j> (Eq. rayleigh_quotient), both (p+1) x (p+1);
* normalisation <psi|psi> = 1, realised here by D^ = D~ / sqrt(Z), Z = psi^T psi;
* energy E = psi^T H psi / Z; centred operator H' = H - E;
* H_eff = <d psi|H'|d psi> (Eq. heff) and the standard Hermitian problem
  H_eff v = lambda v obtained from S ~ I (Eq. standard_evp);
* the full problem H~ c = lambda S~ c (Eq. full_gevp) with c = [1, v].

Readings (the paper is not explicit):
* mode "A" (default): the S ~ I problem on the (p+1)-dimensional centred matrix
  H~' = H~ - E S~ = [[0, g^T / 2], [g / 2, H_eff]] (identity metric); the lowest
  eigenpair (lambda, c) gives the update dtheta = c[1:] / c[0], the reading of
  c = [1, v] under which the eigenvector alone fixes direction and length.
* mode "P": the literal p x p problem H_eff v = lambda v; direction only
  (step length parity unpinned).
* mode "G": the exact generalised problem H~' c = lambda S~ c, solved after
  canonical orthogonalisation of S~.
* mode "C": mode A in the connected tangent basis, whose derivative columns are
  projected against psi, d_i psi - psi (psi^T d_i psi) / Z (the connected
  correlation form named after Eq. centered_hamiltonian).  With sigma =
  D~[:, 1:]^T psi / Z, the linearised wavefunction c_0 psi + sum_i c_i (d_i psi
  - sigma_i psi) is proportional to psi + sum_i dtheta_i d_i psi for dtheta =
  c[1:] / (c_0 - sigma . c[1:]), which is the update taken.

Pins: tests/test_oracle_lm.py (identities, D~ = I reduction to exact
diagonalisation, zero update at an exact wavefunction, exact GEVP, ARPACK's
implicitly restarted Lanczos, finite-difference gradient, predicted decrease);
tests/test_oracle_connected.py (mode C: orthogonality of the connected columns,
invariance under d_i psi -> d_i psi + a_i psi, reduction to mode A when the
derivatives are already orthogonal to psi, zero update at an exact
wavefunction, and the exact generalised problem reaching the same eigenvalue
and linearised wavefunction in either basis).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def exact_sum(x: np.ndarray) -> float:
    """Correctly rounded sum (math.fsum)."""
    return math.fsum(np.asarray(x, dtype=np.float64).tolist())


def energy(psi: np.ndarray, Hmat: sp.spmatrix, e_core: float = 0.0):
    """(Z, E_el, E) with Z = psi^T psi and E_el = psi^T H psi / Z (electronic),
    E = E_el + e_core.  Sums are correctly rounded."""
    r = Hmat @ psi
    Z = exact_sum(psi * psi)
    E_el = exact_sum(psi * r) / Z
    return Z, E_el, E_el + e_core


def gradient(Dt: np.ndarray, Hmat: sp.spmatrix) -> np.ndarray:
    """g = dE/dtheta = 2 J^T (H psi - E psi) / Z (real wavefunction)."""
    psi = Dt[:, 0]
    Z, E_el, _ = energy(psi, Hmat)
    r = Hmat @ psi
    return 2.0 * (Dt[:, 1:].T @ (r - E_el * psi)) / Z


def apply_lm_operator(Dt: np.ndarray, Hmat: sp.spmatrix, v: np.ndarray):
    """Raw, unnormalised operator pair for one vector (matrix-free):
    y_H = D~^T H D~ v, y_S = D~^T D~ v."""
    w = Dt @ v
    u = Hmat @ w
    return Dt.T @ u, Dt.T @ w


def dense_matrices(Dt: np.ndarray, Hmat: sp.spmatrix):
    """Normalised H~ = D^T H D^, S~ = D^T D^ with D^ = D~ / sqrt(Z)."""
    psi = Dt[:, 0]
    Z = exact_sum(psi * psi)
    Dh = Dt / math.sqrt(Z)
    St = Dh.T @ Dh
    Ht = Dh.T @ np.asarray(Hmat @ Dh)
    return Ht, St


def centred(Ht: np.ndarray, St: np.ndarray, E_el: float) -> np.ndarray:
    """H~' = H~ - E S~, symmetrised."""
    Hp = Ht - E_el * St
    return 0.5 * (Hp + Hp.T)


@dataclass
class LMResult:
    E: float            # energy at theta (including e_core)
    E_el: float
    Z: float
    lam: float          # lowest eigenvalue of the chosen problem
    c: np.ndarray       # its eigenvector (unit norm, or S-normalised in mode G)
    dtheta: np.ndarray | None
    gap: float          # lambda_2 - lambda_1
    Hp: np.ndarray      # the centred matrix H~'
    St: np.ndarray


def solve(Dt: np.ndarray, Hmat: sp.spmatrix, mode: str = "A", e_core: float = 0.0,
          s_cut: float = 1e-12) -> LMResult:
    """Dense solve of the LM eigenproblem for the basis D~ (N_s x (p+1))."""
    psi = Dt[:, 0]
    Z, E_el, E = energy(psi, Hmat, e_core)
    Ht, St = dense_matrices(Dt, Hmat)
    Hp = centred(Ht, St, E_el)
    if mode == "A":
        w, U = np.linalg.eigh(Hp)
        c = U[:, 0]
        dtheta = c[1:] / c[0]
        gap = w[1] - w[0] if w.size > 1 else np.inf
        return LMResult(E, E_el, Z, w[0], c, dtheta, gap, Hp, St)
    if mode == "P":
        w, U = np.linalg.eigh(Hp[1:, 1:])
        gap = w[1] - w[0] if w.size > 1 else np.inf
        return LMResult(E, E_el, Z, w[0], U[:, 0], None, gap, Hp, St)
    if mode == "C":
        Dc, sigma = connected_basis(Dt)
        res = solve(Dc, Hmat, mode="A", e_core=e_core)
        res.dtheta = connected_update(res.c, sigma)
        return res
    if mode == "G":
        s, Us = np.linalg.eigh(0.5 * (St + St.T))
        keep = s > s_cut * s.max()
        X = Us[:, keep] / np.sqrt(s[keep])       # canonical orthogonalisation
        w, Y = np.linalg.eigh(X.T @ Hp @ X)
        c = X @ Y[:, 0]
        dtheta = c[1:] / c[0]
        gap = w[1] - w[0] if w.size > 1 else np.inf
        return LMResult(E, E_el, Z, w[0], c, dtheta, gap, Hp, St)
    raise ValueError(mode)


def connected_basis(Dt: np.ndarray):
    """(D_c, sigma): the columns d_i psi of D~ (i >= 1) replaced by their
    components orthogonal to psi, d_i psi - sigma_i psi with sigma_i =
    psi^T d_i psi / Z; column 0 (psi) is kept."""
    psi = Dt[:, 0]
    Z = exact_sum(psi * psi)
    sigma = (Dt[:, 1:].T @ psi) / Z
    Dc = Dt.copy()
    Dc[:, 1:] = Dt[:, 1:] - np.outer(psi, sigma)
    return Dc, sigma


def connected_update(c: np.ndarray, sigma: np.ndarray):
    """dtheta from an eigenvector c in the connected basis: the coefficient of
    psi in the linearised wavefunction is c_0 - sigma . c[1:]."""
    return c[1:] / (c[0] - sigma @ c[1:])


def eigh_lowest(A: np.ndarray):
    """Lowest eigenpair of a dense symmetric matrix (scipy)."""
    w, U = sla.eigh(A, subset_by_index=[0, 0])
    return w[0], U[:, 0]


def streamed_evaluation(keys, n, V, H, theta, h_apply, vs=(), chunk=20_000):
    """Energy, gradient and operator pairs over a large set without holding D~.

    The same definitions as ``energy``, ``gradient`` and ``apply_lm_operator``,
    written for sets whose D~ does not fit in host memory: rows of D~ are
    recomputed from theta (``nqs.dtilde``) chunk by chunk for each product, and
    H is applied matrix-free by ``h_apply(w) -> H w`` over the whole set (the
    plain C Slater-Condon apply).  Each product D~^T y is the sum over row
    chunks of D~_chunk^T y_chunk.  Returns (Z, E_el, g, [(y_H, y_S) per v]).
    Pinned against the dense functions in tests/test_oracle_lm.py.
    """
    from . import nqs

    keys = np.asarray(keys, dtype=np.uint64)
    ns = keys.size
    P = V * H + H + V

    def rows(c0):
        return nqs.dtilde(keys[c0:c0 + chunk], n, V, H, theta)

    psi = np.empty(ns)
    ws = [np.empty(ns) for _ in vs]
    for c0 in range(0, ns, chunk):
        Dc = rows(c0)
        psi[c0:c0 + chunk] = Dc[:, 0]
        for w, v in zip(ws, vs):
            w[c0:c0 + chunk] = Dc @ v
    r = h_apply(psi)
    Z = exact_sum(psi * psi)
    E_el = exact_sum(psi * r) / Z
    us = [h_apply(w) for w in ws]
    resid = r - E_el * psi
    g = np.zeros(P)
    yH = [np.zeros(P + 1) for _ in vs]
    yS = [np.zeros(P + 1) for _ in vs]
    for c0 in range(0, ns, chunk):
        Dc = rows(c0)
        sl = slice(c0, c0 + chunk)
        g += Dc[:, 1:].T @ resid[sl]
        for j in range(len(vs)):
            yH[j] += Dc.T @ us[j][sl]
            yS[j] += Dc.T @ ws[j][sl]
    g *= 2.0 / Z
    return Z, E_el, g, list(zip(yH, yS))
