"""One optimisation step: evaluate the network, solve the LM eigenproblem densely,
update theta, and evaluate the energy at the new parameters.

Methods, "From SR to a Stable Eigenvalue Problem" (update from the lowest
eigenpair) and "Practical Matrix-Free Implementation" (one optimisation step
per eigen-solve).  The iterative solver of Algorithm 1 reaches the lowest
eigenpair of the same matrix; the oracle takes it with a dense eigensolver.
"""
from __future__ import annotations

import numpy as np

from . import lm, nqs


def lm_step(keys, n, V, H, theta, Hmat, mode="A", e_core=0.0):
    """Returns (LMResult at theta, theta_new, E(theta_new)).  In mode P no update
    is defined and theta_new is None."""
    Dt = nqs.dtilde(keys, n, V, H, theta)
    res = lm.solve(Dt, Hmat, mode=mode, e_core=e_core)
    if res.dtheta is None:
        return res, None, None
    theta_new = np.asarray(theta, dtype=np.float64) + res.dtheta
    psi_new, _ = nqs.psi_and_jacobian(keys, n, V, H, theta_new)
    _, _, E_after = lm.energy(psi_new, Hmat, e_core)
    return res, theta_new, E_after


def trajectory(keys, n, V, H, theta, Hmat, steps, mode="A", e_core=0.0):
    """Energies E(theta_0), E(theta_1), ... and the lowest eigenvalues of each
    step for ``steps`` consecutive mode-A (or G) updates."""
    energies, lams, thetas = [], [], [np.asarray(theta, dtype=np.float64)]
    th = thetas[0]
    for _ in range(steps):
        res, th_new, E_after = lm_step(keys, n, V, H, th, Hmat, mode, e_core)
        energies.append(res.E)
        lams.append(res.lam)
        th = th_new
        thetas.append(th)
    psi, _ = nqs.psi_and_jacobian(keys, n, V, H, th)
    energies.append(lm.energy(psi, Hmat, e_core)[2])
    return np.array(energies), np.array(lams), thetas
