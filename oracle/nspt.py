"""Perturbative staple, force and one Euler-Langevin step (NSPT for TEK).

Oracle (test infrastructure only; see the package docstring).

Link series: complex128 [4, ntrunc + 1, N, N] for one replica (direction mu,
order k, matrix); noise: complex128 [4, N, N], Hermitian traceless.

Readings of the paper used here (Section 2, eqs. (2)-(3)):
* the second staple term enters with a plus sign (see ``tek.staple``);
* after the rescaling of the fictitious time the factor beta is absorbed,
  so F^(k) = i[D^(k) - Tr(D^(k))/N], D = S - S^+; the step size eps is the
  rescaled one and the Gaussian noise enters at order g^1 as sqrt(2 eps) eta;
* the order-0 drift is dropped (X^(0) = 0): the expansion is around the
  classical vacuum, where the force vanishes;
* all four directions are updated from the same old links (Jacobi order);
* no stochastic gauge fixing (the paper omits its details).
"""
from __future__ import annotations

import numpy as np

from . import series as ser


def series_staple(u: np.ndarray, z: np.ndarray, mu: int) -> np.ndarray:
    """S_mu = U_mu * sum_{nu != mu} ( z_{mu nu} U_nu * U_mu^+ * U_nu^+
                                   + z_{mu nu}^* U_nu^+ * U_mu^+ * U_nu )
    with every * the truncated star product (eq. (3))."""
    ud = [ser.dagger(u[m]) for m in range(4)]
    acc = np.zeros_like(u[mu])
    for nu in range(4):
        if nu == mu:
            continue
        acc += z[mu, nu] * ser.star(ser.star(u[nu], ud[mu]), ud[nu])
        acc += np.conj(z[mu, nu]) * ser.star(ser.star(ud[nu], ud[mu]), u[nu])
    return ser.star(u[mu], acc)


def project_series(s: np.ndarray) -> np.ndarray:
    """F^(k) = i [ D^(k) - Tr(D^(k))/N * 1 ],  D = S - S^+, for every order k
    (eq. (3), with beta absorbed by the time rescaling)."""
    n = s.shape[-1]
    d = s - ser.dagger(s)
    tr = np.trace(d, axis1=-2, axis2=-1)
    return 1j * (d - tr[:, None, None] / n * np.eye(n)[None])


def series_force(u: np.ndarray, z: np.ndarray, mu: int) -> np.ndarray:
    """The force series F_mu^(k), k = 0..ntrunc."""
    return project_series(series_staple(u, z, mu))


def drift_noise(force: np.ndarray, eta: np.ndarray, eps: float) -> np.ndarray:
    """X^(k) = eps F^(k) + delta_{k,1} sqrt(2 eps) eta, with X^(0) = 0."""
    x = eps * np.array(force, dtype=np.complex128)
    x[0] = 0.0
    if x.shape[0] > 1:
        x[1] += np.sqrt(2.0 * eps) * eta
    return x


def langevin_step(u: np.ndarray, eta: np.ndarray, z: np.ndarray, eps: float) -> np.ndarray:
    """One Euler-Langevin step of the link series of one replica:
    U_mu <- exp(i X_mu) * U_mu for all mu, X_mu from the old links."""
    u = np.asarray(u, dtype=np.complex128)
    new = np.empty_like(u)
    for mu in range(4):
        x = drift_noise(series_force(u, z, mu), eta[mu], eps)
        e = ser.series_exp(1j * x)
        new[mu] = ser.star(e, u[mu])
    return new


def langevin_step_replicas(u: np.ndarray, eta: np.ndarray, z: np.ndarray, eps: float) -> np.ndarray:
    """Replica batch: u [R, 4, ntrunc+1, N, N], eta [R, 4, N, N]."""
    return np.stack([langevin_step(u[r], eta[r], z, eps) for r in range(u.shape[0])])
