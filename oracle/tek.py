"""Dense (non-perturbative) TEK model quantities: action, staple, force.

Oracle (test infrastructure only; see the package docstring).

These are used to pin the perturbative force of ``nspt`` (its sign and
normalisation) against a finite-difference gradient of the action, and to
check that the twisted vacuum is a stationary point.
"""
from __future__ import annotations

import numpy as np


def twist_tensor(L: int, k: int) -> np.ndarray:
    """z_{mu nu} = exp(2 pi i k / L) for mu < nu and its complex conjugate for
    mu > nu (Section 2, below eq. (1): an antisymmetric twist exponent
    n_{mu nu} = -n_{nu mu}, so z_{nu mu} = z_{mu nu}^*).  Diagonal entries
    are unused and set to 0.  Returns complex128 [4, 4]."""
    z = np.zeros((4, 4), dtype=np.complex128)
    ph = np.exp(2j * np.pi * k / L)
    for mu in range(4):
        for nu in range(4):
            if mu < nu:
                z[mu, nu] = ph
            elif mu > nu:
                z[mu, nu] = np.conj(ph)
    return z


def action(u: np.ndarray, z: np.ndarray, beta: float = 1.0) -> float:
    """S(U) = beta sum_{mu != nu} Tr[1 - z_{mu nu} U_mu U_nu U_mu^+ U_nu^+]
    (Section 2, eq. (1), the exponent of the partition function).  u is
    complex128 [4, N, N].  The sum over ordered pairs is real because the
    (nu, mu) term is the complex conjugate of the (mu, nu) term."""
    n = u.shape[-1]
    s = 0.0 + 0.0j
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            plaq = u[mu] @ u[nu] @ u[mu].conj().T @ u[nu].conj().T
            s += n - z[mu, nu] * np.trace(plaq)
    return float(beta * s.real)


def staple(u: np.ndarray, z: np.ndarray, mu: int) -> np.ndarray:
    """S_mu = U_mu sum_{nu != mu} ( z_{mu nu} U_nu U_mu^+ U_nu^+
                                   + z_{mu nu}^* U_nu^+ U_mu^+ U_nu )

    Eq. (2).  The paper prints a minus sign in front of the second term; the
    plus sign is the one that makes F below the gradient of eq. (1) (checked
    by the finite-difference test), and it is the reading used throughout.
    """
    ud = np.conj(np.swapaxes(u, -1, -2))
    acc = np.zeros_like(u[mu])
    for nu in range(4):
        if nu == mu:
            continue
        acc += z[mu, nu] * (u[nu] @ ud[mu] @ ud[nu])
        acc += np.conj(z[mu, nu]) * (ud[nu] @ ud[mu] @ u[nu])
    return u[mu] @ acc


def project_force(s: np.ndarray, beta: float = 1.0) -> np.ndarray:
    """F = i beta [ (S - S^+) - Tr(S - S^+)/N * 1 ]  (eq. (2)).

    S - S^+ is anti-Hermitian; removing its trace and multiplying by i gives
    a traceless Hermitian matrix."""
    n = s.shape[-1]
    d = s - s.conj().T
    return 1j * beta * (d - np.trace(d) / n * np.eye(n))


def force(u: np.ndarray, z: np.ndarray, mu: int, beta: float = 1.0) -> np.ndarray:
    """F_mu of eq. (2) for link configuration u [4, N, N]."""
    return project_force(staple(u, z, mu), beta)
