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
* the Langevin and MD steps carry no gauge fixing (the paper omits its
  details); ``gauge_fix`` below is a separate step of this
  implementation's own design.
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


# --------------------------------------------------------------------------
# Molecular-dynamics form of the tower (Section 2, eq. (3) and the sentence
# after it: the truncated tower is integrated with a symplectic integrator
# and the momenta are refreshed periodically).
#
# With P = (1/g) sum_{k>=1} g^k P^(k) and the fictitious time rescaled by g,
# the equations read dU/dt = i (P * U), dP^(k)/dt = F^(k) for k >= 1, where P
# is the series sum_{k>=1} g^k P^(k) (no order-0 term) and F^(k) is the
# series force above.  Readings used here:
# * the symplectic integrator is the leapfrog in kick-drift-kick order with
#   step dt (the paper does not name one);
# * a refresh sets P^(1) to Hermitian traceless Gaussian noise and every
#   other order to zero (the momentum is O(1) in the full theory, i.e. it sits
#   at order 1 of the series);
# * the force enters at orders k >= 1 only (F^(0) vanishes at the vacuum).
# The series Hamiltonian H = 1/2 sum_mu Tr (P_mu * P_mu) + S(U), S the action
# of eq. (1) at beta = 1 expanded in g, is conserved order by order by the
# exact flow; the leapfrog keeps it up to O(dt^2) per trajectory.
# --------------------------------------------------------------------------


def refresh_momentum(eta: np.ndarray, ntrunc: int) -> np.ndarray:
    """Momentum series after a refresh: P^(1) = eta_mu, other orders zero.
    eta: complex128 [4, N, N] Hermitian traceless; returns [4, ntrunc+1, N, N]."""
    eta = np.asarray(eta, dtype=np.complex128)
    p = np.zeros((4, ntrunc + 1) + eta.shape[1:], dtype=np.complex128)
    if ntrunc >= 1:
        p[:, 1] = eta
    return p


def md_forces(u: np.ndarray, z: np.ndarray) -> np.ndarray:
    """F_mu^(k) for all mu, with the order-0 term set to zero."""
    f = np.stack([series_force(u, z, mu) for mu in range(4)])
    f[:, 0] = 0.0
    return f


def md_drift(u: np.ndarray, p: np.ndarray, dt: float) -> np.ndarray:
    """U_mu <- exp(i dt P_mu) * U_mu for every mu (exact in the truncated series)."""
    return np.stack([ser.star(ser.series_exp(1j * dt * p[mu]), u[mu]) for mu in range(4)])


def md_trajectory(u: np.ndarray, p: np.ndarray, z: np.ndarray, dt: float, nsteps: int):
    """Leapfrog trajectory of nsteps steps of size dt from (U, P):
    half kick, then (drift, kick) nsteps - 1 times, drift, half kick.
    Returns the new (U, P); the inputs are not modified."""
    if nsteps < 1:
        raise ValueError("nsteps must be >= 1")
    u = np.array(u, dtype=np.complex128)
    p = np.array(p, dtype=np.complex128)
    p = p + 0.5 * dt * md_forces(u, z)
    for i in range(nsteps):
        u = md_drift(u, p, dt)
        p = p + (dt if i < nsteps - 1 else 0.5 * dt) * md_forces(u, z)
    return u, p


def md_trajectory_replicas(u: np.ndarray, p: np.ndarray, z: np.ndarray, dt: float, nsteps: int):
    """Replica batch: u, p [R, 4, ntrunc+1, N, N]."""
    out = [md_trajectory(u[r], p[r], z, dt, nsteps) for r in range(u.shape[0])]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def series_action(u: np.ndarray, z: np.ndarray) -> np.ndarray:
    """S^(k) = sum_{mu != nu} Tr[ delta_{k0} 1 - z_{mu nu} (U_mu * U_nu * U_mu^+ * U_nu^+)^(k) ],
    eq. (1) at beta = 1 expanded in g; real for every k (the (nu, mu) term is
    the conjugate of the (mu, nu) term).  Returns float64 [ntrunc+1]."""
    n = u.shape[-1]
    ud = [ser.dagger(u[m]) for m in range(4)]
    s = np.zeros(u.shape[1], dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            plaq = ser.star(ser.star(ser.star(u[mu], u[nu]), ud[mu]), ud[nu])
            s -= z[mu, nu] * np.trace(plaq, axis1=-2, axis2=-1)
    s[0] += 12 * n
    return s.real


def series_hamiltonian(u: np.ndarray, p: np.ndarray, z: np.ndarray) -> np.ndarray:
    """H^(k) = 1/2 sum_mu Tr (P_mu * P_mu)^(k) + S^(k)  (float64 [ntrunc+1])."""
    kin = np.zeros(u.shape[1])
    for mu in range(4):
        kin += 0.5 * np.trace(ser.star(p[mu], p[mu]), axis1=-2, axis2=-1).real
    return kin + series_action(u, z)


def wilson_loop_series(u: np.ndarray, z: np.ndarray, a: int, b: int) -> np.ndarray:
    """a x b Wilson loop of the reduced model as a series in g (the observable
    of the paper's abstract and Section 1):
      W^(k) = 1/(6N) sum_{mu<nu} Re z_{mu nu}^{ab} Tr (U_mu^a * U_nu^b * (U_mu^+)^a * (U_nu^+)^b)^(k),
    every power and product the truncated star product.  The twist factor
    z^{ab} makes W = 1 at the twisted vacuum.  Returns float64 [ntrunc+1]."""
    n = u.shape[-1]
    ua = [_series_power(u[m], a) for m in range(4)]
    ub = [_series_power(u[m], b) for m in range(4)]
    w = np.zeros(u.shape[1], dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            loop = ser.star(ser.star(ser.star(ua[mu], ub[nu]), ser.dagger(ua[mu])), ser.dagger(ub[nu]))
            w += z[mu, nu] ** (a * b) * np.trace(loop, axis1=-2, axis2=-1)
    return w.real / (6 * n)


def _series_power(x: np.ndarray, p: int) -> np.ndarray:
    out = x
    for _ in range(p - 1):
        out = ser.star(out, x)
    return out


# --------------------------------------------------------------------------
# Stochastic gauge fixing (the paper states that it is used and omits its
# details, Section 2; the form below is this implementation's design).
#
# The reduced model is invariant under U_mu -> Omega U_mu Omega^+ with one
# Omega in SU(N) for all directions.  Writing U_mu = V_mu Gamma_mu with the
# twist eaters Gamma_mu = U_mu^(0), this acts on the fluctuation as
# V_mu -> Omega V_mu (Gamma_mu Omega^+ Gamma_mu^+): conjugation by Gamma_mu
# plays the part of the lattice shift by mu, and the reduced-model Landau
# gauge maximises F(Omega) = sum_mu Re Tr (Omega U_mu Omega^+ Gamma_mu^+).
# Its gradient at Omega = 1 is carried by
#     G = sum_mu ( U_mu Gamma_mu^+ - Gamma_mu^+ U_mu ),
# and one steepest-ascent step of size alpha is Omega = exp(Y) with
#     Y = -(alpha/2) [ (G - G^+) - Tr(G - G^+)/N ]
# (anti-Hermitian, traceless).  G^(0) = 0, so Omega^(0) = 1 and the vacuum
# is left alone.  To first order a pure-gauge fluctuation
# U_mu^(1) = i [w, Gamma_mu] with Gamma_nu w Gamma_nu^+ = phi_nu w for all
# nu is damped by the factor 1 - alpha lambda, lambda = sum_nu |1 - phi_nu|^2
# (the lattice Laplacian of that mode).
# --------------------------------------------------------------------------


def gauge_generator(u: np.ndarray) -> np.ndarray:
    """G = sum_mu (U_mu * Gamma_mu^+ - Gamma_mu^+ * U_mu), Gamma_mu = U_mu^(0)
    taken as an order-0 series; every * the truncated star product."""
    g = np.zeros_like(u[0])
    for mu in range(4):
        v = np.zeros_like(u[mu])
        v[0] = u[mu, 0]
        vd = ser.dagger(v)
        g += ser.star(u[mu], vd) - ser.star(vd, u[mu])
    return g


def gauge_exponent(u: np.ndarray, alpha: float) -> np.ndarray:
    """Y = -(alpha/2) [ (G - G^+) - Tr(G - G^+)/N ] for every order, Y^(0) = 0."""
    g = gauge_generator(u)
    n = u.shape[-1]
    d = g - ser.dagger(g)
    tr = np.trace(d, axis1=-2, axis2=-1)
    y = -0.5 * alpha * (d - tr[:, None, None] / n * np.eye(n)[None])
    y[0] = 0.0
    return y


def gauge_fix(u: np.ndarray, alpha: float) -> np.ndarray:
    """One gauge-fixing step of one replica: U_mu <- Omega * U_mu * Omega^+
    for every mu with the same Omega = exp(Y) (series exponential)."""
    u = np.asarray(u, dtype=np.complex128)
    om = ser.series_exp(gauge_exponent(u, alpha))
    omd = ser.dagger(om)
    return np.stack([ser.star(ser.star(om, u[mu]), omd) for mu in range(4)])


def gauge_fix_replicas(u: np.ndarray, alpha: float) -> np.ndarray:
    """Replica batch: u [R, 4, ntrunc+1, N, N]."""
    return np.stack([gauge_fix(u[r], alpha) for r in range(u.shape[0])])


# --------------------------------------------------------------------------
# Noise drawn from a counter-based generator, so that the device and this
# oracle draw the same Gaussian noise from (seed, step) (an optional form of
# the Langevin step; the paper does not say how its noise is generated).
#
# Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), restated from
# its definition.  Per step t, replica r, direction mu and entry pair i <= j
# of the N x N matrix: counter (i N + j, 4 r + mu, t, 0), key (seed, 0).
# Of the four 64-bit outputs x0, x1: u_a = ((x0 >> 11) + 1) 2^-53 in (0, 1],
# u_b = (x1 >> 11) 2^-53 in [0, 1); Box-Muller rho = sqrt(-2 ln u_a),
# z0 = rho cos(2 pi u_b), z1 = rho sin(2 pi u_b).  eta_ij = (z0 + i z1)/sqrt(2)
# and eta_ji = conj(eta_ij) for i < j, eta_ii = z0; then the trace is removed
# from the diagonal (the GUE-traceless recipe of the Langevin noise).
# --------------------------------------------------------------------------

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_MASK64 = (1 << 64) - 1


def _mulhilo(a: np.ndarray, m: int):
    """64 x 64 -> 128-bit product of uint64 arrays a and the constant m, as (hi, lo)."""
    a = a.astype(np.uint64)
    a_lo, a_hi = a & np.uint64(0xFFFFFFFF), a >> np.uint64(32)
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    p0 = a_lo * m_lo
    p1 = a_lo * m_hi
    p2 = a_hi * m_lo
    p3 = a_hi * m_hi
    mid = (p0 >> np.uint64(32)) + (p1 & np.uint64(0xFFFFFFFF)) + (p2 & np.uint64(0xFFFFFFFF))
    hi = p3 + (p1 >> np.uint64(32)) + (p2 >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = a * np.uint64(m)          # wraps modulo 2^64
    return hi, lo


def philox4x64(counter, key, rounds: int = 10):
    """Philox4x64 of counter (4 uint64 arrays) under key (2 uint64 arrays)."""
    c = [np.asarray(x, dtype=np.uint64) for x in counter]
    k = [np.asarray(x, dtype=np.uint64) for x in key]
    with np.errstate(over="ignore"):
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(c[0], _PHILOX_M[0])
            hi1, lo1 = _mulhilo(c[2], _PHILOX_M[1])
            c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
            k = [k[0] + np.uint64(_PHILOX_W[0]), k[1] + np.uint64(_PHILOX_W[1])]
    return c


def philox_noise(seed: int, step: int, replicas: int, n: int) -> np.ndarray:
    """Hermitian traceless noise complex128 [replicas, 4, n, n] of step `step`."""
    i, j = np.triu_indices(n)
    out = np.zeros((replicas, 4, n, n), dtype=np.complex128)
    for r in range(replicas):
        for mu in range(4):
            ctr = [(i * n + j).astype(np.uint64), np.full(i.shape, 4 * r + mu, np.uint64),
                   np.full(i.shape, step, np.uint64), np.zeros(i.shape, np.uint64)]
            x = philox4x64(ctr, [np.full(i.shape, seed, np.uint64), np.zeros(i.shape, np.uint64)])
            ua = ((x[0] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
            ub = (x[1] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
            rho = np.sqrt(-2.0 * np.log(ua))
            z0, z1 = rho * np.cos(2.0 * np.pi * ub), rho * np.sin(2.0 * np.pi * ub)
            e = np.zeros((n, n), dtype=np.complex128)
            off = i < j
            e[i[off], j[off]] = (z0[off] + 1j * z1[off]) / np.sqrt(2.0)
            e[j[off], i[off]] = (z0[off] - 1j * z1[off]) / np.sqrt(2.0)
            d = ~off
            e[i[d], i[d]] = z0[d]
            e -= np.trace(e) / n * np.eye(n)
            out[r, mu] = e
    return out


def langevin_steps_philox(u: np.ndarray, z: np.ndarray, eps: float, seed: int, step0: int,
                          nsteps: int) -> np.ndarray:
    """nsteps Langevin steps of a replica batch u [R, 4, ntrunc+1, N, N] with
    the noise of steps step0 .. step0 + nsteps - 1."""
    for t in range(step0, step0 + nsteps):
        eta = philox_noise(seed, t, u.shape[0], u.shape[-1])
        u = langevin_step_replicas(u, eta, z, eps)
    return u
