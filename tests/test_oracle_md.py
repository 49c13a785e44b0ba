"""Pins of the oracle's molecular-dynamics trajectory (CPU only).

The leapfrog trajectory of the NSPT tower is pinned by: its equivalence with
the (separately pinned) Euler-Langevin step for one step after a refresh
(eps = dt^2 / 2); the closed form of a drift from the vacuum; time
reversibility; the O(dt^2) error of the series Hamiltonian, whose action part
is pinned to the dense action of eq. (1) by its Taylor expansion in g; and the
invariants (unitarity, Hermitian traceless momenta, gauge covariance).  Planted
mistakes in a copy of the integrator break the energy check.
"""
import numpy as np
import pytest

import synth
from oracle import nspt, series as ser, tek


def _series_links(L, k, nt, amp, seed):
    g = synth.twist_eaters(L, k)
    n = L * L
    rng = synth.rng_for(930, seed)
    u = np.zeros((4, nt + 1, n, n), dtype=np.complex128)
    for mu in range(4):
        x = np.zeros((nt + 1, n, n), dtype=np.complex128)
        for kk in range(1, nt + 1):
            x[kk] = amp ** kk * synth.gue_traceless(rng, n)
        gam = np.zeros_like(x)
        gam[0] = g[mu]
        u[mu] = ser.star(ser.series_exp(1j * x), gam)
    return u


def _setup(L=3, k=1, nt=5, amp=0.5, seed=1):
    u = _series_links(L, k, nt, amp, seed)
    z = tek.twist_tensor(L, k)
    eta = synth.langevin_noise(synth.rng_for(931, seed), 1, L * L)[0]
    return u, z, eta, nspt.refresh_momentum(eta, nt)


def test_refresh_puts_the_noise_at_order_one():
    u, z, eta, p = _setup()
    assert np.array_equal(p[:, 1], eta)
    assert not np.any(p[:, 0]) and not np.any(p[:, 2:])


def test_one_step_after_refresh_is_the_langevin_step():
    # P = eta g: half kick, drift exp(i dt (eta g + dt/2 F)) = exp(i (sqrt(2 eps) eta g + eps F))
    u, z, eta, p = _setup(nt=5)
    eps = 0.02
    u1, _ = nspt.md_trajectory(u, p, z, np.sqrt(2 * eps), 1)
    ul = nspt.langevin_step(u, eta, z, eps)
    assert np.abs(u1 - ul).max() < 1e-13


def test_drift_from_the_vacuum_closed_form():
    L, k, nt, dt = 3, 1, 6, 0.3
    u = synth.vacuum_links(L, k, nt)[0]
    z = tek.twist_tensor(L, k)
    eta = synth.langevin_noise(synth.rng_for(932), 1, L * L)[0]
    u1, p1 = nspt.md_trajectory(u, nspt.refresh_momentum(eta, nt), z, dt, 1)
    for mu in range(4):
        term = np.eye(L * L, dtype=np.complex128)
        for m in range(nt + 1):
            assert np.allclose(u1[mu, m], term @ u[mu, 0], atol=1e-14)
            term = term @ (1j * dt * eta[mu]) / (m + 1)
    assert np.array_equal(p1[:, 0], np.zeros_like(p1[:, 0]))


def test_trajectory_is_time_reversible():
    u, z, eta, p = _setup(nt=4, seed=2)
    u1, p1 = nspt.md_trajectory(u, p, z, 0.1, 3)
    u2, p2 = nspt.md_trajectory(u1, -p1, z, 0.1, 3)
    assert np.abs(u2 - u).max() < 1e-12
    assert np.abs(p2 + p).max() < 1e-12


def _energy_ratios(traj, u, p, z, tau=0.4, orders=(2, 3, 4)):
    h0 = nspt.series_hamiltonian(u, p, z)
    dh = []
    for ns in (4, 8):
        u1, p1 = traj(u, p, z, tau / ns, ns)
        dh.append(nspt.series_hamiltonian(u1, p1, z) - h0)
    return np.array([dh[0][k] / dh[1][k] for k in orders]), dh


def test_energy_error_scales_as_dt_squared():
    u, z, eta, p = _setup(nt=5, seed=1)
    r, dh = _energy_ratios(nspt.md_trajectory, u, p, z)
    assert np.all((r > 3.5) & (r < 4.5)), r
    # orders 0 and 1 are conserved exactly (the vacuum is a stationary point)
    assert abs(dh[1][0]) < 1e-12 and abs(dh[1][1]) < 1e-12


def _planted(mistake):
    def traj(u, p, z, dt, nsteps):
        u = np.array(u)
        p = np.array(p)
        first = dt if mistake == "full_first_kick" else 0.5 * dt
        sign = -1.0 if mistake == "force_sign" else 1.0
        p = p + first * sign * nspt.md_forces(u, z)
        for i in range(nsteps):
            u = nspt.md_drift(u, p, 2 * dt if mistake == "double_drift" else dt)
            p = p + (dt if i < nsteps - 1 else 0.5 * dt) * sign * nspt.md_forces(u, z)
        return u, p
    return traj


@pytest.mark.parametrize("mistake", ["full_first_kick", "force_sign", "double_drift"])
def test_energy_check_catches_planted_mistakes(mistake):
    u, z, eta, p = _setup(nt=5, seed=1)
    r, _ = _energy_ratios(_planted(mistake), u, p, z)
    assert not np.all((r > 3.5) & (r < 4.5)), r


def test_series_action_is_the_taylor_expansion_of_the_dense_action():
    L, k, nt = 3, 1, 4
    u = _series_links(L, k, nt, 0.7, 3)
    z = tek.twist_tensor(L, k)
    s = nspt.series_action(u, z)
    errs = []
    for g in (0.05, 0.1):
        dense = np.stack([sum(g ** kk * u[mu, kk] for kk in range(nt + 1)) for mu in range(4)])
        errs.append(abs(tek.action(dense, z) - sum(g ** kk * s[kk] for kk in range(nt + 1))))
    # the remainder is O(g^(nt+1)): halving g divides it by about 2^(nt+1)
    assert errs[1] / errs[0] > 0.6 * 2 ** (nt + 1)


def test_trajectory_keeps_unitarity_and_traceless_hermitian_momenta():
    u, z, eta, p = _setup(nt=4, seed=4)
    u1, p1 = nspt.md_trajectory(u, p, z, 0.15, 3)
    n = u.shape[-1]
    for mu in range(4):
        assert np.allclose(ser.star(u1[mu], ser.dagger(u1[mu])), ser.identity(n, 4), atol=1e-11)
        assert np.allclose(p1[mu], ser.dagger(p1[mu]), atol=1e-12)
        assert np.abs(np.trace(p1[mu], axis1=-2, axis2=-1)).max() < 1e-11
    assert np.array_equal(u1[:, 0], u[:, 0])
    assert not np.any(p1[:, 0])


def test_trajectory_is_gauge_covariant():
    u, z, eta, p = _setup(nt=3, seed=5)
    n = u.shape[-1]
    om = np.linalg.qr(synth.rng_for(933).standard_normal((n, n)) + 1j * synth.rng_for(934).standard_normal((n, n)))[0]
    rot = lambda x: om @ x @ om.conj().T
    u1, p1 = nspt.md_trajectory(u, p, z, 0.2, 2)
    u2, p2 = nspt.md_trajectory(rot(u), rot(p), z, 0.2, 2)
    assert np.abs(u2 - rot(u1)).max() < 1e-12
    assert np.abs(p2 - rot(p1)).max() < 1e-11


def _dense_wilson(u, z, a, b):
    n = u.shape[-1]
    w = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            x = (np.linalg.matrix_power(u[mu], a) @ np.linalg.matrix_power(u[nu], b)
                 @ np.linalg.matrix_power(u[mu].conj().T, a) @ np.linalg.matrix_power(u[nu].conj().T, b))
            w += (z[mu, nu] ** (a * b) * np.trace(x)).real
    return w / (6 * n)


def test_plaquette_is_the_action():
    L, k, nt = 3, 1, 5
    u = _series_links(L, k, nt, 0.6, 11)
    z = tek.twist_tensor(L, k)
    w = nspt.wilson_loop_series(u, z, 1, 1)
    s = nspt.series_action(u, z)
    ref = -s / (12 * L * L)
    ref[0] += 1.0
    assert np.abs(w - ref).max() < 1e-13


@pytest.mark.parametrize("a,b", [(1, 1), (1, 2), (2, 2), (2, 3)])
def test_wilson_loops_are_one_at_the_vacuum(a, b):
    L, k, nt = 5, 2, 4
    u = synth.vacuum_links(L, k, nt)[0]
    w = nspt.wilson_loop_series(u, tek.twist_tensor(L, k), a, b)
    assert abs(w[0] - 1.0) < 1e-13 and np.abs(w[1:]).max() < 1e-13


@pytest.mark.parametrize("a,b", [(1, 2), (2, 2), (2, 3)])
def test_wilson_loop_series_is_the_taylor_expansion_of_the_dense_loop(a, b):
    # small g: the remainder is in its leading O(g^(nt+1)) regime
    L, k, nt = 3, 1, 4
    u = _series_links(L, k, nt, 0.3, 12)
    z = tek.twist_tensor(L, k)
    w = nspt.wilson_loop_series(u, z, a, b)
    errs = []
    for g in (0.01, 0.02):
        dense = np.stack([sum(g ** kk * u[mu, kk] for kk in range(nt + 1)) for mu in range(4)])
        errs.append(abs(_dense_wilson(dense, z, a, b) - sum(g ** kk * w[kk] for kk in range(nt + 1))))
    assert errs[1] / errs[0] > 0.6 * 2 ** (nt + 1)
