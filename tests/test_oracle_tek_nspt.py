"""Pins of the oracle's TEK model and NSPT step (CPU only).

The dense action of eq. (1) fixes the force: a finite-difference gradient
pins its sign and normalisation; the twisted vacuum pins the twist tensor;
the series force is pinned to the dense force by its Taylor expansion in g;
and the Langevin step is pinned by its closed form at the vacuum and by the
invariants it must keep (unitarity, Hermitian traceless drift, global gauge
covariance).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import synth
from oracle import nspt, series as ser, tek


def _links_near_vacuum(L, k, amp, seed):
    g = synth.twist_eaters(L, k)
    rng = synth.rng_for(910, seed)
    n = L * L
    return np.stack([sl.expm(1j * amp * synth.gue_traceless(rng, n)) @ g[m] for m in range(4)])


def _series_links(L, k, nt, amp, seed):
    """U_mu = exp(i sum_{k>=1} g^k A_{mu,k}) * Gamma_mu with traceless Hermitian A."""
    g = synth.twist_eaters(L, k)
    n = L * L
    rng = synth.rng_for(911, seed)
    u = np.zeros((4, nt + 1, n, n), dtype=np.complex128)
    for mu in range(4):
        x = np.zeros((nt + 1, n, n), dtype=np.complex128)
        for kk in range(1, nt + 1):
            x[kk] = amp ** kk * synth.gue_traceless(rng, n)
        gam = np.zeros_like(x)
        gam[0] = g[mu]
        u[mu] = ser.star(ser.series_exp(1j * x), gam)
    return u


@pytest.mark.parametrize("L,k", [(3, 1), (5, 2), (15, 4)])
def test_twist_eaters_solve_the_vacuum_condition(L, k):
    g = synth.twist_eaters(L, k)
    z = tek.twist_tensor(L, k)
    n = L * L
    for mu in range(4):
        assert np.allclose(g[mu] @ g[mu].conj().T, np.eye(n), atol=1e-13)
        assert np.isclose(np.linalg.det(g[mu]), 1.0, atol=1e-9)
        for nu in range(4):
            if mu != nu:
                p = z[mu, nu] * g[mu] @ g[nu] @ g[mu].conj().T @ g[nu].conj().T
                assert np.allclose(p, np.eye(n), atol=1e-12)


def test_twist_tensor_is_antisymmetric_in_the_exponent():
    z = tek.twist_tensor(15, 4)
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                assert np.isclose(z[nu, mu], np.conj(z[mu, nu]))
                assert np.isclose(abs(z[mu, nu]), 1.0)


def test_vacuum_has_zero_action_and_force():
    for L, k in [(3, 1), (5, 2)]:
        g = synth.twist_eaters(L, k)
        z = tek.twist_tensor(L, k)
        assert abs(tek.action(g, z)) < 1e-12
        for mu in range(4):
            assert np.abs(tek.force(g, z, mu)).max() < 1e-12


def test_force_is_minus_the_gradient_of_the_action():
    # d/dh S(exp(i h X) U_mu) at h = 0 equals -Tr[X F_mu]
    L, k = 3, 1
    u = _links_near_vacuum(L, k, 0.3, 1)
    z = tek.twist_tensor(L, k)
    rng = synth.rng_for(912)
    for mu in range(4):
        x = synth.gue_traceless(rng, L * L)
        h = 1e-5

        def s_at(t):
            v = u.copy()
            v[mu] = sl.expm(1j * t * x) @ u[mu]
            return tek.action(v, z)

        fd = (s_at(h) - s_at(-h)) / (2 * h)
        f = tek.force(u, z, mu)
        assert np.allclose(f, f.conj().T, atol=1e-12)
        assert abs(np.trace(f)) < 1e-12
        assert abs(fd - (-np.trace(x @ f).real)) < 1e-6 * max(1.0, abs(fd))


def test_printed_minus_sign_fails_the_gradient_check():
    # planted in a copy: the staple's second term with the printed minus sign
    L, k = 3, 1
    u = _links_near_vacuum(L, k, 0.3, 2)
    z = tek.twist_tensor(L, k)

    def staple_minus(uu, mu):
        ud = np.conj(np.swapaxes(uu, -1, -2))
        acc = np.zeros_like(uu[mu])
        for nu in range(4):
            if nu != mu:
                acc += z[mu, nu] * (uu[nu] @ ud[mu] @ ud[nu])
                acc -= np.conj(z[mu, nu]) * (ud[nu] @ ud[mu] @ uu[nu])
        return uu[mu] @ acc

    rng = synth.rng_for(913)
    x = synth.gue_traceless(rng, L * L)
    h = 1e-5

    def s_at(t):
        v = u.copy()
        v[0] = sl.expm(1j * t * x) @ u[0]
        return tek.action(v, z)

    fd = (s_at(h) - s_at(-h)) / (2 * h)
    bad = tek.project_force(staple_minus(u, 0))
    assert abs(fd - (-np.trace(x @ bad).real)) > 1e-3


def test_series_force_is_the_taylor_expansion_of_the_dense_force():
    L, k, nt = 3, 1, 3
    u = _series_links(L, k, nt, 0.8, 3)
    z = tek.twist_tensor(L, k)
    for mu in (0, 2):
        f = nspt.series_force(u, z, mu)
        errs = []
        for gval in (0.02, 0.01):
            ug = np.stack([sum(gval ** kk * u[m, kk] for kk in range(nt + 1)) for m in range(4)])
            dense = tek.force(ug, z, mu)
            approx = sum(gval ** kk * f[kk] for kk in range(nt + 1))
            errs.append(np.abs(dense - approx).max())
        assert errs[0] / errs[1] > 0.6 * 2 ** (nt + 1)


def test_series_force_hermitian_traceless_every_order():
    L, k, nt = 3, 1, 4
    u = _series_links(L, k, nt, 0.7, 4)
    z = tek.twist_tensor(L, k)
    for mu in range(4):
        f = nspt.series_force(u, z, mu)
        for kk in range(nt + 1):
            assert np.allclose(f[kk], f[kk].conj().T, atol=1e-12)
            assert abs(np.trace(f[kk])) < 1e-11
        assert np.abs(f[0]).max() < 1e-12          # vacuum at order 0


def test_step_from_vacuum_closed_form():
    # U = Gamma: F == 0 at every order, so U'^(m) = (i sqrt(2 eps) eta)^m / m! Gamma
    L, k, nt, eps = 3, 1, 6, 0.02
    u = synth.vacuum_links(L, k, nt)[0]
    z = tek.twist_tensor(L, k)
    eta = synth.langevin_noise(synth.rng_for(914), 1, L * L)[0]
    new = nspt.langevin_step(u, eta, z, eps)
    for mu in range(4):
        a = 1j * np.sqrt(2 * eps) * eta[mu]
        term = np.eye(L * L, dtype=np.complex128)
        for m in range(nt + 1):
            assert np.allclose(new[mu, m], term @ u[mu, 0], atol=1e-14)
            term = term @ a / (m + 1)


def test_step_keeps_unitarity_order_by_order_and_order_zero():
    L, k, nt, eps = 3, 1, 5, 0.05
    u = _series_links(L, k, nt, 0.5, 5)
    z = tek.twist_tensor(L, k)
    rng = synth.rng_for(915)
    for _ in range(2):
        eta = synth.langevin_noise(rng, 1, L * L)[0]
        new = nspt.langevin_step(u, eta, z, eps)
        assert np.array_equal(new[:, 0], u[:, 0])
        u = new
    for mu in range(4):
        uu = ser.star(u[mu], ser.dagger(u[mu]))
        assert np.allclose(uu, ser.identity(L * L, nt), atol=1e-11)


def test_drift_noise_is_traceless_hermitian_with_zero_order0():
    L, k, nt, eps = 3, 1, 4, 0.03
    u = _series_links(L, k, nt, 0.6, 6)
    z = tek.twist_tensor(L, k)
    eta = synth.langevin_noise(synth.rng_for(916), 1, L * L)[0]
    for mu in range(4):
        x = nspt.drift_noise(nspt.series_force(u, z, mu), eta[mu], eps)
        assert np.array_equal(x[0], np.zeros_like(x[0]))
        for kk in range(nt + 1):
            assert np.allclose(x[kk], x[kk].conj().T, atol=1e-12)
            assert abs(np.trace(x[kk])) < 1e-11


def test_step_is_gauge_covariant():
    # U_mu -> W U_mu W^+, eta -> W eta W^+ commutes with the step
    L, k, nt, eps = 3, 1, 3, 0.04
    u = _series_links(L, k, nt, 0.6, 7)
    z = tek.twist_tensor(L, k)
    n = L * L
    rng = synth.rng_for(917)
    eta = synth.langevin_noise(rng, 1, n)[0]
    w = sl.expm(1j * synth.gue_traceless(rng, n))
    wd = w.conj().T
    ut = np.einsum("ij,mkjl,lp->mkip", w, u, wd)
    etat = np.einsum("ij,mjl,lp->mip", w, eta, wd)
    a = nspt.langevin_step(ut, etat, z, eps)
    b = np.einsum("ij,mkjl,lp->mkip", w, nspt.langevin_step(u, eta, z, eps), wd)
    assert np.allclose(a, b, atol=1e-11)


def test_replica_batch_is_independent():
    L, k, nt, eps = 3, 1, 2, 0.05
    z = tek.twist_tensor(L, k)
    u = np.stack([_series_links(L, k, nt, 0.5, 20 + r) for r in range(2)])
    eta = synth.langevin_noise(synth.rng_for(918), 2, L * L)
    both = nspt.langevin_step_replicas(u, eta, z, eps)
    for r in range(2):
        assert np.array_equal(both[r], nspt.langevin_step(u[r], eta[r], z, eps))
