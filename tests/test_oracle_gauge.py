"""Pins of the oracle's stochastic gauge-fixing step (CPU only).

The step U_mu <- Omega U_mu Omega^+, Omega = exp(Y) with
Y = -(alpha/2) [(G - G^+) - Tr/N], G = sum_mu (U_mu Gamma_mu^+ - Gamma_mu^+ U_mu),
is pinned by: the closed-form damping 1 - alpha lambda of a pure-gauge
eigenmode at first order (lambda the reduced-model lattice Laplacian of the
mode, from the twist phases); the Taylor expansion of the same step written
with dense matrices and a matrix exponential; the ascent of the Landau
functional sum_mu Re Tr(U_mu Gamma_mu^+) under the dense step; and the
invariants (action and Wilson loops unchanged, unitarity kept, vacuum and
alpha = 0 left alone).  Planted mistakes in a copy of the generator break
the damping pin.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import nspt, series as ser, tek


def _series_links(L, k, nt, amp, seed):
    g = synth.twist_eaters(L, k)
    n = L * L
    rng = synth.rng_for(960, seed)
    u = np.zeros((4, nt + 1, n, n), dtype=np.complex128)
    for mu in range(4):
        x = np.zeros((nt + 1, n, n), dtype=np.complex128)
        for kk in range(1, nt + 1):
            x[kk] = amp ** kk * synth.gue_traceless(rng, n)
        gam = np.zeros_like(x)
        gam[0] = g[mu]
        u[mu] = ser.star(ser.series_exp(1j * x), gam)
    return u


def _pure_gauge(L, k, nt, w):
    """U_mu = Omega0 * Gamma_mu * Omega0^+ with Omega0 = exp(i w g)."""
    gam = synth.twist_eaters(L, k)
    n = L * L
    y = np.zeros((nt + 1, n, n), dtype=np.complex128)
    y[1] = 1j * w
    om = ser.series_exp(y)
    u = np.zeros((4, nt + 1, n, n), dtype=np.complex128)
    for mu in range(4):
        g0 = np.zeros_like(y)
        g0[0] = gam[mu]
        u[mu] = ser.star(ser.star(om, g0), ser.dagger(om))
    return u, gam


def _mode(gam, a, b):
    """J = Gamma_a Gamma_b: every conjugation by a twist eater multiplies it by
    a phase (the twist eaters commute up to phases)."""
    return gam[a] @ gam[b]


def _laplacian_eigenvalue(gam, j):
    lam = 0.0
    for nu in range(4):
        c = gam[nu] @ j @ gam[nu].conj().T
        phi = np.vdot(j, c) / np.vdot(j, j)
        assert np.abs(c - phi * j).max() < 1e-12          # J is an eigenvector
        lam += abs(1.0 - phi) ** 2
    return lam


@pytest.mark.parametrize("a,b", [(0, 0), (0, 2), (1, 3)])
@pytest.mark.parametrize("alpha", [0.05, 0.2])
def test_first_order_pure_gauge_mode_is_damped_by_one_minus_alpha_lambda(a, b, alpha):
    L, k, nt = 3, 1, 3
    gam = synth.twist_eaters(L, k)
    j = _mode(gam, a, b)
    assert abs(np.trace(j)) < 1e-12
    w = j + j.conj().T
    lam = _laplacian_eigenvalue(gam, j)
    assert lam > 0.5
    u, _ = _pure_gauge(L, k, nt, w)
    u1 = nspt.gauge_fix(u, alpha)
    assert np.abs(u1[:, 1] - (1.0 - alpha * lam) * u[:, 1]).max() < 1e-13
    assert np.array_equal(u1[:, 0], u[:, 0])


def _planted_exponent(mistake):
    def y(u, alpha):
        g = nspt.gauge_generator(u)
        if mistake == "one_sided":
            g = np.zeros_like(u[0])
            for mu in range(4):
                v = np.zeros_like(u[mu]); v[0] = u[mu, 0]
                g += ser.star(u[mu], ser.dagger(v))
        n = u.shape[-1]
        d = g - ser.dagger(g)
        tr = np.trace(d, axis1=-2, axis2=-1)
        f = {"sign": 0.5, "no_half": -1.0}.get(mistake, -0.5)
        out = f * alpha * (d - tr[:, None, None] / n * np.eye(n)[None])
        out[0] = 0.0
        return out
    return y


@pytest.mark.parametrize("mistake", ["sign", "no_half", "one_sided"])
def test_planted_mistakes_break_the_damping_pin(mistake):
    L, k, nt, alpha = 3, 1, 3, 0.1
    gam = synth.twist_eaters(L, k)
    j = _mode(gam, 0, 2)
    w = j + j.conj().T
    lam = _laplacian_eigenvalue(gam, j)
    u, _ = _pure_gauge(L, k, nt, w)
    om = ser.series_exp(_planted_exponent(mistake)(u, alpha))
    u1 = np.stack([ser.star(ser.star(om, u[mu]), ser.dagger(om)) for mu in range(4)])
    assert np.abs(u1[:, 1] - (1.0 - alpha * lam) * u[:, 1]).max() > 1e-3


def _dense_step(u, gam, alpha):
    n = u.shape[-1]
    g = sum(u[mu] @ gam[mu].conj().T - gam[mu].conj().T @ u[mu] for mu in range(4))
    d = g - g.conj().T
    y = -0.5 * alpha * (d - np.trace(d) / n * np.eye(n))
    om = scipy.linalg.expm(y)
    return np.stack([om @ u[mu] @ om.conj().T for mu in range(4)])


def test_series_step_is_the_taylor_expansion_of_the_dense_step():
    L, k, nt, alpha = 3, 1, 4, 0.3
    u = _series_links(L, k, nt, 0.5, 1)
    gam = synth.twist_eaters(L, k)
    u1 = nspt.gauge_fix(u, alpha)
    errs = []
    for g in (0.01, 0.02):
        dense = np.stack([sum(g ** kk * u[mu, kk] for kk in range(nt + 1)) for mu in range(4)])
        ser_sum = np.stack([sum(g ** kk * u1[mu, kk] for kk in range(nt + 1)) for mu in range(4)])
        errs.append(np.abs(_dense_step(dense, gam, alpha) - ser_sum).max())
    # the remainder is O(g^(nt+1)): doubling g multiplies it by about 2^(nt+1)
    assert errs[1] / errs[0] > 0.6 * 2 ** (nt + 1), errs


def test_dense_step_climbs_the_landau_functional():
    L, k = 3, 1
    gam = synth.twist_eaters(L, k)
    n = L * L
    rng = synth.rng_for(961)
    u = np.stack([scipy.linalg.expm(0.2j * synth.gue_traceless(rng, n)) @ gam[mu] for mu in range(4)])
    f = lambda x: sum(np.trace(x[mu] @ gam[mu].conj().T).real for mu in range(4))
    f0 = f(u)
    for alpha in (0.01, 0.05):
        assert f(_dense_step(u, gam, alpha)) > f0


def test_step_keeps_action_wilson_loops_and_unitarity():
    L, k, nt = 3, 1, 5
    u = _series_links(L, k, nt, 0.6, 2)
    z = tek.twist_tensor(L, k)
    u1 = nspt.gauge_fix(u, 0.3)
    assert np.abs(u1 - u).max() > 1e-3                       # it does move the links
    assert np.abs(nspt.series_action(u1, z) - nspt.series_action(u, z)).max() < 1e-11
    assert np.abs(nspt.wilson_loop_series(u1, z, 1, 2) - nspt.wilson_loop_series(u, z, 1, 2)).max() < 1e-12
    n = L * L
    for mu in range(4):
        assert np.abs(ser.star(u1[mu], ser.dagger(u1[mu])) - ser.identity(n, nt)).max() < 1e-12


def test_vacuum_and_zero_alpha_are_left_alone():
    L, k, nt = 3, 1, 4
    vac = synth.vacuum_links(L, k, nt)[0]
    assert np.abs(nspt.gauge_fix(vac, 0.4) - vac).max() < 1e-15
    u = _series_links(L, k, nt, 0.5, 3)
    assert np.abs(nspt.gauge_fix(u, 0.0) - u).max() < 1e-15


def test_repeated_steps_shrink_the_gauge_generator():
    L, k, nt = 3, 1, 3
    u = _series_links(L, k, nt, 0.5, 4)
    norms = []
    for _ in range(4):
        y = nspt.gauge_exponent(u, 1.0)
        norms.append(np.abs(y[1]).max())
        u = nspt.gauge_fix(u, 0.1)
    assert all(b < a for a, b in zip(norms, norms[1:])), norms
