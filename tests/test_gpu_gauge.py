"""GPU parity of the stochastic gauge-fixing step (nspt_gauge_fix) against the
FP64 oracle, through the C ABI, plus what holds at any size: the closed-form
first-order damping of a pure-gauge eigenmode, invariance of the action,
unitarity, and alpha = 0 leaving the links untouched."""
import numpy as np
import pytest

import synth
from oracle import nspt, series as ser
import paper_2001_02835_amd as pm
from gpu_util import order_errors, to_dev, to_host
from nspt_util import series_links

pytestmark = pytest.mark.gpu

STEP_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-3}
ALPHA = 0.1


def _gpu_fix(u, L, k, nt, alpha, prec="fp64"):
    du = to_dev(u)
    pm.nspt_gauge_fix(du, pm.nspt_params(L, k, nt, 0.01), alpha, precision=prec)
    return to_host(du)


@pytest.mark.parametrize("L,k,nt,R", [(3, 1, 5, 2), (5, 2, 7, 1), (3, 1, 1, 1), (3, 1, 0, 1), (5, 1, 15, 1),
                                      (7, 2, 31, 1), (1, 0, 3, 1), (3, 1, 63, 1)])
def test_gauge_fix_matches_oracle(L, k, nt, R):
    u = series_links(L, k, nt, 0.6, 21, replicas=R)
    got = _gpu_fix(u, L, k, nt, ALPHA)
    ref = nspt.gauge_fix_replicas(u, ALPHA)
    for r in range(R):
        for mu in range(4):
            e = order_errors(got[r, mu], ref[r, mu])
            print(f"L={L} nt={nt} r={r} mu={mu}: err {e.max():.2e}")
            assert e.max() < STEP_TOL["fp64"], (r, mu, e)
            assert np.array_equal(got[r, mu, 0], u[r, mu, 0])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_gauge_fix_precisions(prec):
    L, k, nt = 5, 2, 15
    u = series_links(L, k, nt, 0.6, 22)
    got = _gpu_fix(u, L, k, nt, ALPHA, prec)
    ref = nspt.gauge_fix_replicas(u, ALPHA)
    worst = max(order_errors(got[0, mu], ref[0, mu]).max() for mu in range(4))
    print(f"{prec}: worst per-order error {worst:.2e}")
    assert worst < STEP_TOL[prec]


def _pure_gauge(L, k, nt, w):
    gam = synth.twist_eaters(L, k)
    n = L * L
    y = np.zeros((nt + 1, n, n), dtype=np.complex128)
    y[1] = 1j * w
    om = ser.series_exp(y)
    u = np.zeros((1, 4, nt + 1, n, n), dtype=np.complex128)
    for mu in range(4):
        g0 = np.zeros_like(y)
        g0[0] = gam[mu]
        u[0, mu] = ser.star(ser.star(om, g0), ser.dagger(om))
    return u, gam


@pytest.mark.parametrize("L,k,nt,a,b", [(5, 2, 7, 0, 2), (15, 4, 7, 1, 3), (15, 4, 7, 0, 0)])
def test_pure_gauge_mode_is_damped_by_one_minus_alpha_lambda(L, k, nt, a, b):
    gam = synth.twist_eaters(L, k)
    j = gam[a] @ gam[b]
    lam = 0.0
    for nu in range(4):
        c = gam[nu] @ j @ gam[nu].conj().T
        phi = np.vdot(j, c) / np.vdot(j, j)
        assert np.abs(c - phi * j).max() < 1e-12
        lam += abs(1.0 - phi) ** 2
    assert lam > 0.1
    w = (j + j.conj().T) / np.sqrt(L * L)
    u, _ = _pure_gauge(L, k, nt, w)
    got = _gpu_fix(u, L, k, nt, ALPHA)
    # directions whose twist eater commutes with the mode have U^(1) = 0:
    # measure against the largest first-order coefficient
    scale = max(np.linalg.norm(u[0, mu, 1]) for mu in range(4))
    for mu in range(4):
        e = np.linalg.norm(got[0, mu, 1] - (1.0 - ALPHA * lam) * u[0, mu, 1]) / scale
        assert e < 1e-12, (mu, e, lam)


def test_action_and_unitarity_kept_at_full_size():
    L, k, nt = 15, 4, 31
    n = L * L
    u = series_links(L, k, nt, 0.5, 23)
    prm = pm.nspt_params(L, k, nt, 0.01)
    du = to_dev(u)
    s0 = to_host(pm.nspt_action(du, prm))[0]
    pm.nspt_gauge_fix(du, prm, ALPHA)
    gu = to_host(du)
    s1 = to_host(pm.nspt_action(du, prm))[0]
    assert order_errors(gu[0, 0], u[0, 0]).max() > 1e-3             # the links moved
    # the action series is gauge invariant: its change at every order is
    # compared with the largest order
    scale = np.abs(s0).max()
    print("max |S1 - S0| / max |S0|:", np.abs(s1 - s0).max() / scale)
    assert np.abs(s1 - s0).max() < 1e-9 * scale
    for mu in range(4):
        ud = ser.dagger(gu[0, mu])
        uu = to_host(pm.polymat_mul(du[0, mu].contiguous(), to_dev(ud)))
        c = ser.order_norm_bound(gu[0, mu], ud)
        e = np.sqrt(np.sum(np.abs(uu - ser.identity(n, nt)) ** 2, axis=(-2, -1))) / c
        assert e.max() < 1e-12, (mu, e)


def test_zero_alpha_leaves_links_untouched():
    L, k, nt = 5, 2, 7
    u = series_links(L, k, nt, 0.6, 24)
    got = _gpu_fix(u, L, k, nt, 0.0)
    assert np.array_equal(got, u)
