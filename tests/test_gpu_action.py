"""GPU parity of the action series (nspt_action, the plaquette observable)
against the oracle's series action, which is pinned to the dense action of
eq. (1) by its Taylor expansion in g."""
import numpy as np
import pytest

import synth
from oracle import nspt, series as ser, tek
import paper_2001_02835_amd as pm
from gpu_util import to_dev
from nspt_util import series_links

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 1e-4}


def _scale(u):
    """B_k = sum_{mu<nu} 2 sqrt(N) c_k, c the norm bound of the four-fold product
    (|Tr X| <= sqrt(N) ||X||_F): the size of the terms that make up S^(k)."""
    n = u.shape[-1]
    nrm = np.sqrt(np.sum(np.abs(u) ** 2, axis=(-2, -1)))       # [4, nord]
    nord = u.shape[1]
    b = np.zeros(nord)
    for m in range(4):
        for q in range(m + 1, 4):
            c = nrm[m]
            for f in (nrm[q], nrm[m], nrm[q]):
                c = np.convolve(c, f)[:nord]
            b += 2 * np.sqrt(n) * c
    b[0] += 12 * n
    return b


@pytest.mark.parametrize("L,k,nt,R", [(3, 1, 7, 2), (5, 2, 15, 1), (9, 2, 31, 1), (3, 1, 63, 1)])
def test_action_matches_oracle(L, k, nt, R):
    u = series_links(L, k, nt, 0.6, 40 + L, replicas=R)
    z = tek.twist_tensor(L, k)
    got = pm.nspt_action(to_dev(u), pm.nspt_params(L, k, nt, 0.01)).cpu().numpy()
    for r in range(R):
        ref = nspt.series_action(u[r], z)
        err = np.abs(got[r] - ref) / _scale(u[r])
        assert err.max() < TOL["fp64"], (r, err)


def test_action_vanishes_at_the_vacuum():
    L, k, nt = 5, 2, 7
    u = synth.vacuum_links(L, k, nt, replicas=2)
    got = pm.nspt_action(to_dev(u), pm.nspt_params(L, k, nt, 0.01)).cpu().numpy()
    assert np.abs(got).max() < 1e-11 * 12 * L * L


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_action_precisions(prec):
    L, k, nt = 5, 2, 15
    u = series_links(L, k, nt, 0.6, 45)
    got = pm.nspt_action(to_dev(u), pm.nspt_params(L, k, nt, 0.01), precision=prec).cpu().numpy()
    ref = nspt.series_action(u[0], tek.twist_tensor(L, k))
    err = np.abs(got[0] - ref) / _scale(u[0])
    assert err.max() < TOL[prec], err


@pytest.mark.parametrize("a,b", [(1, 1), (1, 2), (2, 2), (2, 3), (4, 1)])
def test_wilson_loops_match_oracle(a, b):
    L, k, nt, R = 5, 2, 7, 2
    u = series_links(L, k, nt, 0.6, 47, replicas=R)
    z = tek.twist_tensor(L, k)
    got = pm.nspt_wilson_loop(to_dev(u), pm.nspt_params(L, k, nt, 0.01), a, b).cpu().numpy()
    for r in range(R):
        ref = nspt.wilson_loop_series(u[r], z, a, b)
        # terms of W^(k) are bounded by the 4-fold norm convolution of the powers, / (6N) * sqrt(N)
        err = np.abs(got[r] - ref)
        assert err.max() < 1e-11 * max(1.0, np.abs(ref).max()), (r, err)


def test_wilson_loops_at_the_vacuum_and_plaquette_relation():
    L, k, nt = 15, 4, 31
    u = synth.vacuum_links(L, k, nt, replicas=1)
    prm = pm.nspt_params(L, k, nt, 0.01)
    for a, b in [(1, 1), (2, 2), (3, 2)]:
        w = pm.nspt_wilson_loop(to_dev(u), prm, a, b).cpu().numpy()[0]
        assert abs(w[0] - 1.0) < 1e-12 and np.abs(w[1:]).max() < 1e-12, (a, b)
    us = series_links(L, k, 15, 0.5, 48)
    prm = pm.nspt_params(L, k, 15, 0.01)
    w = pm.nspt_wilson_loop(to_dev(us), prm, 1, 1).cpu().numpy()[0]
    s = pm.nspt_action(to_dev(us), prm).cpu().numpy()[0]
    ref = -s / (12 * L * L)
    ref[0] += 1.0
    assert np.abs(w - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
