"""GPU parity of the NSPT Euler-Langevin step (nspt_langevin_step) against
the FP64 oracle step, through the C ABI, plus the invariants the step keeps."""
import numpy as np
import pytest
import torch

import synth
from oracle import nspt, series as ser, tek
import paper_2001_02835_amd as pm
from gpu_util import DEV, order_errors, to_dev, to_host
from nspt_util import series_links

pytestmark = pytest.mark.gpu

# per-order tolerance of the updated links against the oracle step
STEP_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-3}


def gpu_step(u, eta, L, k, nt, eps, prec="fp64"):
    du = to_dev(u)
    pm.nspt_langevin_step(du, to_dev(eta), pm.nspt_params(L, k, nt, eps), precision=prec)
    return to_host(du)


@pytest.mark.parametrize("L,k,nt,R", [(3, 1, 7, 2), (5, 2, 5, 1), (3, 1, 0, 1), (3, 1, 1, 1), (5, 1, 15, 1),
                                      (1, 0, 3, 1), (7, 2, 31, 1), (3, 1, 63, 1)])
def test_step_matches_oracle(L, k, nt, R):
    eps = 0.05
    u = series_links(L, k, nt, 0.6, L * 100 + nt, replicas=R)
    eta = synth.langevin_noise(synth.rng_for(931, L, nt), R, L * L)
    got = gpu_step(u, eta, L, k, nt, eps)
    ref = nspt.langevin_step_replicas(u, eta, tek.twist_tensor(L, k), eps)
    for r in range(R):
        for mu in range(4):
            e = order_errors(got[r, mu], ref[r, mu])
            assert e.max() < STEP_TOL["fp64"], (r, mu, e)
            assert np.array_equal(got[r, mu, 0], u[r, mu, 0])      # order 0 untouched


def test_step_from_vacuum_closed_form():
    L, k, nt, eps = 3, 1, 7, 0.02
    n = L * L
    u = synth.vacuum_links(L, k, nt, replicas=1)
    eta = synth.langevin_noise(synth.rng_for(932), 1, n)
    got = gpu_step(u, eta, L, k, nt, eps)
    for mu in range(4):
        a = 1j * np.sqrt(2 * eps) * eta[0, mu]
        term = np.eye(n, dtype=np.complex128)
        ref = np.empty((nt + 1, n, n), dtype=np.complex128)
        for m in range(nt + 1):
            ref[m] = term @ u[0, mu, 0]
            term = term @ a / (m + 1)
        assert order_errors(got[0, mu], ref).max() < 1e-11


def test_steps_keep_unitarity_and_order_zero():
    L, k, nt, eps = 5, 2, 7, 0.05
    n = L * L
    u = synth.vacuum_links(L, k, nt, replicas=2)
    du = to_dev(u)
    rng = synth.rng_for(933)
    prm = pm.nspt_params(L, k, nt, eps)
    for _ in range(4):
        pm.nspt_langevin_step(du, to_dev(synth.langevin_noise(rng, 2, n)), prm)
    got = to_host(du)
    assert np.array_equal(got[:, :, 0], u[:, :, 0])
    for r in range(2):
        for mu in range(4):
            uu = ser.star(got[r, mu], ser.dagger(got[r, mu]))
            err = np.abs(uu - ser.identity(n, nt))
            scale = ser.order_norm_bound(got[r, mu], got[r, mu])
            for kk in range(nt + 1):
                assert err[kk].max() <= 1e-11 * max(scale[kk], 1.0), (r, mu, kk)


def test_step_is_gauge_covariant_on_gpu():
    L, k, nt, eps = 3, 1, 5, 0.05
    n = L * L
    u = series_links(L, k, nt, 0.6, 7)
    rng = synth.rng_for(934)
    eta = synth.langevin_noise(rng, 1, n)
    import scipy.linalg as sl
    w = sl.expm(1j * synth.gue_traceless(rng, n))
    wd = w.conj().T
    ut = np.einsum("ij,rmkjl,lp->rmkip", w, u, wd)
    etat = np.einsum("ij,rmjl,lp->rmip", w, eta, wd)
    a = gpu_step(ut, etat, L, k, nt, eps)
    b = np.einsum("ij,rmkjl,lp->rmkip", w, gpu_step(u, eta, L, k, nt, eps), wd)
    for mu in range(4):
        assert order_errors(a[0, mu], b[0, mu]).max() < 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_step_precisions(prec):
    L, k, nt, eps = 5, 2, 7, 0.05
    u = series_links(L, k, nt, 0.6, 11)
    eta = synth.langevin_noise(synth.rng_for(935), 1, L * L)
    got = gpu_step(u, eta, L, k, nt, eps, prec)
    ref = nspt.langevin_step_replicas(u, eta, tek.twist_tensor(L, k), eps)
    worst = max(order_errors(got[0, mu], ref[0, mu]).max() for mu in range(4))
    print(f"{prec}: worst per-order error of the step {worst:.3e}")
    assert worst < STEP_TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nt", [7, 31])
def test_step_one_by_one_matrices_reduced_precisions(prec, nt):
    # N = 1 (L = 1): the split-BF16 rows are padded to 8 entries, so the copies
    # of Y^b at the shorter Horner lengths are larger than a product result
    L, k, eps = 1, 0, 0.05
    u = series_links(L, k, nt, 0.6, 17)
    eta = synth.langevin_noise(synth.rng_for(937, nt), 1, 1)
    got = gpu_step(u, eta, L, k, nt, eps, prec)
    ref = nspt.langevin_step_replicas(u, eta, tek.twist_tensor(L, k), eps)
    worst = max(order_errors(got[0, mu], ref[0, mu]).max() for mu in range(4))
    assert worst < STEP_TOL[prec], worst
