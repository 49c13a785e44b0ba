"""GPU parity of the counter-based Langevin noise (nspt_noise) and of runs of
Langevin steps that draw it on the device (nspt_langevin_steps) against the
oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import nspt, tek
import paper_2001_02835_amd as pm
from gpu_util import DEV, order_errors, to_dev, to_host
from nspt_util import series_links

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("R,n,seed,step", [(2, 9, 5, 3), (1, 1, 7, 0), (1, 17, 2**63 + 1, 2**40), (2, 225, 123, 9)])
def test_noise_matches_oracle(R, n, seed, step):
    got = to_host(pm.nspt_noise(R, n, seed, step, DEV))
    ref = nspt.philox_noise(seed, step, R, n)
    err = np.abs(got - ref).max()
    print(f"R={R} n={n}: max |eta - eta_ref| = {err:.2e}")
    assert err < 1e-13
    assert np.array_equal(got, got.conj().transpose(0, 1, 3, 2))          # exactly Hermitian
    assert np.abs(np.trace(got, axis1=-2, axis2=-1)).max() < 1e-12


@pytest.mark.parametrize("L,k,nt,R", [(3, 1, 7, 2), (5, 2, 15, 1)])
def test_steps_match_oracle(L, k, nt, R):
    eps, seed, step0, nsteps = 0.05, 11, 100, 2
    u = series_links(L, k, nt, 0.6, 40 + L, replicas=R)
    du = to_dev(u)
    pm.nspt_langevin_steps(du, pm.nspt_params(L, k, nt, eps), seed, step0, nsteps)
    got = to_host(du)
    ref = nspt.langevin_steps_philox(u, tek.twist_tensor(L, k), eps, seed, step0, nsteps)
    for r in range(R):
        for mu in range(4):
            e = order_errors(got[r, mu], ref[r, mu])
            assert e.max() < 1e-10, (r, mu, e)


def test_one_step_equals_the_step_with_the_same_noise():
    L, k, nt, R, eps = 5, 2, 7, 2, 0.05
    u = series_links(L, k, nt, 0.6, 50, replicas=R)
    prm = pm.nspt_params(L, k, nt, eps)
    a = to_dev(u)
    pm.nspt_langevin_steps(a, prm, 3, 17, 1)
    b = to_dev(u)
    pm.nspt_langevin_step(b, pm.nspt_noise(R, L * L, 3, 17, DEV), prm)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
