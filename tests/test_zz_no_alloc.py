"""The allocation-free product entry point (polymat_mul_noalloc) against
polymat_mul, through the C ABI: two calls in a row on the library's
built-in scratch array, the second with a smaller input, each compared with
the workspace form (same kernels, so the results agree bitwise) and with the
FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import series as ser
import paper_2001_02835_amd as pm
from gpu_util import TOL, order_errors, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_workspace_form_two_calls(prec):
    for n, nt, r in ((225, 31, 0.5), (40, 7, 0.9)):      # the second call is smaller
        a = synth.random_series(synth.rng_for(970, n, 0), n, nt, r)
        b = synth.random_series(synth.rng_for(970, n, 1), n, nt, r)
        da, db = to_dev(a), to_dev(b)
        want = to_host(pm.polymat_mul(da, db, precision=prec))
        got = to_host(pm.polymat_mul_noalloc(da, db, precision=prec))
        assert np.array_equal(got, want), (prec, n, nt)
        assert order_errors(got, ser.star(a, b)).max() < TOL[prec], (prec, n, nt)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    n, nt = 300, 63
    need = pm.workspace_size(n, nt, "fp64")
    assert need > pm.NOALLOC_SCRATCH_BYTES
    a = torch.zeros((nt + 1, n, n), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(pm.PolymatError) as ei:
        pm.polymat_mul_noalloc(a, a.clone())
    assert ei.value.status == pm.PM_ERR_UNSUPPORTED
