"""GPU parity at the benchmarked sizes, through the C ABI, against the FP64
oracle on the same seeded inputs the benchmark uses:

* the 64-product uneven batch (N in {64, 121, 169, 225, 289}, ntrunc in
  {15, 31, 63}, entries N(0,1) 0.7^k), one batched call, FP64 and split-BF16
  products, every product compared order by order;
* one replica of the NSPT Euler-Langevin step at N = 225 (L = 15, k = 4),
  ntrunc = 31 in all three product precisions, compared both on the updated
  links and on the increment U_new - U_old (the step changes the links by
  about eps F + sqrt(2 eps) eta, so the increment is the stricter test);
* a split-BF16 leapfrog trajectory at N = 81 (L = 9), ntrunc = 31;
* the opt-in finiteness check (PM_ERR_NONFINITE).

The measured maximum per-order errors are printed (pytest -s shows them).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nspt, series as ser, tek
import paper_2001_02835_amd as pm
from gpu_util import DEV, TOL, order_errors, to_dev, to_host
from nspt_util import series_links

pytestmark = pytest.mark.gpu

_CACHE = {}


def _cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


# ------------------------------------------------------- uneven 64-product batch

def _uneven_inputs():
    shapes = synth.uneven_batch_shapes(synth.rng_for(4, 0), 64)
    ops = []
    for i, (n, nt) in enumerate(shapes):
        a = synth.random_series(synth.rng_for(4, 1 + i, 0), n, nt, 0.7)
        b = synth.random_series(synth.rng_for(4, 1 + i, 1), n, nt, 0.7)
        ops.append((a, b))
    return shapes, ops


def _uneven_oracle():
    shapes, ops = _cached("uneven_inputs", _uneven_inputs)
    return [ser.star(a, b) for a, b in ops]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_uneven_64_product_batch(prec):
    shapes, ops = _cached("uneven_inputs", _uneven_inputs)
    refs = _cached("uneven_oracle", _uneven_oracle)
    items = []
    for a, b in ops:
        da = to_dev(a)
        items.append(dict(A=da, B=to_dev(b), C=torch.empty_like(da), scale=0.0))
    pm.polymat_mul_batched(items, precision=prec)
    worst, where = 0.0, None
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        if e.max() > worst:
            worst, where = float(e.max()), (i, shapes[i], int(e.argmax()))
        assert e.max() < TOL[prec], (i, shapes[i], e.max())
    print(f"uneven batch {prec}: max per-order error {worst:.3e} at (problem, (N, ntrunc), order) = {where}")


def test_uneven_64_product_batch_one_launch_pipeline(monkeypatch):
    """The same batch through the persistent one-launch pipeline
    (POLYMAT_PIPELINE=1): every step of every product in one launch, tickets
    ordered largest problem first and gated by per-problem counters."""
    monkeypatch.setenv("POLYMAT_PIPELINE", "1")
    shapes, ops = _cached("uneven_inputs", _uneven_inputs)
    refs = _cached("uneven_oracle", _uneven_oracle)
    items = []
    for a, b in ops:
        da = to_dev(a)
        items.append(dict(A=da, B=to_dev(b), C=torch.empty_like(da), scale=0.0))
    pm.timing_read()
    pm.timing_enable(True)
    pm.polymat_mul_batched(items, precision="fp64")
    torch.cuda.synchronize()
    pm.timing_enable(False)
    ph = pm.timing_read()
    assert ph["pipeline"][1] >= 2 and ph["product"][1] == 0     # set-up + one persistent launch
    worst = 0.0
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        worst = max(worst, float(e.max()))
        assert e.max() < TOL["fp64"], (i, shapes[i], e.max())
    print(f"uneven batch, one-launch pipeline: max per-order error {worst:.3e}")


@pytest.mark.parametrize("scale", [0.0, 1.0])
def test_pipeline_mixed_operand_forms_and_ragged_sizes(monkeypatch, scale):
    monkeypatch.setenv("POLYMAT_PIPELINE", "1")
    shapes = [(1, 0), (9, 7), (65, 15), (33, 63), (130, 31), (17, 3), (64, 1), (100, 5)]
    items, refs = [], []
    for i, (n, nt) in enumerate(shapes):
        a = synth.random_series(synth.rng_for(965, i, 0), n, nt, 0.8)
        b = synth.random_series(synth.rng_for(965, i, 1), n, nt, 0.8)
        op_a, op_b = i % 2, (i // 2) % 2
        refs.append(ser.star(ser.dagger(a) if op_a else a, ser.dagger(b) if op_b else b))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                          op_a=op_a, op_b=op_b, scale=scale))
    pm.polymat_mul_batched(items, precision="fp64")
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL["fp64"], (i, shapes[i], e.max())


def test_pipeline_bounded_wait_aborts_and_reports(monkeypatch):
    """With a spin limit of zero the first wait that is not already satisfied
    gives up: the launch sets its abort flag and every work-group leaves, so
    the kernel ends normally; with the finiteness check on the call reports
    PM_ERR_DEVICE, and the next call with the normal limit is correct."""
    monkeypatch.setenv("POLYMAT_PIPELINE", "1")
    n, nt = 96, 31
    a = synth.random_series(synth.rng_for(966, 0), n, nt, 0.5)
    b = synth.random_series(synth.rng_for(966, 1), n, nt, 0.5)
    da, db = to_dev(a), to_dev(b)
    ws = pm.workspace(pm.workspace_size(n, nt, "fp64"), DEV)
    monkeypatch.setenv("POLYMAT_PIPE_SPIN_LIMIT", "0")
    pm.check_enable(True)
    try:
        with pytest.raises(pm.PolymatError) as ei:
            pm.polymat_mul(da, db, precision="fp64", ws=ws)
        assert ei.value.status == pm.PM_ERR_DEVICE
    finally:
        pm.check_enable(False)
    monkeypatch.delenv("POLYMAT_PIPE_SPIN_LIMIT")
    c = to_host(pm.polymat_mul(da, db, precision="fp64", ws=ws))
    assert order_errors(c, ser.star(a, b)).max() < TOL["fp64"]


# ------------------------------------------------- NSPT step at N = 225, ntrunc 31

# tolerances of the updated links and of the increment U_new - U_old (orders
# >= 1), per precision of the mode-wise products; the measured values are
# recorded in the design notes
STEP_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-3}
INC_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-3}


def _step_inputs():
    L, k, nt = 15, 4, 31
    u = series_links(L, k, nt, 0.5, 15)
    eta = synth.langevin_noise(synth.rng_for(936), 1, L * L)
    return u, eta


def _step_oracle():
    u, eta = _cached("step_inputs", _step_inputs)
    return nspt.langevin_step_replicas(u, eta, tek.twist_tensor(15, 4), 0.01)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_step_paper_scale_all_precisions(prec):
    L, k, nt, eps = 15, 4, 31, 0.01
    u, eta = _cached("step_inputs", _step_inputs)
    ref = _cached("step_oracle", _step_oracle)
    du = to_dev(u)
    pm.nspt_langevin_step(du, to_dev(eta), pm.nspt_params(L, k, nt, eps), precision=prec)
    got = to_host(du)
    worst_u = max(order_errors(got[0, mu], ref[0, mu]).max() for mu in range(4))
    worst_d = max(order_errors(got[0, mu, 1:] - u[0, mu, 1:], ref[0, mu, 1:] - u[0, mu, 1:]).max()
                  for mu in range(4))
    print(f"N=225 ntrunc=31 step {prec}: links {worst_u:.3e}, increment {worst_d:.3e}")
    assert np.array_equal(got[0, :, 0], u[0, :, 0])
    assert worst_u < STEP_TOL[prec]
    assert worst_d < INC_TOL[prec]


# ------------------------------------------ split-BF16 MD trajectory at N = 81

def test_md_trajectory_bf16_n81_ntrunc31():
    L, k, nt, dt, nsteps = 9, 2, 31, 0.1, 2
    u = series_links(L, k, nt, 0.6, 3)
    eta = synth.langevin_noise(synth.rng_for(950, L, nt, 3), 1, L * L)
    z = tek.twist_tensor(L, k)
    p0 = np.stack([nspt.refresh_momentum(eta[0], nt)])
    ou, op = nspt.md_trajectory_replicas(u, p0, z, dt, nsteps)
    res = {}
    for prec in ("fp64", "bf16x3"):
        du, dp = to_dev(u), torch.empty(u.shape, dtype=torch.complex128, device=DEV)
        pm.nspt_md_trajectory(du, dp, pm.nspt_params(L, k, nt, dt), nsteps, eta=to_dev(eta), precision=prec)
        gu, gp = to_host(du), to_host(dp)
        eu = max(order_errors(gu[0, mu], ou[0, mu]).max() for mu in range(4))
        ed = max(order_errors(gu[0, mu, 1:] - u[0, mu, 1:], ou[0, mu, 1:] - u[0, mu, 1:]).max() for mu in range(4))
        ep = max(order_errors(gp[0, mu, 1:], op[0, mu, 1:]).max() for mu in range(4))
        res[prec] = (eu, ed, ep)
        print(f"N=81 ntrunc=31 MD {prec}: links {eu:.3e}, increment {ed:.3e}, momenta {ep:.3e}")
    assert max(res["fp64"]) < 1e-9
    assert max(res["bf16x3"]) < 1e-3


# -------------------------------------------------------- finiteness check

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("bad,scale", [(float("nan"), 0.0), (float("inf"), 0.0), (float("inf"), 1.0),
                                       (float("nan"), 1.25)])
def test_nonfinite_operand_reported_when_checked(prec, bad, scale):
    n, nt = 20, 7
    a = synth.random_series(synth.rng_for(960, 0), n, nt, 0.8)
    b = synth.random_series(synth.rng_for(960, 1), n, nt, 0.8)
    a_bad = a.copy()
    a_bad[3, 4, 5] = complex(bad, 0.0)
    pm.check_enable(True)
    try:
        # finite operands pass, and the result is the product
        c = to_host(pm.polymat_mul(to_dev(a), to_dev(b), precision=prec, scale=scale))
        assert order_errors(c, ser.star(a, b)).max() < TOL[prec]
        with pytest.raises(pm.PolymatError) as ei:
            pm.polymat_mul(to_dev(a_bad), to_dev(b), precision=prec, scale=scale)
        assert ei.value.status == pm.PM_ERR_NONFINITE
        # one bad problem in a batch is reported for the batch
        items = [dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                      scale=scale),
                 dict(A=to_dev(b), B=to_dev(a_bad), C=torch.empty((nt + 1, n, n), dtype=torch.complex128,
                                                                  device=DEV), scale=scale)]
        with pytest.raises(pm.PolymatError) as ei:
            pm.polymat_mul_batched(items, precision=prec)
        assert ei.value.status == pm.PM_ERR_NONFINITE
    finally:
        pm.check_enable(False)
    # check off: the call returns PM_OK and the result carries the NaN / Inf
    c = to_host(pm.polymat_mul(to_dev(a_bad), to_dev(b), precision=prec, scale=scale))
    assert not np.all(np.isfinite(c))


def test_check_mode_single_order_takes_checked_path():
    # ntrunc = 0 FP64 would take the direct form; with the check on it is
    # routed through the transform path so that the status words are written
    n = 12
    a = synth.random_series(synth.rng_for(961, 0), n, 0)
    b = synth.random_series(synth.rng_for(961, 1), n, 0)
    a_bad = a.copy()
    a_bad[0, 0, 0] = np.inf
    pm.check_enable(True)
    try:
        c = to_host(pm.polymat_mul(to_dev(a), to_dev(b)))
        assert order_errors(c, ser.star(a, b)).max() < TOL["fp64"]
        with pytest.raises(pm.PolymatError) as ei:
            pm.polymat_mul(to_dev(a_bad), to_dev(b))
        assert ei.value.status == pm.PM_ERR_NONFINITE
    finally:
        pm.check_enable(False)
