"""The entry points enqueue kernels only, so a call captured into a HIP graph
replays to the eager result (bitwise: the same kernels in the same order).
Each replay is checked, with eager work and synchronisations in between."""
import numpy as np
import pytest
import torch

import synth
import paper_2001_02835_amd as pm
from gpu_util import DEV, to_dev
from nspt_util import series_links

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def test_batched_product_graph_replays():
    items = []
    for i, (n, nt) in enumerate([(33, 7), (64, 15), (17, 3)]):
        a = to_dev(synth.random_series(synth.rng_for(60, i, 0), n, nt, 0.8))
        b = to_dev(synth.random_series(synth.rng_for(60, i, 1), n, nt, 0.8))
        items.append(dict(A=a, B=b, C=torch.empty_like(a), op_a=i % 2, op_b=0))
    ws = pm.workspace(pm.batched_workspace_size(items, "fp64"), DEV)
    pm.polymat_mul_batched(items, "fp64", ws=ws)
    torch.cuda.synchronize()
    eager = [it["C"].clone() for it in items]
    g = _capture(lambda: pm.polymat_mul_batched(items, "fp64", ws=ws))
    for rep in range(3):
        for it in items:
            it["C"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, ref in zip(items, eager):
            assert torch.equal(it["C"], ref), rep
        pm.polymat_mul_batched(items, "fp64", ws=ws)     # eager work between replays
        torch.cuda.synchronize()


def test_langevin_step_graph_replays():
    L, k, nt, R = 3, 1, 5, 2
    u0 = to_dev(series_links(L, k, nt, 0.6, 61, replicas=R))
    eta = to_dev(synth.langevin_noise(synth.rng_for(62), R, L * L))
    prm = pm.nspt_params(L, k, nt, 0.02)
    ws = pm.workspace(pm.nspt_workspace_size(R, prm), DEV)
    u = u0.clone()
    pm.nspt_langevin_step(u, eta, prm, ws=ws)
    torch.cuda.synchronize()
    eager = u.clone()
    g = _capture(lambda: pm.nspt_langevin_step(u, eta, prm, ws=ws))
    for rep in range(3):
        u.copy_(u0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, eager), rep


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_gauge_fix_graph_replays(prec):
    L, k, nt, R = 5, 2, 7, 2
    u0 = to_dev(series_links(L, k, nt, 0.6, 63, replicas=R))
    prm = pm.nspt_params(L, k, nt, 0.02)
    ws = pm.workspace(pm.nspt_workspace_size(R, prm, prec), DEV)
    u = u0.clone()
    pm.nspt_gauge_fix(u, prm, 0.1, prec, ws=ws)
    torch.cuda.synchronize()
    eager = u.clone()
    g = _capture(lambda: pm.nspt_gauge_fix(u, prm, 0.1, prec, ws=ws))
    for rep in range(3):
        u.copy_(u0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, eager), rep
        v = u0.clone()
        pm.nspt_gauge_fix(v, prm, 0.1, prec, ws=ws)      # eager work between replays
        torch.cuda.synchronize()
