"""GPU parity of the FFT-CONV path against the FP64 oracle, through the C ABI.

Inputs come from the seeded generators of `synth`; every expected value comes
from `oracle` (the naive star product or the literal FFT-CONV steps).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fftconv, series as ser
import paper_2001_02835_amd as pm
from gpu_util import DEV, TOL, order_errors, to_dev, to_host

pytestmark = pytest.mark.gpu


def rs(seed, n, nt, r=1.0):
    return synth.random_series(synth.rng_for(700, seed), n, nt, r)


@pytest.mark.parametrize("n,nt,s", [(9, 7, 1.0), (5, 0, 1.0), (7, 3, 0.7), (17, 12, 1.3), (3, 31, 0.9), (4, 63, 1.05)])
def test_forward_transform_matches_definition(n, nt, s):
    a = rs(1, n, nt)
    L = pm.transform_length(nt)
    got = to_host(pm.forward_transform(to_dev(a), scale=s))
    scaled = a * (s ** np.arange(nt + 1))[:, None, None]
    ref = fftconv.forward(scaled, L)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    # both sides round: the oracle sums L terms directly (error ~ eps L), the
    # kernel in log2(L) butterfly stages; the bound is 1e-15 L
    assert err < 1e-15 * L, err


@pytest.mark.parametrize("n,nt,s", [(9, 7, 1.0), (5, 0, 1.0), (6, 5, 2.0), (17, 31, 0.8), (4, 63, 1.02)])
def test_inverse_transform_matches_definition(n, nt, s):
    L = pm.transform_length(nt)
    ct = synth.random_series(synth.rng_for(701, n, nt), n, L - 1)
    got = to_host(pm.inverse_transform(to_dev(ct), nt, scale=s))
    ref = fftconv.inverse(ct)[: nt + 1] * (s ** -np.arange(nt + 1.0))[:, None, None]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-15 * L, err


def test_small_product_matches_naive_oracle():
    # N = 9, ntrunc = 7 (transform length 16), i.i.d. N(0,1) entries
    a, b = rs(2, 9, 7), rs(3, 9, 7)
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b)))
    e = order_errors(c, ser.star(a, b))
    assert e.max() < TOL["fp64"], e


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 63, 64, 65, 100, 130])
@pytest.mark.parametrize("nt", [0, 1, 5, 15])
def test_ragged_shapes_fp64(n, nt):
    a, b = rs(4, n, nt, 0.8), rs(5, n, nt, 0.8)
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b)))
    e = order_errors(c, ser.star(a, b))
    assert e.max() < TOL["fp64"], e


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n", [1, 2, 5, 8, 9, 31, 32, 63, 64, 65, 100, 130])
def test_ragged_shapes_reduced_precisions_all_operand_forms(prec, n):
    """Ragged tiles and row pitches (split-BF16 rows padded to a multiple of
    8 entries, contracted index on either side of the transposing LDS read)
    for the four operand forms X, X^+ on either side."""
    nt = 5
    items, refs = [], []
    for i in range(4):
        a, b = rs(100 + i, n, nt, 0.8), rs(110 + i, n, nt, 0.8)
        op_a, op_b = i % 2, i // 2
        refs.append(ser.star(ser.dagger(a) if op_a else a, ser.dagger(b) if op_b else b))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                          op_a=op_a, op_b=op_b, scale=0.0))
    pm.polymat_mul_batched(items, precision=prec)
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL[prec], (i, e)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n,nt,r", [(33, 7, 1.0), (70, 31, 0.5), (48, 63, 1.3)])
def test_precisions_with_auto_rescale(prec, n, nt, r):
    a, b = rs(6, n, nt, r), rs(7, n, nt, r)
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b), precision=prec))
    e = order_errors(c, ser.star(a, b))
    assert e.max() < TOL[prec], (prec, e.max(), e)


def test_fixed_scale_equals_exact_product():
    a, b = rs(8, 20, 15, 0.5), rs(9, 20, 15, 0.5)
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b), scale=2.0))
    assert order_errors(c, ser.star(a, b)).max() < TOL["fp64"]


def test_output_may_alias_an_input():
    a, b = rs(10, 24, 7), rs(11, 24, 7)
    ref = ser.star(a, b)
    da, db = to_dev(a), to_dev(b)
    pm.polymat_mul(da, db, C=da)
    assert order_errors(to_host(da), ref).max() < TOL["fp64"]
    da, db = to_dev(a), to_dev(b)
    pm.polymat_mul(da, db, C=db)
    assert order_errors(to_host(db), ref).max() < TOL["fp64"]


def test_bitwise_reproducible():
    a, b = to_dev(rs(12, 65, 15)), to_dev(rs(13, 65, 15))
    c1 = to_host(pm.polymat_mul(a, b))
    c2 = to_host(pm.polymat_mul(a, b))
    assert np.array_equal(c1, c2)


def test_batched_uneven_with_conjugated_operands():
    shapes = [(9, 7), (20, 3), (33, 15), (5, 0), (64, 31), (17, 12)]
    items, refs = [], []
    for i, (n, nt) in enumerate(shapes):
        a, b = rs(20 + i, n, nt, 0.9), rs(40 + i, n, nt, 0.9)
        op_a, op_b = i % 2, (i // 2) % 2
        aa = ser.dagger(a) if op_a else a
        bb = ser.dagger(b) if op_b else b
        refs.append(ser.star(aa, bb))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                          op_a=op_a, op_b=op_b, scale=0.0))
    pm.polymat_mul_batched(items)
    for it, ref in zip(items, refs):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL["fp64"], e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nt", [(121, 31), (130, 63), (100, 15)])
def test_tuned_tile_shapes_per_length(prec, n, nt):
    """Sizes and transform lengths (L = 32, 64, 128) where the tile table
    may pick a shape other than the default one (FP32 at 93 <= n <= 145 and
    L >= 64), all four operand forms."""
    items, refs = [], []
    for i in range(4):
        a, b = rs(130 + i, n, nt, 0.7), rs(140 + i, n, nt, 0.7)
        op_a, op_b = i % 2, i // 2
        refs.append(ser.star(ser.dagger(a) if op_a else a, ser.dagger(b) if op_b else b))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                          op_a=op_a, op_b=op_b, scale=0.0))
    pm.polymat_mul_batched(items, precision=prec)
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL[prec], (i, e)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n", [17, 33, 81, 161, 193, 225, 289])
def test_thin_edge_sizes_all_operand_forms(prec, n):
    """n = 16 m + 1: the last row and column of each mode product take the
    vector-unit path; all four operand forms (X, X^+ on either side)."""
    nt = 3
    items, refs = [], []
    for i in range(4):
        a, b = rs(80 + i, n, nt, 0.9), rs(90 + i, n, nt, 0.9)
        op_a, op_b = i % 2, i // 2
        refs.append(ser.star(ser.dagger(a) if op_a else a, ser.dagger(b) if op_b else b))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV),
                          op_a=op_a, op_b=op_b, scale=0.0))
    pm.polymat_mul_batched(items, precision=prec)
    for i, (it, ref) in enumerate(zip(items, refs)):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL[prec], (i, e)


def test_batched_matches_single_calls_bitwise():
    a = [to_dev(rs(60 + i, 40, 15)) for i in range(3)]
    b = [to_dev(rs(70 + i, 40, 15)) for i in range(3)]
    single = [to_host(pm.polymat_mul(a[i], b[i])) for i in range(3)]
    items = [dict(A=a[i], B=b[i], C=torch.empty_like(a[i])) for i in range(3)]
    pm.polymat_mul_batched(items)
    for i in range(3):
        assert np.array_equal(to_host(items[i]["C"]), single[i])


def test_paper_scale_four_products_fp64():
    # one product per direction: N = 225, ntrunc = 31 (L = 64), entries N(0,1) 0.5^k
    n, nt = 225, 31
    items, refs = [], []
    for mu in range(4):
        a = synth.random_series(synth.rng_for(2, mu, 0), n, nt, 0.5)
        b = synth.random_series(synth.rng_for(2, mu, 1), n, nt, 0.5)
        refs.append(ser.star(a, b))
        items.append(dict(A=to_dev(a), B=to_dev(b), C=torch.empty((nt + 1, n, n), dtype=torch.complex128, device=DEV)))
    pm.polymat_mul_batched(items, precision="fp64")
    for it, ref in zip(items, refs):
        e = order_errors(to_host(it["C"]), ref)
        assert e.max() < TOL["fp64"], e.max()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_paper_scale_growing_series(prec):
    # N = 225, ntrunc = 63 (L = 128), entries N(0,1) 1.3^k, automatic rescaling
    n, nt = 225, 63
    a = synth.random_series(synth.rng_for(3, 0, 0), n, nt, 1.3)
    b = synth.random_series(synth.rng_for(3, 0, 1), n, nt, 1.3)
    ref = _cached_star(a, b, key=("c3",))
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b), precision=prec))
    e = order_errors(c, ref)
    print(f"{prec}: max per-order error {e.max():.3e}")
    assert e.max() < TOL[prec], e.max()


_STAR_CACHE = {}


def _cached_star(a, b, key):
    if key not in _STAR_CACHE:
        _STAR_CACHE[key] = ser.star(a, b)
    return _STAR_CACHE[key]


@pytest.mark.parametrize("n", [1, 17, 33, 65, 100])
@pytest.mark.parametrize("nt", [0, 1, 2, 5, 15])
def test_naive_direct_form_matches_oracle(n, nt):
    a, b = rs(100 + n, n, nt, 0.9), rs(200 + n, n, nt, 0.9)
    for op_a in (0, 1):
        for op_b in (0, 1):
            c = to_host(pm.polymat_mul_naive(to_dev(a), to_dev(b), op_a=op_a, op_b=op_b))
            ref = ser.star(ser.dagger(a) if op_a else a, ser.dagger(b) if op_b else b)
            e = order_errors(c, ref)
            assert e.max() < 1e-12, (op_a, op_b, e)


def test_naive_direct_form_paper_scale():
    n, nt = 225, 7
    a = synth.random_series(synth.rng_for(4, 0, 0), n, nt, 0.5)
    b = synth.random_series(synth.rng_for(4, 0, 1), n, nt, 0.5)
    c = to_host(pm.polymat_mul_naive(to_dev(a), to_dev(b)))
    assert order_errors(c, ser.star(a, b)).max() < 1e-12


def test_naive_rejects_aliasing_output():
    a = to_dev(rs(300, 9, 2))
    b = to_dev(rs(301, 9, 2))
    with pytest.raises(pm.PolymatError):
        pm.polymat_mul_naive(a, b, C=a)


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_short_series_dispatch_and_alias_fallback(nt):
    # polymat_mul takes the direct form for short FP64 series, and the
    # transform path when C aliases an operand; both agree with the oracle
    a, b = rs(310 + nt, 40, nt), rs(320 + nt, 40, nt)
    ref = ser.star(a, b)
    c = to_host(pm.polymat_mul(to_dev(a), to_dev(b)))
    assert order_errors(c, ref).max() < 1e-12
    da, db = to_dev(a), to_dev(b)
    pm.polymat_mul(da, db, C=da)
    assert order_errors(to_host(da), ref).max() < TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_maximum_matrix_size_sampled(prec):
    # N = PM_MAX_N: every index of the kernels and the workspace at its largest;
    # checked on sampled entries computed one by one from eq. (5)
    n, nt = 4096, 1
    rng = np.random.default_rng(4096)
    a = to_dev(synth.random_series(synth.rng_for(40, 0), n, nt, 0.5))
    b = to_dev(synth.random_series(synth.rng_for(40, 1), n, nt, 0.5))
    items = [dict(A=a, B=b, C=torch.empty_like(a))]
    pm.polymat_mul_batched(items, precision=prec)
    c = items[0]["C"]
    ks, iis, jjs = rng.integers(0, nt + 1, 48), rng.integers(0, n, 48), rng.integers(0, n, 48)
    got = c[torch.as_tensor(ks, device=DEV), torch.as_tensor(iis, device=DEV), torch.as_tensor(jjs, device=DEV)]
    got = got.cpu().numpy()
    for t, (k, i, j) in enumerate(zip(ks, iis, jjs)):
        terms = [(a[l, i, :].cpu().numpy(), b[k - l, :, j].cpu().numpy()) for l in range(k + 1)]
        ref = sum(np.dot(x, y) for x, y in terms)
        scale = sum(np.linalg.norm(x) * np.linalg.norm(y) for x, y in terms)
        assert abs(got[t] - ref) <= TOL[prec] * scale, (prec, k, i, j, got[t], ref)


def test_batched_output_aliasing_another_problems_input():
    """C of one problem is the A of another: every A and B is read before any
    C is written, so the second product uses the original contents."""
    n, nt = 40, 7
    a0, b0, x, b1 = (rs(130 + i, n, nt, 0.8) for i in range(4))
    dx = to_dev(x)
    items = [dict(A=to_dev(a0), B=to_dev(b0), C=dx),
             dict(A=dx, B=to_dev(b1), C=torch.empty_like(dx))]
    pm.polymat_mul_batched(items)
    assert order_errors(to_host(items[0]["C"]), ser.star(a0, b0)).max() < TOL["fp64"]
    assert order_errors(to_host(items[1]["C"]), ser.star(x, b1)).max() < TOL["fp64"]
