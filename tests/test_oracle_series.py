"""Pins of the oracle's series algebra and FFT-CONV steps (CPU only).

Each test checks the oracle against something other than itself: a hand
worked example, a textbook routine it reduces to, a closed form, or an
identity the mathematics fixes.  The mutation tests at the end plant
plausible mistakes in a copy of the oracle and show that these pins fail.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import fftconv, series as ser


def rs(seed, n, nt, r=1.0):
    return synth.random_series(synth.rng_for(900, seed), n, nt, r)


def test_star_matches_hand_worked_example(golden):
    g = golden("star_2x2_ntrunc2.txt")
    c = ser.star(g["A"], g["B"])
    assert np.array_equal(c, g["C"])


def test_star_matches_scalar_loop_brute_force():
    # every entry written as a sum over (l, m) of products of scalars
    for n, nt in [(1, 0), (2, 3), (3, 2)]:
        a, b = rs(1, n, nt), rs(2, n, nt)
        c = ser.star(a, b)
        ref = np.zeros_like(c)
        for k in range(nt + 1):
            for i in range(n):
                for j in range(n):
                    s = 0j
                    for l in range(k + 1):
                        for m in range(n):
                            s += a[l, i, m] * b[k - l, m, j]
                    ref[k, i, j] = s
        assert np.allclose(c, ref, rtol=1e-14, atol=1e-13)


def test_star_n1_is_numpy_convolve():
    for nt in [0, 1, 7, 20]:
        a, b = rs(3, 1, nt), rs(4, 1, nt)
        c = ser.star(a, b)[:, 0, 0]
        ref = np.convolve(a[:, 0, 0], b[:, 0, 0])[: nt + 1]
        assert np.allclose(c, ref, rtol=1e-13, atol=1e-13)


def test_star_diagonal_reduces_to_scalar_convolutions():
    n, nt = 5, 9
    rng = synth.rng_for(901)
    da = rng.standard_normal((nt + 1, n)) + 1j * rng.standard_normal((nt + 1, n))
    db = rng.standard_normal((nt + 1, n)) + 1j * rng.standard_normal((nt + 1, n))
    a = np.stack([np.diag(x) for x in da])
    b = np.stack([np.diag(x) for x in db])
    c = ser.star(a, b)
    for i in range(n):
        ref = np.convolve(da[:, i], db[:, i])[: nt + 1]
        assert np.allclose(np.diagonal(c, axis1=1, axis2=2)[:, i], ref, rtol=1e-13, atol=1e-13)
    off = c - np.stack([np.diag(np.diag(x)) for x in c])
    assert np.abs(off).max() == 0


def test_star_unit_and_shift():
    n, nt = 4, 6
    a = rs(5, n, nt)
    one = ser.identity(n, nt)
    assert np.array_equal(ser.star(a, one), a)
    assert np.array_equal(ser.star(one, a), a)
    gser = np.zeros_like(a)
    gser[1] = np.eye(n)                       # the series "g * 1"
    c = ser.star(a, gser)
    assert np.array_equal(c[0], np.zeros((n, n)))
    assert np.array_equal(c[1:], a[:-1])


def test_star_keeps_factor_order():
    # non-commuting coefficients: A * B differs from B * A
    a, b = rs(6, 3, 2), rs(7, 3, 2)
    assert np.abs(ser.star(a, b) - ser.star(b, a)).max() > 1e-3


def test_dagger_reverses_products():
    a, b = rs(8, 4, 5), rs(9, 4, 5)
    lhs = ser.dagger(ser.star(a, b))
    rhs = ser.star(ser.dagger(b), ser.dagger(a))
    assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-12)


def test_star_associative_and_bilinear():
    a, b, c = rs(10, 4, 5), rs(11, 4, 5), rs(12, 4, 5)
    assert np.allclose(ser.star(ser.star(a, b), c), ser.star(a, ser.star(b, c)), atol=1e-11)
    al, be = 0.3 - 1.1j, 2.0 + 0.5j
    assert np.allclose(ser.star(al * a + be * b, c), al * ser.star(a, c) + be * ser.star(b, c), atol=1e-11)


def test_geometric_series_closed_form():
    # (1 - g M) * (sum_k g^k M^k) = 1 exactly in exact arithmetic
    n, nt = 4, 10
    m = synth.random_series(synth.rng_for(902), n, 0)[0] * 0.3
    left = ser.identity(n, nt)
    left[1] = -m
    geo = np.stack([np.linalg.matrix_power(m, k) for k in range(nt + 1)])
    prod = ser.star(left, geo)
    assert np.allclose(prod, ser.identity(n, nt), atol=1e-13)


def test_commuting_polynomials_diagonalise():
    # A^(k) = p_k(M), B^(k) = q_k(M) -> scalar convolutions in M's eigenbasis
    n, nt = 4, 5
    rng = synth.rng_for(903)
    m = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lam, v = np.linalg.eig(m)
    pc = rng.standard_normal((nt + 1, 3))
    qc = rng.standard_normal((nt + 1, 3))
    def poly(coefs, x):
        return sum(c * np.linalg.matrix_power(x, d) for d, c in enumerate(coefs))
    a = np.stack([poly(pc[k], m) for k in range(nt + 1)])
    b = np.stack([poly(qc[k], m) for k in range(nt + 1)])
    c = ser.star(a, b)
    vinv = np.linalg.inv(v)
    for e in range(n):
        pa = np.array([sum(pc[k, d] * lam[e] ** d for d in range(3)) for k in range(nt + 1)])
        pb = np.array([sum(qc[k, d] * lam[e] ** d for d in range(3)) for k in range(nt + 1)])
        ref = np.convolve(pa, pb)[: nt + 1]
        got = np.array([(vinv @ c[k] @ v)[e, e] for k in range(nt + 1)])
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-9)


def test_exp_of_scalar_series_closed_form():
    # N = 1, Y = c g:  exp(c g) = sum_k c^k / k! g^k
    nt = 12
    cval = 0.7 - 0.4j
    y = np.zeros((nt + 1, 1, 1), dtype=np.complex128)
    y[1, 0, 0] = cval
    e = ser.series_exp(y)[:, 0, 0]
    ref = np.array([cval ** k / math.factorial(k) for k in range(nt + 1)])
    assert np.allclose(e, ref, rtol=1e-14, atol=1e-15)


def test_exp_times_exp_minus_is_one():
    n, nt = 5, 7
    x = rs(13, n, nt)
    x[0] = 0
    e1 = ser.series_exp(x)
    e2 = ser.series_exp(-x)
    prod = ser.star(e1, e2)
    err = np.abs(prod - ser.identity(n, nt))
    scale = ser.order_norm_bound(e1, e2)
    for k in range(nt + 1):
        assert err[k].max() <= 1e-13 * max(scale[k], 1.0)


def test_exp_matches_dense_expm_to_truncation_order():
    # sum_k g^k exp(Y)^(k) - expm(Y(g)) = O(g^(nt+1))
    import scipy.linalg as sl
    n, nt = 4, 4
    y = rs(14, n, nt)
    y[0] = 0
    e = ser.series_exp(y)
    errs = []
    for gval in (0.1, 0.05):
        dense = sl.expm(sum(gval ** k * y[k] for k in range(nt + 1)))
        approx = sum(gval ** k * e[k] for k in range(nt + 1))
        errs.append(np.abs(dense - approx).max())
    # halving g shrinks the error by about 2^(nt+1) = 32
    assert errs[0] / errs[1] > 0.6 * 2 ** (nt + 1)


def test_forward_transform_of_delta_is_a_pure_phase():
    L, n = 16, 3
    for j in [0, 1, 5, 7]:
        a = np.zeros((8, n, n), dtype=np.complex128)
        a[j] = np.eye(n)
        at = fftconv.forward(a, L)
        ph = np.exp(2j * np.pi * j * np.arange(L) / L)
        for p in range(L):
            assert np.allclose(at[p], ph[p] * np.eye(n), atol=1e-14)


def test_forward_transform_equals_L_times_numpy_ifft():
    # eq. (7) uses w = exp(+2 pi i / L): that is L times numpy's inverse FFT
    a = rs(15, 3, 7)
    L = 16
    ref = L * np.fft.ifft(fftconv.pad(a, L), axis=0)
    assert np.allclose(fftconv.forward(a, L), ref, atol=1e-12)
    back = fftconv.inverse(fftconv.forward(a, L))
    assert np.allclose(back[:8], a, atol=1e-13) and np.abs(back[8:]).max() < 1e-13


def test_parseval():
    a = rs(16, 4, 15)
    L = 32
    at = fftconv.forward(a, L)
    assert np.isclose(np.sum(np.abs(at) ** 2), L * np.sum(np.abs(a) ** 2), rtol=1e-12)


def test_dagger_in_fourier_space_is_a_reflection():
    # (U^+)~^(p) = ((U~^(-p mod L)))^+
    a = rs(17, 4, 7)
    L = 16
    lhs = fftconv.forward(ser.dagger(a), L)
    at = fftconv.forward(a, L)
    for p in range(L):
        assert np.allclose(lhs[p], at[(-p) % L].conj().T, atol=1e-12)


@pytest.mark.parametrize("n,nt", [(1, 0), (3, 1), (9, 7), (4, 5), (6, 12), (5, 31)])
def test_fft_conv_steps_reproduce_star(n, nt):
    a, b = rs(18, n, nt), rs(19, n, nt)
    c = fftconv.fft_conv(a, b)
    ref = ser.star(a, b)
    e = ser.order_rel_errors(c, ref)
    assert e.max() < 1e-12


def test_transform_length():
    assert [fftconv.transform_length(t) for t in (0, 1, 3, 7, 15, 31, 63, 5, 12)] == \
        [2, 4, 8, 16, 32, 64, 128, 16, 32]


# ---- mutation tests: plausible mistakes planted in a copy of the oracle ----

def _star_dropped_term(a, b):
    nt1 = a.shape[0]
    c = np.zeros_like(a)
    for k in range(nt1):
        for l in range(k):                 # forgets l = k
            c[k] += a[l] @ b[k - l]
    return c


def _star_transposed(a, b):
    nt1 = a.shape[0]
    c = np.zeros_like(a)
    for k in range(nt1):
        for l in range(k + 1):
            c[k] += b[k - l] @ a[l]        # factors swapped
    return c


def _star_wrong_index(a, b):
    nt1 = a.shape[0]
    c = np.zeros_like(a)
    for k in range(nt1):
        for l in range(k + 1):
            c[k] += a[l] @ b[k - l - 1 if k - l - 1 >= 0 else 0]
    return c


@pytest.mark.parametrize("bad", [_star_dropped_term, _star_transposed, _star_wrong_index])
def test_pins_catch_planted_star_mistakes(golden, bad):
    g = golden("star_2x2_ntrunc2.txt")
    caught = not np.array_equal(bad(g["A"], g["B"]), g["C"])
    a, b, c = rs(20, 3, 4), rs(21, 3, 4), rs(22, 3, 4)
    caught |= not np.allclose(ser.dagger(bad(a, b)), bad(ser.dagger(b), ser.dagger(a)))
    caught |= not np.allclose(bad(bad(a, b), c), bad(a, bad(b, c)))
    assert caught
