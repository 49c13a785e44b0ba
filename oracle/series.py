"""Truncated matrix power series: the star product by its definition.

Oracle (test infrastructure only; see the package docstring).

A series is a complex128 array X of shape [ntrunc + 1, N, N]; X[k] is the
coefficient X^(k) of g^k (Section 2, eq. (4)).  All products are truncated
at O(g^ntrunc).
"""
from __future__ import annotations

import math

import numpy as np


def star(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C = A * B with C^(k) = sum_{l=0..k} A^(l) B^(k-l), k = 0..ntrunc.

    Section 2, eq. (5): the convolution product of two truncated polynomial
    matrices; the matrix factors keep their order (A on the left).  This is
    the naive algorithm, (ntrunc+1)(ntrunc+2)/2 matrix products.
    """
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    if a.shape != b.shape or a.ndim != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("star: operands must both be [ntrunc+1, N, N]")
    nt1 = a.shape[0]
    c = np.zeros_like(a)
    for k in range(nt1):
        acc = np.zeros(a.shape[1:], dtype=np.complex128)
        for l in range(k + 1):
            acc += a[l] @ b[k - l]
        c[k] = acc
    return c


def dagger(a: np.ndarray) -> np.ndarray:
    """Series Hermitian conjugate: (A^+)^(k) = (A^(k))^+ (g is real).

    Implicit in eq. (3), where U^+ of a link series enters the staples.
    """
    return np.conj(np.swapaxes(a, -1, -2))


def identity(n: int, ntrunc: int) -> np.ndarray:
    """The unit series 1 = 1 + 0 g + 0 g^2 + ..."""
    e = np.zeros((ntrunc + 1, n, n), dtype=np.complex128)
    e[0] = np.eye(n)
    return e


def truncate(a: np.ndarray, ntrunc: int) -> np.ndarray:
    """Keep the coefficients of g^0..g^ntrunc."""
    return np.array(a[: ntrunc + 1], dtype=np.complex128)


def series_exp(y: np.ndarray) -> np.ndarray:
    """exp(Y) = sum_{n=0..ntrunc} Y^{*n} / n!  for a series with Y^(0) = 0.

    With Y = O(g) the n-th power starts at order g^n, so the sum truncated at
    n = ntrunc is exact to O(g^ntrunc).  Used for the link update of the
    Euler-Langevin step (exp of i times the drift-plus-noise series).
    """
    y = np.asarray(y, dtype=np.complex128)
    if np.any(y[0] != 0):
        raise ValueError("series_exp: order-0 coefficient must vanish")
    nt1, n = y.shape[0], y.shape[1]
    out = identity(n, nt1 - 1)
    term = identity(n, nt1 - 1)
    for m in range(1, nt1):
        term = star(term, y) / m      # Y^{*m} / m!
        out += term
    return out


def order_rel_errors(c: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """e_k = ||C^(k) - C_ref^(k)||_F / ||C_ref^(k)||_F for every order k.

    Orders whose reference is exactly zero report the absolute error instead.
    """
    c = np.asarray(c)
    ref = np.asarray(ref)
    num = np.sqrt(np.sum(np.abs(c - ref) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-2, -1)))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def order_norm_bound(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """c_k = sum_{l<=k} ||A^(l)||_F ||B^(k-l)||_F, a scale for order-k errors.

    Used where C^(k) itself cancels (identities): the error of order k is then
    measured against c_k rather than ||C^(k)||.
    """
    na = np.sqrt(np.sum(np.abs(a) ** 2, axis=(-2, -1)))
    nb = np.sqrt(np.sum(np.abs(b) ** 2, axis=(-2, -1)))
    nt1 = a.shape[0]
    return np.array([sum(na[l] * nb[k - l] for l in range(k + 1)) for k in range(nt1)])


def factorial(m: int) -> float:
    return float(math.factorial(m))
