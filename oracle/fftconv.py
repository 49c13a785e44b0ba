"""The FFT-CONV steps of Section 2 written out with explicit DFT sums.

Oracle (test infrastructure only; see the package docstring).

These functions restate Steps 1-5 (eqs. (6)-(9)) literally, with the DFT
written as a sum over a w^{kp} matrix rather than a fast transform, so that
they can be read against the paper.  They serve to pin the forward transform
stage of the GPU path (the Fourier coefficients it produces) and to show that
the five steps reproduce the star product of ``series.star``.
"""
from __future__ import annotations

import numpy as np


def transform_length(ntrunc: int) -> int:
    """L = 2 N_p for N_p = ntrunc + 1 a power of two (Step 1; the paper's
    restriction N_trunc = N_p - 1, N_p = 2^s).  For other ntrunc the smallest
    power of two >= 2 (ntrunc + 1) is used: any L >= 2 ntrunc + 1 avoids
    wrap-around onto the kept orders."""
    need = 2 * (ntrunc + 1)
    L = 1
    while L < need:
        L *= 2
    return L


def pad(a: np.ndarray, L: int) -> np.ndarray:
    """Step 1 (eq. (6)): append zero coefficients up to length L."""
    out = np.zeros((L,) + a.shape[1:], dtype=np.complex128)
    out[: a.shape[0]] = a
    return out


def dft_matrix(L: int, sign: int) -> np.ndarray:
    """W[p, k] = w^{sign * k p}, w = exp(2 pi i / L) (eqs. (7) and (9))."""
    k = np.arange(L)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / L)


def forward(a: np.ndarray, L: int) -> np.ndarray:
    """Step 2 (eq. (7)): A~^(p) = sum_k A^(k) w^{kp} of the padded series."""
    ap = pad(a, L)
    return np.einsum("pk,kij->pij", dft_matrix(L, +1), ap)


def modewise(at: np.ndarray, bt: np.ndarray) -> np.ndarray:
    """Step 3 (eq. (8)): C~^(p) = A~^(p) B~^(p) for every mode p."""
    return np.stack([at[p] @ bt[p] for p in range(at.shape[0])])


def inverse(ct: np.ndarray) -> np.ndarray:
    """Step 4 (eq. (9)): C^(k) = (1/L) sum_p C~^(p) w^{-kp}."""
    L = ct.shape[0]
    return np.einsum("kp,pij->kij", dft_matrix(L, -1), ct) / L


def fft_conv(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Steps 1-5: pad, transform, mode-wise product, inverse, and Step 5,
    discard the orders above ntrunc."""
    nt1 = a.shape[0]
    L = transform_length(nt1 - 1)
    c = inverse(modewise(forward(a, L), forward(b, L)))
    return c[:nt1]
