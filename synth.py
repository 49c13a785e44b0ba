"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module only draws random numbers and builds fixed input configurations.
It holds none of the series arithmetic of the method (no products, no
transforms, no exponentials): both the CPU oracle and the GPU path consume
what it produces, and neither of them is imported here.

Series layout: a truncated power series in g with N x N complex coefficients
is a complex128 array of shape [ntrunc + 1, N, N]; index k holds the
coefficient of g^k (paper, Section 2, eq. (4)).
"""
from __future__ import annotations

import numpy as np


def rng_for(*key: int) -> np.random.Generator:
    """A generator keyed by a tuple of small integers (config, item, operand...)."""
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def random_series(rng: np.random.Generator, n: int, ntrunc: int, ratio: float = 1.0) -> np.ndarray:
    """Coefficient k has i.i.d. N(0,1) real and imaginary parts, times ratio**k.

    This is the workload recipe of the benchmark configurations (geometric
    growth or decay of the coefficient magnitudes with the order).
    """
    shape = (ntrunc + 1, n, n)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    scale = ratio ** np.arange(ntrunc + 1, dtype=np.float64)
    return (re + 1j * im) * scale[:, None, None]


def gue_traceless(rng: np.random.Generator, n: int) -> np.ndarray:
    """Hermitian traceless Gaussian matrix.

    Diagonal entries N(0,1); strictly upper entries have real and imaginary
    parts N(0,1/2), mirrored to the lower triangle by Hermitian symmetry;
    then the trace part Tr/N times the identity is removed.  With this
    normalisation eta = sum_a xi_a T^a for an orthonormal basis Tr(T^a T^b)
    = delta_ab of traceless Hermitian matrices and i.i.d. unit normals xi_a.
    """
    h = np.zeros((n, n), dtype=np.complex128)
    iu = np.triu_indices(n, 1)
    m = len(iu[0])
    off = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * np.sqrt(0.5)
    h[iu] = off
    h = h + h.conj().T
    h[np.diag_indices(n)] = rng.standard_normal(n)
    h -= np.trace(h) / n * np.eye(n)
    return h


def langevin_noise(rng: np.random.Generator, replicas: int, n: int) -> np.ndarray:
    """Noise for one Langevin step: complex128 [replicas, 4, n, n], Hermitian traceless."""
    out = np.empty((replicas, 4, n, n), dtype=np.complex128)
    for r in range(replicas):
        for mu in range(4):
            out[r, mu] = gue_traceless(rng, n)
    return out


def twist_eaters(L: int, k: int) -> np.ndarray:
    """Four SU(N) matrices (N = L*L) that solve the twisted vacuum condition.

    Built from the L x L shift S (S e_j = e_{j+1}) and clock C = diag(w^j),
    w = exp(2 pi i / L), which obey C S = w S C:
        G1 = S x 1,   G2 = C^k x 1,   G3 = S^-1 C^k x S,   G4 = S^-1 C^k x C^k
    (x = Kronecker product).  For X = S^a C^b, Y = S^c C^d one has
    X Y = w^(bc - ad) Y X, and the exponents above make every pair mu < nu
    obey G_mu G_nu = w^-k G_nu G_mu, i.e. z_{mu nu} G_mu G_nu G_mu^+ G_nu^+ = 1
    for z_{mu nu} = exp(2 pi i k / L); the tests check this.
    Returned as complex128 [4, N, N].
    """
    w = np.exp(2j * np.pi / L)
    shift = np.roll(np.eye(L), 1, axis=0)          # maps e_j -> e_{j+1}
    clock = np.diag(w ** np.arange(L))
    one = np.eye(L)
    sinv = shift.T
    ck = np.linalg.matrix_power(clock, k)           # C^k
    g = np.empty((4, L * L, L * L), dtype=np.complex128)
    g[0] = np.kron(shift, one)
    g[1] = np.kron(ck, one)
    g[2] = np.kron(sinv @ ck, shift)
    g[3] = np.kron(sinv @ ck, ck)
    return g


def vacuum_links(L: int, k: int, ntrunc: int, replicas: int = 1) -> np.ndarray:
    """Link series at the classical vacuum: U^(0) = twist eaters, all higher orders 0.

    complex128 [replicas, 4, ntrunc + 1, N, N].
    """
    g = twist_eaters(L, k)
    n = L * L
    u = np.zeros((replicas, 4, ntrunc + 1, n, n), dtype=np.complex128)
    u[:, :, 0] = g[None]
    return u


def uneven_batch_shapes(rng: np.random.Generator, count: int,
                        sizes=(64, 121, 169, 225, 289), truncs=(15, 31, 63)):
    """(n, ntrunc) pairs drawn uniformly from the given sets."""
    ns = rng.choice(np.asarray(sizes), size=count)
    ts = rng.choice(np.asarray(truncs), size=count)
    return [(int(a), int(b)) for a, b in zip(ns, ts)]
