"""Pins of the oracle's counter-based Langevin noise (CPU only).

The Philox4x64-10 generator restated in `oracle.nspt.philox4x64` is pinned to
numpy's independent implementation (`numpy.random.Philox`, which advances
its 256-bit counter before each block), including carries across counter
words; the noise built from it is pinned by its invariants (Hermitian,
traceless, a pure function of (seed, step)) and by the variances of the GUE
recipe (diagonal 1, real and imaginary parts of the off-diagonal entries 1/2
each, before the trace removal), which a dropped 1/sqrt(2) or a swapped
cos/sin pairing would break.
"""
import numpy as np
import pytest

from oracle import nspt


def _as_int(words):
    return sum(int(w) << (64 * i) for i, w in enumerate(words))


@pytest.mark.parametrize("ctr,key", [([1, 0, 0, 0], [0, 0]), ([7, 3, 9, 11], [123, 456]),
                                     ([2**64 - 1, 5, 0, 1], [2**63 + 5, 77]),
                                     ([0, 1, 0, 0], [2**64 - 1, 2**64 - 1])])
def test_philox_matches_numpy(ctr, key):
    prev = (_as_int(ctr) - 1) % 2**256
    ref = np.random.Philox(key=_as_int(key), counter=prev).random_raw(4)
    got = nspt.philox4x64([np.uint64(x) for x in ctr], [np.uint64(x) for x in key])
    assert [int(v) for v in ref] == [int(v) for v in got]


def test_philox_vectorised_equals_scalar():
    ctr = [np.arange(5, dtype=np.uint64), np.full(5, 3, np.uint64), np.full(5, 9, np.uint64),
           np.zeros(5, np.uint64)]
    key = [np.full(5, 42, np.uint64), np.zeros(5, np.uint64)]
    vec = nspt.philox4x64(ctr, key)
    for t in range(5):
        one = nspt.philox4x64([c[t] for c in ctr], [k[t] for k in key])
        assert [int(v[t]) for v in vec] == [int(v) for v in one]


def test_noise_is_hermitian_traceless_and_a_function_of_seed_and_step():
    e = nspt.philox_noise(7, 3, 2, 9)
    assert e.shape == (2, 4, 9, 9)
    assert np.abs(e - e.conj().transpose(0, 1, 3, 2)).max() == 0.0
    assert np.abs(np.trace(e, axis1=-2, axis2=-1)).max() < 1e-14
    assert np.array_equal(e, nspt.philox_noise(7, 3, 2, 9))
    assert not np.allclose(e, nspt.philox_noise(7, 4, 2, 9))
    assert not np.allclose(e, nspt.philox_noise(8, 3, 2, 9))
    assert not np.allclose(e[0], e[1]) and not np.allclose(e[0, 0], e[0, 1])


def test_noise_variances_follow_the_gue_recipe():
    n = 96
    e = nspt.philox_noise(11, 0, 2, n)
    iu = np.triu_indices(n, 1)
    off = np.concatenate([e[r, m][iu] for r in range(2) for m in range(4)])
    diag = np.concatenate([np.diagonal(e[r, m]).real for r in range(2) for m in range(4)])
    # about 36000 off-diagonal and 770 diagonal samples
    assert abs(off.real.var() - 0.5) < 0.02 and abs(off.imag.var() - 0.5) < 0.02
    assert abs(np.mean(off.real * off.imag)) < 0.02
    assert abs(diag.var() * n / (n - 1) - 1.0) < 0.15
    assert abs(off.real.mean()) < 0.02 and abs(off.imag.mean()) < 0.02


def test_steps_use_consecutive_noise():
    from oracle import tek
    import synth
    L, k, nt = 3, 1, 3
    u = synth.vacuum_links(L, k, nt, replicas=1)
    z = tek.twist_tensor(L, k)
    two = nspt.langevin_steps_philox(u, z, 0.02, 5, 10, 2)
    ref = nspt.langevin_step_replicas(u, nspt.philox_noise(5, 10, 1, L * L), z, 0.02)
    ref = nspt.langevin_step_replicas(ref, nspt.philox_noise(5, 11, 1, L * L), z, 0.02)
    assert np.array_equal(two, ref)
