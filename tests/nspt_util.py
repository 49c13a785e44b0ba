"""Link-series inputs for the NSPT tests, built with the oracle's series algebra."""
import numpy as np

import synth
from oracle import series as ser


def series_links(L, k, nt, amp, seed, replicas=1):
    """U_mu = exp(i sum_{j>=1} g^j A_{mu,j}) * Gamma_mu with traceless Hermitian A
    (|A_j| ~ amp^j), complex128 [replicas, 4, nt+1, N, N]."""
    g = synth.twist_eaters(L, k)
    n = L * L
    rng = synth.rng_for(930, seed)
    u = np.zeros((replicas, 4, nt + 1, n, n), dtype=np.complex128)
    for r in range(replicas):
        for mu in range(4):
            x = np.zeros((nt + 1, n, n), dtype=np.complex128)
            for j in range(1, nt + 1):
                x[j] = amp ** j * synth.gue_traceless(rng, n) / np.sqrt(n)
            gam = np.zeros_like(x)
            gam[0] = g[mu]
            u[r, mu] = ser.star(ser.series_exp(1j * x), gam)
    return u
