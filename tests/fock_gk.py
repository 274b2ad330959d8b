"""G(tau, k) of the 2 x 2 cluster from the Fock-space helper (test helper):
the exact Trotterised values on a slice grid and the exact continuous-time
values, both in the paper's sign (eq. (4)) and in the cos(k (r_i - r_j))
form the library measures, averaged over the two spins."""
from __future__ import annotations

import math

import numpy as np

from tests.fock import Cluster


def to_gk(gt, L: int) -> np.ndarray:
    """[n, N, N] per spin (positive convention) -> [n, N] paper-sign G(tau, k)."""
    N = L * L
    n = gt[0].shape[0]
    out = np.zeros((n, N))
    for k in range(N):
        kx, ky = 2 * math.pi * (k % L) / L, 2 * math.pi * (k // L) / L
        ph = np.array([[math.cos(kx * ((i % L) - (j % L)) + ky * ((i // L) - (j // L))) for j in range(N)]
                       for i in range(N)])
        for l in range(n):
            out[l, k] = -0.5 * sum(np.sum(ph * gt[s][l]) for s in range(2)) / N
    return out


def trotterised_gk(cl: Cluster, beta: float, dtau: float) -> np.ndarray:
    return to_gk([cl.gtau(beta, dtau, s) for s in range(2)], cl.L)


def continuous_gk(cl: Cluster, beta: float, taus) -> np.ndarray:
    return to_gk([cl.gtau_exact(beta, taus, s) for s in range(2)], cl.L)


def continuous_giw_k(cl: Cluster, beta: float, n_freq: int) -> np.ndarray:
    """G_k(i w_n) [n_freq, N] of the continuous-time model in the same
    cos(k (r_i - r_j)) form, averaged over the spins (Lehmann sums)."""
    L, N = cl.L, cl.N
    g = [cl.giw_exact(beta, n_freq, s) for s in range(2)]
    out = np.zeros((n_freq, N), dtype=complex)
    for k in range(N):
        kx, ky = 2 * math.pi * (k % L) / L, 2 * math.pi * (k // L) / L
        ph = np.array([[math.cos(kx * ((i % L) - (j % L)) + ky * ((i // L) - (j // L))) for j in range(N)]
                       for i in range(N)])
        for a in range(n_freq):
            out[a, k] = 0.5 * sum(np.sum(ph * g[s][a]) for s in range(2)) / N
    return out
