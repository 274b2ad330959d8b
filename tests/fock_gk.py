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


def spectral_moments_k(cl: Cluster, beta: float, pmax: int) -> np.ndarray:
    """int w^p A_k(w) dw for p = 0..pmax, array [pmax + 1, N], averaged over
    the spins, A_k the spectral function whose eq. (4) transform is G(tau, k):
    the thermal expectation <{X_p, c_k^dagger}> with X_0 = c_k and
    X_{p+1} = [X_p, H], c_k = N^-1/2 sum_i e^{-i k r_i} c_i (the frequency
    moments of A follow from the time derivatives of the anticommutator
    function at t = 0)."""
    L, N = cl.L, cl.N
    H = cl.Ht + cl.HU
    E, V = np.linalg.eigh(H)
    w = np.exp(-beta * (E - E.min()))
    rho = (V * (w / w.sum())) @ V.T
    out = np.zeros((pmax + 1, N))
    for k in range(N):
        kx, ky = 2 * math.pi * (k % L) / L, 2 * math.pi * (k // L) / L
        for s in range(2):
            ck = sum(np.exp(-1j * (kx * (i % L) + ky * (i // L))) * cl.c[i + N * s] for i in range(N)) / math.sqrt(N)
            cd = ck.conj().T
            X = ck
            for p in range(pmax + 1):
                out[p, k] += 0.5 * np.real(np.trace(rho @ (X @ cd + cd @ X)))
                X = X @ H - H @ X
    return out
