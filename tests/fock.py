"""Fock-space exact treatment of tiny Hubbard clusters (test helper).

Independent of the oracle: the many-body operators are built from
Jordan-Wigner strings, the Hamiltonian of eq. (1) from the lattice directly,
and the Trotter product of eq. (2) with dense matrix exponentials.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def annihilators(n_orb: int):
    """c_o for o = 0..n_orb-1 on the 2^n_orb Fock space (Jordan-Wigner)."""
    dim = 1 << n_orb
    ops = []
    for o in range(n_orb):
        c = np.zeros((dim, dim))
        for s in range(dim):
            if (s >> o) & 1:
                parity = bin(s & ((1 << o) - 1)).count("1") & 1
                c[s ^ (1 << o), s] = -1.0 if parity else 1.0
        ops.append(c)
    return ops


class Cluster:
    """Periodic L x L Hubbard cluster; orbital index o = i + N * s (s=0 up, 1 down)."""

    def __init__(self, L: int, t: float, U: float):
        self.L, self.N = L, L * L
        self.c = annihilators(2 * self.N)
        N = self.N
        dim = 1 << (2 * N)
        Ht = np.zeros((dim, dim))
        for s in range(2):
            for y in range(L):
                for x in range(L):
                    i = x + L * y
                    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                        j = (x + dx) % L + L * ((y + dy) % L)
                        Ht += -t * self.c[j + N * s].T @ self.c[i + N * s]
        HU = np.zeros((dim, dim))
        eye = np.eye(dim)
        for i in range(N):
            nu = self.c[i].T @ self.c[i]
            nd = self.c[i + N].T @ self.c[i + N]
            HU += U * (nu - 0.5 * eye) @ (nd - 0.5 * eye)
        self.Ht, self.HU = Ht, HU

    def slice_op(self, dtau: float) -> np.ndarray:
        """One factor of eq. (2): e^{-dtau H_t} e^{-dtau H_U}."""
        return sla.expm(-dtau * self.Ht) @ sla.expm(-dtau * self.HU)

    def trotter(self, beta: float, dtau: float):
        lam = int(round(beta / dtau))
        T = self.slice_op(dtau)
        powers = [np.eye(T.shape[0])]
        for _ in range(lam):
            powers.append(T @ powers[-1])
        return lam, powers  # powers[l] = T^l

    def z_trotter(self, beta: float, dtau: float) -> float:
        lam, P = self.trotter(beta, dtau)
        return float(np.trace(P[lam]))

    def double_occ(self, beta: float, dtau: float) -> float:
        lam, P = self.trotter(beta, dtau)
        N = self.N
        D = sum(self.c[i].T @ self.c[i] @ self.c[i + N].T @ self.c[i + N] for i in range(N)) / N
        return float(np.trace(P[lam] @ D) / np.trace(P[lam]))

    def gtau_exact(self, beta: float, taus, spin: int) -> np.ndarray:
        """<c_i(tau) c_j^dagger(0)> in continuous imaginary time, H = H_t + H_U
        with no Trotter split, from the eigenbasis of H: Tr[e^{-(beta-tau)H} c_i
        e^{-tau H} c_j^dagger] / Z, array [len(taus), N, N] (positive convention)."""
        E, V = np.linalg.eigh(self.Ht + self.HU)
        E = E - E.min()
        Z = np.sum(np.exp(-beta * E))
        N = self.N
        C = [V.T @ self.c[i + N * spin] @ V for i in range(N)]
        out = np.zeros((len(taus), N, N))
        for a, tau in enumerate(taus):
            f = np.exp(-(beta - tau) * E)[:, None] * np.exp(-tau * E)[None, :]
            for i in range(N):
                for j in range(N):
                    out[a, i, j] = np.sum(f * C[i] * C[j]) / Z
        return out

    def giw_exact(self, beta: float, n_freq: int, spin: int) -> np.ndarray:
        """G_ij(i w_n) = int_0^beta e^{i w_n tau} G_ij(tau) dtau in the sign of
        eq. (4), G(tau) = -<c_i(tau) c_j^dagger>, w_n = (2n+1) pi / beta, from
        the Lehmann sum over the eigenstates of H = H_t + H_U:
        (1/Z) sum_mn (e^{-beta E_m} + e^{-beta E_n}) <m|c_i|n><n|c_j^dagger|m>
        / (i w_n + E_m - E_n); array [n_freq, N, N] (complex)."""
        E, V = np.linalg.eigh(self.Ht + self.HU)
        E = E - E.min()
        w = np.exp(-beta * E)
        Z = np.sum(w)
        N = self.N
        C = [V.T @ self.c[i + N * spin] @ V for i in range(N)]
        wn = (2 * np.arange(n_freq) + 1) * np.pi / beta
        out = np.zeros((n_freq, N, N), dtype=complex)
        occ = (w[:, None] + w[None, :]) / Z
        dE = E[:, None] - E[None, :]
        for a, x in enumerate(wn):
            den = occ / (1j * x + dE)
            for i in range(N):
                for j in range(N):
                    out[a, i, j] = np.sum(den * C[i] * C[j])
        return out

    def gtau(self, beta: float, dtau: float, spin: int) -> np.ndarray:
        """<c_i(tau_l) c_j^dagger(0)> = Tr[T^{Lam-l} c_i T^l c_j^dagger] / Z for l = 0..Lam
        (positive convention), array [Lam+1, N, N]."""
        lam, P = self.trotter(beta, dtau)
        Z = np.trace(P[lam])
        N = self.N
        out = np.zeros((lam + 1, N, N))
        for l in range(lam + 1):
            for i in range(N):
                A = P[lam - l] @ self.c[i + N * spin]
                for j in range(N):
                    out[l, i, j] = np.trace(A @ P[l] @ self.c[j + N * spin].T) / Z
        return out
