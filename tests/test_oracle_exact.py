"""Pins of the oracle against exact results: brute-force field sums against
Fock-space traces (eqs. (2)-(3)), closed forms at U = 0 and t = 0, and
particle-hole invariants."""
import itertools
import math

import numpy as np
import pytest

from tests.fock import Cluster

T = 0.25


def all_fields(lam, N):
    for bits in itertools.product((1, -1), repeat=lam * N):
        yield np.array(bits, dtype=np.int8).reshape(lam, N)


@pytest.mark.parametrize("U,beta,dtau", [(2.0, 1.0, 0.5), (2.0, 2.0, 0.5), (4.0, 1.2, 0.4)])
def test_bruteforce_z_matches_fock_trace(orc, U, beta, dtau):
    """sum_h C^{N Lam} det M_up det M_dn = Tr[(e^{-dtau H_t} e^{-dtau H_U})^Lam]
    on the 2 x 2 cluster, summing all 2^{N Lam} fields (eqs. (2)-(3))."""
    c = orc.Chain(2, U, T, beta, dtau, 3, 0, 0, 2)
    N, lam = c.N, c.Lam
    C = math.exp(-dtau * U / 4) / 2
    Z = 0.0
    for f in all_fields(lam, N):
        la, sa = c.log_det_M(0, f)
        lb, sb = c.log_det_M(1, f)
        assert sa * sb == 1           # sign-free at half filling
        Z += math.exp(N * lam * math.log(C) + la + lb)
    Zf = Cluster(2, T, U).z_trotter(beta, dtau)
    assert abs(Z - Zf) < 1e-12 * Zf


@pytest.mark.parametrize("U,beta,dtau", [(2.0, 1.5, 0.5), (3.0, 1.0, 0.5)])
def test_bruteforce_observables_match_fock(orc, U, beta, dtau):
    """Weighted field averages of the per-field estimators equal the Trotter
    traces: double occupancy at tau = 0 and G(tau_l, 0) for all l."""
    c = orc.Chain(2, U, T, beta, dtau, 5, 0, 0, 2)
    N, lam = c.N, c.Lam
    Zw = 0.0
    D = 0.0
    Gt = np.zeros((2, lam + 1, N, N))
    gk = np.zeros((lam + 1, N))
    for f in all_fields(lam, N):
        la, _ = c.log_det_M(0, f)
        lb, _ = c.log_det_M(1, f)
        w = math.exp(la + lb)
        Zw += w
        Gu = c.fresh_green(1, 0, f)
        Gd = c.fresh_green(1, 1, f)
        D += w * np.mean((1 - np.diag(Gu)) * (1 - np.diag(Gd)))
        for s in range(2):
            for l in range(lam + 1):
                Gt[s, l] += w * c.gtau0(l, s, f)
        c.set_field(f)
        gk += w * c.measure()[1]
    D /= Zw
    Gt /= Zw
    gk /= Zw
    cl = Cluster(2, T, U)
    assert abs(D - cl.double_occ(beta, dtau)) < 1e-12
    for s in range(2):
        ref = cl.gtau(beta, dtau, s)
        assert np.max(np.abs(Gt[s] - ref)) < 1e-12
    # k-resolved, paper sign: -1/2 sum_s (1/N) sum_ij cos(k.(r_i - r_j)) G_ij
    L = 2
    ref_k = np.zeros((lam + 1, N))
    for s in range(2):
        G = cl.gtau(beta, dtau, s)
        for k in range(N):
            kx, ky = 2 * math.pi * (k % L) / L, 2 * math.pi * (k // L) / L
            ph = np.array([[math.cos(kx * ((i % L) - (j % L)) + ky * ((i // L) - (j // L)))
                            for j in range(N)] for i in range(N)])
            ref_k[:, k] += -0.5 * np.einsum("lij,ij->l", G, ph) / N
    assert np.max(np.abs(gk - ref_k)) < 1e-12


def dispersion(L):
    return np.array([-2 * T * (math.cos(2 * math.pi * (k % L) / L) + math.cos(2 * math.pi * (k // L) / L))
                     for k in range(L * L)])


@pytest.mark.parametrize("L,beta,dtau", [(4, 4.0, 0.5), (4, 20.0, 0.5), (6, 10.0, 0.4)])
def test_u0_closed_form(orc, L, beta, dtau):
    """U = 0: every proposal has R = 1, the sweep keeps G exact and
    G(tau_l, k) = -e^{-eps_k tau_l} / (1 + e^{-beta eps_k}), D = 1/4."""
    c = orc.Chain(L, 0.0, T, beta, dtau, 9, 0, 0, 4)
    c.sweep(2)
    st = c.stats()
    assert st["accepted"] == st["proposals"]
    d, gk = c.measure()
    eps = dispersion(L)
    tau = np.arange(c.Lam + 1) * dtau
    ref = -np.exp(-np.outer(tau, eps)) / (1 + np.exp(-beta * eps))
    assert abs(d - 0.25) < 1e-12
    assert np.max(np.abs(gk - ref)) < 1e-12
    assert st["drift_max"] < 1e-12


def binned_mean_err(x, nbins=20):
    x = np.asarray(x)
    m = len(x) // nbins
    b = x[: m * nbins].reshape(nbins, m, *x.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / math.sqrt(nbins)


def test_atomic_limit_within_error_bars(orc):
    """t = 0: sites decouple and the Trotter product is exact;
    D = 1/(2(1 + e^{beta U/2})), G(tau) = -cosh(U(beta-2tau)/4)/(2 cosh(beta U/4))."""
    U, beta, dtau, L = 2.0, 4.0, 0.5, 4
    c = orc.Chain(L, U, 0.0, beta, dtau, 21, 0, 0, 4)
    c.sweep(50)
    ds, gs = [], []
    for _ in range(600):
        c.sweep(1)
        d, g = c.measure()
        ds.append(d)
        gs.append(g)
    dm, de = binned_mean_err(ds)
    gm, ge = binned_mean_err(gs)
    dref = 1 / (2 * (1 + math.exp(beta * U / 2)))
    tau = np.arange(c.Lam + 1) * dtau
    gref = -np.cosh(U * (beta - 2 * tau) / 4) / (2 * math.cosh(beta * U / 4))
    assert abs(dm - dref) < 4 * de + 1e-12
    z = np.abs(gm - gref[:, None]) / (ge + 1e-12)
    assert np.all(z < 5), z.max()


def test_particle_hole_invariants(orc):
    """Bipartite lattice at mu = 0: per field G_dn = I - P G_up^T P with
    P = diag((-1)^{x+y}), R_dn = R_up e^{2 lambda h}, and det M_up det M_dn > 0."""
    L = 4
    c = orc.Chain(L, 2.0, T, 4.0, 0.5, 33, 0, 0, 4)
    P = np.diag([(-1) ** ((i % L) + (i // L)) for i in range(L * L)])
    for _ in range(3):
        c.step_slices(3)
        Gu, Gd = c.green(0), c.green(1)
        assert np.max(np.abs(Gd - (np.eye(L * L) - P @ Gu.T @ P))) < 1e-10
        l = c.slice
        f = c.field()
        for i in range(0, L * L, 5):
            ru, rd = c.ratio(l, i)
            assert abs(rd - ru * math.exp(2 * c.lam * f[l - 1, i])) < 1e-10 * abs(rd)
        la, sa = c.log_det_M(0)
        lb, sb = c.log_det_M(1)
        assert sa * sb == 1
