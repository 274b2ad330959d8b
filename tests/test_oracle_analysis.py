"""Pins of the oracle's post-processing (oracle/analysis.py) against exact
results: polynomial data the splines reproduce, the U = 0 closed forms,
particle-hole symmetry, 80-digit quadrature, and a brute-force field sum
against Fock-space traces for the spin correlation."""
import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import analysis as an
from tests.fock import Cluster

T = 0.25


def cubic(c, tau):
    return c[0] + c[1] * tau + c[2] * tau ** 2 + c[3] * tau ** 3


def test_trotter_extrapolation_recovers_polynomial_data():
    """G_dtau(tau) = f(tau) + a(tau) dtau^2 + b(tau) dtau^4 with cubic f, a, b:
    the not-a-knot splines reproduce cubics exactly, so the dtau^2 fit of
    order 2 over three grids returns f on the fine grid to rounding, and the
    order-1 fit over two grids does when b = 0."""
    rng = np.random.default_rng(5)
    beta = 4.0
    f, a, b = rng.standard_normal((3, 4, 2))           # two "k points"
    tau_f = np.linspace(0, beta, 161)
    want = np.stack([cubic(f[:, k], tau_f) for k in range(2)], axis=1)

    def data(dt, with_b):
        tau = an.slice_grid(beta, dt)
        return np.stack([cubic(f[:, k], tau) + cubic(a[:, k], tau) * dt ** 2
                         + (cubic(b[:, k], tau) * dt ** 4 if with_b else 0) for k in range(2)], axis=1)

    dts = [0.4, 0.5, 0.8]
    got = an.trotter_extrapolate(dts, [data(d, True) for d in dts], beta, tau_f)
    assert np.max(np.abs(got - want)) < 1e-11
    got2 = an.trotter_extrapolate(dts[:2], [data(d, False) for d in dts[:2]], beta, tau_f)
    assert np.max(np.abs(got2 - want)) < 1e-11
    # the extrapolation is in dtau^2: fitting the same data as if it were
    # linear in dtau would leave a visible error
    x = np.array(dts[:2])
    V = np.vander(x, 2, increasing=True)
    al = np.stack([an.align(d, beta, data(d, False), tau_f) for d in dts[:2]])
    wrong = np.linalg.lstsq(V, al.reshape(2, -1), rcond=None)[0][0].reshape(want.shape)
    assert np.max(np.abs(wrong - want)) > 1e-3


def test_trotter_extrapolation_of_u0_data():
    """U = 0 has no Trotter error: G_k(tau_l) = -e^{-eps tau}/(1 + e^{-beta eps})
    on every grid.  Where all grids share a node (tau = 0 and 4 for dtau =
    0.4, 0.5, 0.8 at beta = 4) the extrapolation is exact; in between only
    the splines' interpolation error remains."""
    beta, dts = 4.0, [0.4, 0.5, 0.8]
    eps = np.array([-1.0, -0.5, 0.0, 0.7])
    ref = lambda tau: -np.exp(-np.outer(tau, eps)) / (1 + np.exp(-beta * eps))
    tau_f = np.linspace(0, beta, 81)
    got = an.trotter_extrapolate(dts, [ref(an.slice_grid(beta, d)) for d in dts], beta, tau_f)
    common = [0, 80]
    assert np.max(np.abs(got[common] - ref(tau_f[common]))) < 1e-14
    assert np.max(np.abs(got - ref(tau_f))) < 2e-3


def test_matsubara_of_a_cubic_against_high_precision_quadrature():
    """eq. (5) with e^{+i w_n tau} for a cubic G(tau): the spline is the cubic
    itself, so the transform equals the 40-digit integral."""
    beta = 5.0
    c = [-0.3, 0.11, -0.05, 0.013]
    tau = np.linspace(0, beta, 26)
    got = an.matsubara(tau, cubic(c, tau), beta, 12)
    with mpmath.workdps(40):
        for n in range(12):
            w = (2 * n + 1) * mpmath.pi / beta
            ref = mpmath.quad(lambda x: (c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3) * mpmath.exp(1j * w * x),
                              [0, beta])
            assert abs(got[n] - complex(ref)) < 1e-12, n


@pytest.mark.parametrize("eps", [-0.8, -0.2, 0.0, 0.5])
def test_u0_transform_and_dyson(eps):
    """U = 0: G(tau) = -e^{-eps tau}/(1 + e^{-beta eps}) transforms to
    1/(i w_n - eps) and eq. (6) gives Sigma = mu = 0 at half filling; at
    eps = 0 (k = (pi, 0)) G(tau) = -1/2, G(i w_n) = 1/(i w_n) is purely
    imaginary and Re Sigma vanishes exactly."""
    beta = 10.0
    tau = np.linspace(0, beta, 401)
    G = -np.exp(-eps * tau) / (1 + np.exp(-beta * eps))
    giw = an.matsubara(tau, G, beta, 20)
    w = an.matsubara_frequencies(beta, 20)
    assert np.max(np.abs(giw - 1 / (1j * w - eps))) < 1e-7
    sig = an.dyson(w, eps, 0.0, giw)
    assert np.max(np.abs(sig)) < 1e-5
    if eps == 0.0:
        assert np.max(np.abs(giw.real)) < 1e-14 and np.max(np.abs(sig.real)) < 1e-12


def test_finite_size_extrapolation():
    """Values a + b L^-2 + c L^-4: the quadratic fit returns a; the linear fit
    is the least-squares line; result = their average, error = their
    difference."""
    Ls = np.array([8, 10, 12, 14, 16])
    x = 1.0 / Ls ** 2
    a, b, c = 0.3 - 0.2j, -4.0 + 1.0j, 30.0 - 5.0j
    vals = a + b * x + c * x ** 2
    val, err, lin, quad = an.finite_size_extrapolate(Ls, vals)
    assert abs(quad - a) < 1e-12
    slope, icpt = np.polyfit(x, vals.real, 1)[0], np.polyfit(x, vals.real, 1)[1]
    assert abs(lin.real - icpt) < 1e-12 and abs(lin.imag - np.polyfit(x, vals.imag, 1)[1]) < 1e-12
    assert abs(val - 0.5 * (lin + quad)) < 1e-15 and abs(err - abs(lin - quad)) < 1e-15
    assert err > 1e-4   # the curvature makes the two fits differ


def free_green(L, beta):
    """U = 0 equal-time G_ij = <c_i c_j^+> = (1/N) sum_k e^{ik(r_i - r_j)} (1 - f(eps_k))."""
    N = L * L
    G = np.zeros((N, N))
    for k in range(N):
        kx, ky = 2 * math.pi * (k % L) / L, 2 * math.pi * (k // L) / L
        e = -2 * T * (math.cos(kx) + math.cos(ky))
        occ = 1.0 / (1.0 + math.exp(beta * e))
        ph = np.array([kx * (i % L) + ky * (i // L) for i in range(N)])
        G += np.cos(ph[:, None] - ph[None, :]) * (1 - occ)
    return G / N


def test_spin_correlation_u0_closed_form():
    """U = 0 (both spins free, same G): C(0) = n(1 - n)/2 = 1/8 at n = 1/2 and
    C(r) = -G_0r G_r0 / 2 otherwise."""
    L, beta = 4, 6.0
    G = free_green(L, beta)
    C = an.spin_correlation(G, G, L)
    assert abs(C[0] - 0.125) < 1e-14
    for r in range(1, L * L):
        assert abs(C[r] + 0.5 * G[0, r] * G[r, 0]) < 1e-14


def test_spin_correlation_bruteforce_against_fock(orc):
    """2 x 2, Lambda = 2: the weighted sum over all 2^8 fields of the per-field
    Wick estimator equals Tr[T^Lambda S^z_0 S^z_r] / Z_dtau in Fock space."""
    U, beta, dtau, L = 2.0, 1.0, 0.5, 2
    c = orc.Chain(L, U, T, beta, dtau, 5, 0, 0, 2)
    N, lam = c.N, c.Lam
    Zw, C = 0.0, np.zeros(N)
    for bits in itertools.product((1, -1), repeat=lam * N):
        f = np.array(bits, dtype=np.int8).reshape(lam, N)
        la, _ = c.log_det_M(0, f)
        lb, _ = c.log_det_M(1, f)
        w = math.exp(la + lb)
        Zw += w
        C += w * an.spin_correlation(c.fresh_green(1, 0, f), c.fresh_green(1, 1, f), L)
    C /= Zw
    cl = Cluster(L, T, U)
    lamT, P = cl.trotter(beta, dtau)
    Sz = [0.5 * (cl.c[i].T @ cl.c[i] - cl.c[i + N].T @ cl.c[i + N]) for i in range(N)]
    Z = np.trace(P[lamT])
    for r in range(N):
        ref = np.trace(P[lamT] @ Sz[0] @ Sz[r]) / Z
        assert abs(C[r] - ref) < 1e-12, r
    assert C[1] < 0 < C[0]   # antiferromagnetic neighbours


def test_correlation_length_of_exact_exponential():
    L, xi, A = 16, 3.7, 0.21
    N = L * L
    C = np.zeros(N)
    for r in range(N):
        x, y = r % L, r // L
        d = min(x, L - x) + min(y, L - y)
        C[r] = A * (-1) ** (x + y) * math.exp(-d / xi)
    got_xi, got_A = an.correlation_length(C, L)
    assert abs(got_xi - xi) < 1e-12 and abs(got_A - A) < 1e-13
