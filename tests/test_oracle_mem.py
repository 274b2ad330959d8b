"""Pins of the oracle's maximum-entropy step (oracle/mem.py): eq. (4) on a
single level against the free-fermion closed form, the second-order
agreement with ridge regression (the closed-form minimiser of the quadratic
expansion of Q about the default model), the alpha -> infinity limit, a
brute-force minimisation on a two-point grid, the historic alpha, and the
smoothing that Sec. 3 uses the method for."""
import math

import numpy as np
import pytest

from oracle import mem
from tests.mem_data import ingredients, two_band_spectrum

BETA = 20.0


def synthetic_green(beta, n_tau, n_w, noise, seed):
    """(tau, noisy G, sigma, w, m): the two-band spectrum through the
    oracle's eq. (4) plus seeded noise."""
    tau, w, A, eta, sig, m = ingredients(beta, n_tau, n_w, noise, seed)
    return tau, mem.green(tau, w, A, beta) + eta, sig, w, m


@pytest.mark.parametrize("beta", [1.0, 20.0, 200.0])
def test_eq4_of_a_single_level_is_the_free_green_function(beta):
    """A = delta(w - eps) (one grid point carrying weight 1/q_k) gives
    G(tau) = -e^{-eps tau} / (1 + e^{-beta eps}), the U = 0 Green function of
    a level at eps, for eps of both signs and beta |eps| up to 800 (no
    overflow); G(0) + G(beta) = -1."""
    w = np.linspace(-4, 4, 81)
    q = mem.trapezoid_weights(w)
    tau = np.linspace(0, beta, 33)
    for k in (0, 20, 40, 61, 80):
        A = np.zeros_like(w)
        A[k] = 1.0 / q[k]
        eps = w[k]
        with np.errstate(over="ignore"):
            ref = np.array([-math.exp(-eps * t) / (1 + math.exp(-beta * eps)) if eps >= 0 else
                            -math.exp(eps * (beta - t)) / (math.exp(eps * beta) + 1) for t in tau])
        got = mem.green(tau, w, A, beta)
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref)) < 1e-15
        assert abs(got[0] + got[-1] + 1.0) < 1e-15


def test_trapezoid_weights_integrate_linear_functions_exactly():
    w = np.sort(np.random.default_rng(3).uniform(-3, 5, 17))
    q = mem.trapezoid_weights(w)
    assert abs(q.sum() - (w[-1] - w[0])) < 1e-14
    assert abs(q @ (2 * w - 1) - ((w[-1] ** 2 - w[0] ** 2) - (w[-1] - w[0]))) < 1e-13


def test_gradient_against_finite_differences():
    """dQ/dA against central differences of Q itself at a random A > 0."""
    tau, G, sig, w, m = synthetic_green(BETA, n_tau=21, n_w=41, noise=1e-3, seed=2)
    P = mem.Problem(tau, G, sig, BETA, w, m)
    A = m * np.exp(np.random.default_rng(4).uniform(-1, 1, len(w)))
    alpha = 3.0
    g = P.gradient(A, alpha)
    h = 1e-6
    for j in range(0, len(w), 5):
        e = np.zeros_like(A)
        e[j] = h * A[j]
        fd = (P.Q(A + e, alpha) - P.Q(A - e, alpha)) / (2 * e[j])
        assert abs(fd - g[j]) < 1e-6 * (abs(g[j]) + 1e-3 * np.max(np.abs(g))), j


def test_near_the_default_model_mem_is_ridge_regression_to_second_order():
    """Q = chi^2/2 - alpha S with S = -sum q (A - m)^2 / (2m) + O((A - m)^3):
    for data made from A = m (1 + e f) the minimiser differs from the ridge
    solution A_r = m + (B^T B + alpha diag(q/m))^{-1} B^T (d - B m) by
    O(e^2).  Halving e quarters the difference (a missing factor anywhere in
    chi^2, S or the kernel would leave an O(e) difference, halved)."""
    w = np.linspace(-3, 3, 61)
    tau = np.linspace(0, BETA, 41)
    m = np.full_like(w, 1.0 / 6.0)
    f = np.cos(2 * w) * np.exp(-w ** 2)
    sig = np.full_like(tau, 1e-3)
    alpha = 2.0
    diffs = []
    for e in (1e-3, 5e-4):
        G = mem.green(tau, w, m * (1 + e * f), BETA)
        P = mem.Problem(tau, G, sig, BETA, w, m)
        A = P.solve(alpha)
        Ar = m + np.linalg.solve(P.B.T @ P.B + np.diag(alpha * P.q / m), P.B.T @ (P.d - P.B @ m))
        assert np.max(np.abs(Ar - m)) > 1e-3 * e * np.max(m)   # the perturbation is seen
        diffs.append(np.max(np.abs(A - Ar)))
    ratio = diffs[0] / diffs[1]
    assert 3.6 < ratio < 4.4, (diffs, ratio)


def test_large_alpha_gives_the_default_model():
    """alpha -> infinity: the entropy wins, A -> m with A - m = O(1/alpha)."""
    tau, G, sig, w, m = synthetic_green(BETA, n_tau=21, n_w=41, noise=1e-2, seed=1)
    devs = []
    for alpha in (1e8, 1e9):
        A, _, _ = mem.spectrum(tau, G, sig, BETA, w, m, alpha)
        devs.append(np.max(np.abs(A - m)))
    assert devs[0] < 1e-4 * np.max(m)
    assert 9.0 < devs[0] / devs[1] < 11.0


def test_two_point_grid_against_brute_force():
    """M = 2: Q on a dense grid of (A_1, A_2) > 0, refined around its
    minimum, against the Newton minimiser."""
    beta = 4.0
    w = np.array([-0.7, 0.9])
    tau = np.linspace(0, beta, 5)
    m = np.array([0.4, 0.6])
    G = mem.green(tau, w, np.array([0.3, 0.85]), beta) + 1e-3 * np.array([1, -2, 0.5, 1, -1])
    sig = np.full_like(tau, 0.01)
    alpha = 0.5
    P = mem.Problem(tau, G, sig, beta, w, m)
    A = P.solve(alpha)
    c, span = np.array([0.5, 0.5]), 0.49
    for _ in range(12):
        a1 = np.linspace(c[0] - span, c[0] + span, 81)
        a2 = np.linspace(c[1] - span, c[1] + span, 81)
        Qs = np.array([[P.Q(np.array([x, y]), alpha) for y in a2] for x in a1])
        i, j = np.unravel_index(np.argmin(Qs), Qs.shape)
        c, span = np.array([a1[i], a2[j]]), span / 8
    assert np.max(np.abs(A - c)) < 1e-9


def test_historic_alpha_and_monotone_chi2():
    tau, G, sig, w, m = synthetic_green(BETA, n_tau=41, n_w=121, noise=1e-4, seed=7)
    A, alpha, chi2 = mem.spectrum(tau, G, sig, BETA, w, m)
    assert abs(chi2 - len(tau)) < 1e-8 * len(tau)
    c = [mem.spectrum(tau, G, sig, BETA, w, m, a)[2] for a in (alpha / 10, alpha, alpha * 10)]
    assert c[0] < c[1] < c[2]
    assert np.all(A > 0)


def test_smoothing_brings_noisy_data_closer_to_the_exact_green_function():
    """Sec. 3: the G(tau) given back by the MEM spectrum (eq. (4)) is closer
    to the exact G than the noisy data it was fitted to, and keeps the sum
    rule and the particle-hole symmetry of the spectrum within the noise."""
    rms = lambda x: float(np.sqrt(np.mean(x ** 2)))
    ratios = []
    for seed in (0, 1, 2, 11):
        tau, G, sig, w, m = synthetic_green(BETA, n_tau=81, n_w=121, noise=1e-4, seed=seed)
        exact = mem.green(tau, w, two_band_spectrum(w), BETA)
        A, _, _ = mem.spectrum(tau, G, sig, BETA, w, m)
        Gs = mem.green(tau, w, A, BETA)
        ratios.append(rms(Gs - exact) / rms(G - exact))
        assert abs(Gs[0] + Gs[-1] + 1.0) < 5e-4
        assert np.max(np.abs(Gs - Gs[::-1])) < 5e-4
    assert max(ratios) < 0.8 and np.mean(ratios) < 0.6, ratios


def test_historic_alpha_that_does_not_exist_is_an_error():
    """Noise whose own chi^2 is 98 for 81 points: no A >= 0 brings chi^2 down
    to 81 (the best fit stays near 84), so the historic alpha does not
    exist and the oracle says so."""
    tau, G, sig, w, m = synthetic_green(BETA, n_tau=81, n_w=121, noise=1e-4, seed=3)
    with pytest.raises(RuntimeError):
        mem.spectrum(tau, G, sig, BETA, w, m)
