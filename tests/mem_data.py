"""Seeded synthetic ingredients for the maximum-entropy tests; none of the
method's arithmetic is here (the tests form G(tau) from them with the
oracle's eq. (4)).

The spectrum is particle-hole symmetric and shaped like that of the
half-filled Hubbard model at k = (pi, 0) for U = 2, t = 0.25: lower and upper
Hubbard bands at -+1.2 and a narrow quasiparticle peak at 0, on a uniform
w grid; the noise is independent Gaussian with one standard error for all
tau points; the default model is flat over the grid."""
import numpy as np


def two_band_spectrum(w):
    """Normalised so that the trapezoid sum over the grid is 1."""
    A = (0.5 * np.exp(-(w - 1.2) ** 2 / 0.18) + 0.5 * np.exp(-(w + 1.2) ** 2 / 0.18)
         + 0.6 * np.exp(-w ** 2 / 0.045))
    h = np.diff(w)
    return A / float(np.sum(0.5 * h * (A[:-1] + A[1:])))


def ingredients(beta, n_tau, n_w, noise, seed, w_max=4.0):
    """(tau, w, A, noise draws [n_tau], sigma, default model)."""
    w = np.linspace(-w_max, w_max, n_w)
    tau = np.linspace(0.0, beta, n_tau)
    rng = np.random.default_rng(seed)
    return (tau, w, two_band_spectrum(w), noise * rng.standard_normal(n_tau), np.full(n_tau, noise),
            np.full(n_w, 1.0 / (2 * w_max)))
