"""Post-processing of the sweep's output, computed plainly -- TEST
INFRASTRUCTURE ONLY (part of the oracle; only the tests, the smoke check and
the benchmark's cpu_baseline leg may use it).

What the paper does with the Green functions after the sweep (Rost &
Bluemer, "Deciding the fate of the false Mott transition in two dimensions
by exact quantum Monte Carlo methods"):

- Trotter elimination (Sec. 3, "Trotter bias" paragraph): the G(tau) of each
  slice width dtau are aligned on a common fine tau grid by splines and
  extrapolated pointwise to dtau -> 0.
- the Matsubara transform of eq. (5) and the Dyson self-energy of eq. (6);
- the finite-size extrapolation of the self-energy in 1/L^2 (Sec. 3, last
  paragraph): linear and quadratic fits, their average as the result and
  their difference as the error bar;
- the real-space spin correlation function and its correlation length from an
  exponential fit (Sec. 4, Fig. 5).

Readings where the paper is silent (the same readings the library takes):
- splines are cubic with not-a-knot ends, one per k through the slice grid
  tau_l = l dtau, l = 0..Lambda;
- the dtau -> 0 extrapolation is a least-squares polynomial in dtau^2 of
  order min(2, number of grids - 1);
- eq. (5) with the sign of eq. (4)'s convention: G(i w_n) = int_0^beta dtau
  G(tau) e^{+i w_n tau}, w_n = (2n + 1) pi / beta (e^{-i w_n tau} as printed
  would contradict eq. (6));
- the error bar of the finite-size extrapolation is |linear - quadratic|;
- the spin correlation is C(r) = (1/N) sum_i <S^z_i S^z_{i+r}>, S^z =
  (n_up - n_dn)/2, from Wick's theorem for each field; the correlation length
  comes from a least-squares fit of log|C| linear in the distance, over
  1 <= x <= L/2 along the lattice axes (|C(x, 0)| and |C(0, x)| averaged).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline


def slice_grid(beta: float, dtau: float) -> np.ndarray:
    """tau_l = l dtau, l = 0..Lambda (eq. (2): Lambda = beta / dtau)."""
    lam = int(round(beta / dtau))
    return np.arange(lam + 1) * dtau


def align(dtau: float, beta: float, G: np.ndarray, tau_fine: np.ndarray) -> np.ndarray:
    """G [Lambda + 1, ...] on the slice grid of dtau, spline-interpolated to
    tau_fine (Sec. 3, Trotter bias: aligning the raw data on a common grid)."""
    return CubicSpline(slice_grid(beta, dtau), G, axis=0, bc_type="not-a-knot")(tau_fine)


def trotter_extrapolate(dtaus, Gs, beta: float, tau_fine: np.ndarray) -> np.ndarray:
    """Pointwise dtau -> 0 extrapolation (Sec. 3, Trotter bias): the aligned
    values at each fine-grid point and k are fitted by least squares with a
    polynomial in dtau^2 of order min(2, len(dtaus) - 1); its constant term
    is returned, shape [len(tau_fine), ...]."""
    assert len(dtaus) == len(Gs) and len(dtaus) >= 2
    aligned = np.stack([align(dt, beta, G, tau_fine) for dt, G in zip(dtaus, Gs)])   # [A, M, ...]
    x = np.asarray(dtaus, dtype=float) ** 2
    order = min(2, len(dtaus) - 1)
    V = np.vander(x, order + 1, increasing=True)                                   # [A, order + 1]
    flat = aligned.reshape(len(dtaus), -1)
    coef, *_ = np.linalg.lstsq(V, flat, rcond=None)
    return coef[0].reshape(aligned.shape[1:])


def matsubara_frequencies(beta: float, n: int) -> np.ndarray:
    return (2 * np.arange(n) + 1) * np.pi / beta


def matsubara(tau: np.ndarray, G: np.ndarray, beta: float, n_freq: int) -> np.ndarray:
    """eq. (5): G(i w_n) = int_0^beta G(tau) e^{+i w_n tau} dtau for the cubic
    not-a-knot spline through (tau, G), by Gauss-Legendre quadrature on every
    spline interval, subdivided so that w_n h <= 1 (the quadrature is then
    exact to rounding for the smooth integrand)."""
    sp = CubicSpline(tau, G, bc_type="not-a-knot")
    wn = matsubara_frequencies(beta, n_freq)
    xg, wg = np.polynomial.legendre.leggauss(24)
    out = np.zeros(n_freq, dtype=complex)
    for n, w in enumerate(wn):
        acc = 0.0 + 0.0j
        for a, b in zip(tau[:-1], tau[1:]):
            nsub = int(np.ceil(w * (b - a))) + 1
            edges = np.linspace(a, b, nsub + 1)
            for u, v in zip(edges[:-1], edges[1:]):
                t = 0.5 * (v - u) * xg + 0.5 * (u + v)
                acc += 0.5 * (v - u) * np.sum(wg * sp(t) * np.exp(1j * w * t))
        out[n] = acc
    return out


def dyson(w: np.ndarray, eps_k: float, mu: float, G_iw: np.ndarray) -> np.ndarray:
    """eq. (6): Sigma_k(i w_n) = i w_n + mu - eps_k - 1 / G_k(i w_n)."""
    return 1j * w + mu - eps_k - 1.0 / G_iw


def finite_size_extrapolate(Ls, values):
    """Sec. 3, finite-size extrapolation: values [len(Ls), ...] (real or
    complex) against 1/L^2, least-squares fits of first and second order;
    returns (average of the two constant terms, |linear - quadratic|,
    linear, quadratic)."""
    x = 1.0 / np.asarray(Ls, dtype=float) ** 2
    y = np.asarray(values).reshape(len(Ls), -1)
    out = []
    for order in (1, 2):
        V = np.vander(x, order + 1, increasing=True)
        coef, *_ = np.linalg.lstsq(V.astype(y.dtype), y, rcond=None)
        out.append(coef[0])
    lin, quad = out
    shape = np.asarray(values).shape[1:]
    return (0.5 * (lin + quad)).reshape(shape), np.abs(lin - quad).reshape(shape), lin.reshape(shape), \
        quad.reshape(shape)


def spin_correlation(G_up: np.ndarray, G_dn: np.ndarray, L: int) -> np.ndarray:
    """C(r) = (1/N) sum_i <S^z_i S^z_{i+r}> for one field, from the
    equal-time Green functions G_sigma = <c c^+> by Wick's theorem (the spins
    decouple for a fixed field): <n_i s> = 1 - G_s,ii,
    <n_i s n_j s> = <n_i s><n_j s> + (delta_ij - G_s,ji) G_s,ij,
    <n_i s n_j s'> = <n_i s><n_j s'> for s != s'.  r = dx + L dy."""
    N = L * L
    Gs = (G_up, G_dn)
    n = [1.0 - np.diag(G) for G in Gs]
    C = np.zeros(N)
    for i in range(N):
        xi, yi = i % L, i // L
        for r in range(N):
            j = (xi + r % L) % L + L * ((yi + r // L) % L)
            acc = 0.0
            for a in range(2):
                for b in range(2):
                    sab = 1.0 if a == b else -1.0
                    nn = n[a][i] * n[b][j]
                    if a == b:
                        nn += ((1.0 if i == j else 0.0) - Gs[a][j, i]) * Gs[a][i, j]
                    acc += sab * nn
            C[r] += 0.25 * acc
    return C / N


def correlation_length(C: np.ndarray, L: int):
    """Sec. 4 (Fig. 5): exponential fit |C(x)| = A e^{-x/xi} over
    1 <= x <= L/2 along the axes (|C(x, 0)| and |C(0, x)| averaged), by least
    squares on log|C|.  Returns (xi, A)."""
    xs = np.arange(1, L // 2 + 1)
    c = 0.5 * (np.abs(C[xs]) + np.abs(C[xs * L]))
    slope, icpt = np.polyfit(xs, np.log(c), 1)
    return -1.0 / slope, float(np.exp(icpt))
