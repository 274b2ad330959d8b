"""Maximum-entropy regularisation of G(tau), computed plainly -- TEST
INFRASTRUCTURE ONLY (part of the oracle; only the tests, the smoke check and
the benchmark's cpu_baseline leg may use it).

Sec. 3 (Trotter-bias paragraph) smooths the extrapolated G(tau) by a maximum
entropy method: a spectral function A(w) >= 0 is fitted to the data through
eq. (4),

    G(tau) = - int dw A(w) e^{-w tau} / (1 + e^{-w beta}),

and only the G(tau) that this A(w) gives back is used further.  The paper
names neither the entropy, the default model, the choice of alpha nor the w
grid.  Readings (the library takes the same):

- A lives on a caller-given increasing grid w_j with trapezoid weights q_j;
  eq. (4) becomes G_i = - sum_j q_j K(tau_i, w_j) A_j;
- the misfit is chi^2 = sum_i ((G_i(A) - Gbar_i) / sigma_i)^2 with one
  standard error per tau point (no covariance);
- the entropy is Shannon-Jaynes relative to a caller-given default model m > 0,
  S = sum_j q_j (A_j - m_j - A_j ln(A_j / m_j));
- A minimises Q = chi^2 / 2 - alpha S (strictly convex in A > 0, so the
  minimiser is unique) at a fixed alpha, or at the "historic" alpha where
  chi^2 = number of tau points.

The minimisation is Newton's method on the convex Q in A itself, with the
exact gradient and Hessian written out below, backtracking and steps that
keep A > 0; the historic alpha is a bracketed root (Brent) of
chi^2(alpha) - n in ln alpha, every alpha solved from A = m.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def trapezoid_weights(w: np.ndarray) -> np.ndarray:
    """q_j of the trapezoid rule on the grid w (int f dw ~ sum_j q_j f(w_j))."""
    w = np.asarray(w, dtype=float)
    q = np.zeros_like(w)
    h = np.diff(w)
    q[:-1] += 0.5 * h
    q[1:] += 0.5 * h
    return q


def kernel(tau: np.ndarray, w: np.ndarray, beta: float) -> np.ndarray:
    """K(tau_i, w_j) = e^{-w tau} / (1 + e^{-w beta}) of eq. (4), written for
    w < 0 as e^{w (beta - tau)} / (e^{w beta} + 1) so nothing overflows."""
    t = np.asarray(tau, dtype=float)[:, None]
    x = np.asarray(w, dtype=float)[None, :]
    pos = np.exp(-np.maximum(x, 0) * t) / (1 + np.exp(-np.maximum(x, 0) * beta))
    neg = np.exp(np.minimum(x, 0) * (beta - t)) / (np.exp(np.minimum(x, 0) * beta) + 1)
    return np.where(x >= 0, pos, neg)


def green(tau, w, A, beta):
    """eq. (4) on the grid: G(tau_i) = - sum_j q_j K(tau_i, w_j) A_j."""
    return -kernel(tau, w, beta) @ (trapezoid_weights(w) * np.asarray(A, dtype=float))


class Problem:
    """chi^2, S and Q for the data (tau, G, sigma) and the grid (w, m)."""

    def __init__(self, tau, G, sigma, beta, w, m):
        self.G = np.asarray(G, dtype=float)
        self.sigma = np.asarray(sigma, dtype=float)
        self.m = np.asarray(m, dtype=float)
        self.q = trapezoid_weights(w)
        # B[i, j] = d G_i(A) / d A_j / sigma_i
        self.B = -kernel(tau, w, beta) * self.q[None, :] / self.sigma[:, None]
        self.d = self.G / self.sigma

    def residual(self, A):
        return self.B @ A - self.d

    def chi2(self, A):
        r = self.residual(A)
        return float(r @ r)

    def entropy(self, A):
        return float(np.sum(self.q * (A - self.m - A * np.log(A / self.m))))

    def Q(self, A, alpha):
        return 0.5 * self.chi2(A) - alpha * self.entropy(A)

    def gradient(self, A, alpha):
        """dQ/dA = B^T r + alpha q ln(A/m)   (dS/dA_j = -q_j ln(A_j/m_j))."""
        return self.B.T @ self.residual(A) + alpha * self.q * np.log(A / self.m)

    def hessian(self, A, alpha):
        """d2Q/dA2 = B^T B + alpha diag(q / A), positive definite for A > 0."""
        return self.B.T @ self.B + np.diag(alpha * self.q / A)

    def solve(self, alpha, A0=None, max_iter=5000):
        """The minimiser A of Q at this alpha by Newton's method with
        backtracking (Armijo) from A0 (default m), each step cut to keep
        A > 0; the Newton system is solved in the variables A^{-1/2} dA,
        where it is well scaled.  Once the Newton decrement -g.dA (twice
        the predicted decrease of Q) is below 1e-10 |Q|, the iteration is in
        its quadratic phase and takes full steps until no component of A
        changes by more than 1e-8 of itself, which leaves every component at
        the rounding floor of the gradient (the decrement alone weighs
        components by their curvature and would leave small A_j behind)."""
        A = self.m.copy() if A0 is None else np.array(A0, dtype=float)
        Qa = self.Q(A, alpha)
        quadratic = False
        for _ in range(max_iter):
            if not np.min(A) > 1e-290:
                raise RuntimeError("MEM oracle: A underflows (alpha too small for these data)")
            g = self.gradient(A, alpha)
            D = np.sqrt(A)
            dA = D * np.linalg.solve(D[:, None] * self.hessian(A, alpha) * D[None, :], -D * g)
            dec = -float(g @ dA)
            quadratic = quadratic or dec <= 1e-10 * max(1.0, abs(Qa))
            if quadratic:
                if not np.all(A + dA > 0):
                    raise RuntimeError("MEM oracle: full step leaves A > 0 in the quadratic phase")
                A = A + dA
                if np.max(np.abs(dA) / A) <= 1e-8:
                    return A
                Qa = self.Q(A, alpha)
                continue
            t = 1.0
            neg = dA < 0
            if np.any(neg):
                t = min(1.0, 0.99 * float(np.min(-A[neg] / dA[neg])))
            while True:
                An = A + t * dA
                Qn = self.Q(An, alpha)
                if Qn <= Qa - 1e-4 * t * dec:
                    break
                t *= 0.5
                if t < 1e-30:
                    raise RuntimeError("MEM oracle: line search failed")
            A, Qa = An, Qn
        raise RuntimeError("MEM oracle: Newton iteration did not converge")


def spectrum(tau, G, sigma, beta, w, m, alpha=None, alpha_range=(1e-8, 1e12)):
    """A(w) by maximum entropy.  alpha > 0: that alpha; None: the historic
    alpha with chi^2(A) = len(tau), bracketed by decades downwards from the
    top of alpha_range (chi^2 grows with alpha).  Returns (A, alpha, chi^2)."""
    P = Problem(tau, G, sigma, beta, w, m)
    if alpha is not None:
        A = P.solve(alpha)
        return A, alpha, P.chi2(A)
    n = len(P.G)

    def f(la):
        return P.chi2(P.solve(np.exp(la))) - n

    lmin, dec = np.log(alpha_range[0]), np.log(10.0)
    hi = np.log(alpha_range[1])
    if f(hi) < 0:
        raise RuntimeError("chi^2 < n already at the largest alpha")
    lo = hi - dec
    while f(lo) >= 0:
        hi, lo = lo, lo - dec
        if lo < lmin:
            raise RuntimeError("chi^2 = n is not reached inside the alpha range")
    la = brentq(f, lo, hi, xtol=1e-13, rtol=1e-14)
    A = P.solve(np.exp(la))
    return A, float(np.exp(la)), P.chi2(A)
