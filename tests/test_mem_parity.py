"""Parity of the library's maximum-entropy step (bss_mem_spectrum,
bss_mem_green) with the oracle's on the same seeded inputs.  Host code: runs
without a GPU.

The two share only the readings: the library solves the stationarity
condition in the singular space of the kernel (one-sided Jacobi SVD, Newton
on alpha u + Sigma V^T r = 0, backtracked on Q) and finds the historic alpha
by regula falsi with warm starts; the oracle runs Newton's method on Q in A itself and
scipy's Brent root finder with every alpha solved from the default model.
The minimiser of Q is unique, so both must land on it to the rounding floor
of the gradient (about 1e-9 relative in A for these data)."""
import numpy as np
import pytest

import paper_1504_05090_amd as bss
from oracle import mem
from tests.mem_data import ingredients

BETA = 20.0


def data(n_tau, n_w, noise, seed, beta=BETA):
    tau, w, A, eta, sig, m = ingredients(beta, n_tau, n_w, noise, seed)
    return tau, mem.green(tau, w, A, beta) + eta, sig, w, m


def compare(tau, G, sig, w, m, alpha, beta=BETA):
    Ao, ao, co = mem.spectrum(tau, G, sig, beta, w, m, alpha)
    Al, al, cl = bss.mem_spectrum(tau, G, sig, beta, w, m, alpha)
    assert abs(al - ao) <= 1e-10 * ao
    assert abs(cl - co) <= 1e-10 * max(1.0, co)
    big = Ao > 1e-6 * Ao.max()
    assert np.max(np.abs(Al - Ao)[big] / Ao[big]) < 1e-8
    assert np.max(np.abs(Al - Ao)) < 1e-10 * Ao.max()
    assert np.all(Al > 0)
    Gl = bss.mem_green(beta, w, Al, tau)
    assert np.max(np.abs(Gl - mem.green(tau, w, Ao, beta))) < 1e-12
    return Al, al


@pytest.mark.parametrize("seed,n_tau,n_w", [(0, 81, 121), (1, 81, 121), (11, 41, 201)])
def test_historic_alpha_parity(seed, n_tau, n_w):
    tau, G, sig, w, m = data(n_tau, n_w, 1e-4, seed)
    A, alpha = compare(tau, G, sig, w, m, None)
    assert 10.0 < alpha < 1e4


@pytest.mark.parametrize("alpha,n_tau,n_w,noise", [(10.0, 81, 121, 1e-4), (1e3, 81, 121, 1e-4),
                                                   (3.0, 21, 41, 1e-4), (0.05, 41, 61, 1e-2)])
def test_fixed_alpha_parity(alpha, n_tau, n_w, noise):
    tau, G, sig, w, m = data(n_tau, n_w, noise, 2)
    compare(tau, G, sig, w, m, alpha)


def cluster_draws():
    """G(tau, k) of the 2 x 2 Hubbard cluster (U = 2, t = 0.25, beta = 2) in
    continuous time from its Fock space, on 41 points, with N(0, 1e-4^2)
    noise, at k = (pi, 0), (0, 0), (pi, pi) (a spectrum of a few sharp
    lines, unlike the smooth synthetic ones above)."""
    from tests.fock import Cluster
    from tests.fock_gk import continuous_gk
    tau = np.linspace(0.0, 2.0, 41)
    G = continuous_gk(Cluster(2, 0.25, 2.0), 2.0, tau)
    sig = np.full(tau.size, 1e-4)
    rng = np.random.default_rng(5)
    return tau, sig, {k: G[:, k] + sig * rng.standard_normal(tau.size) for k in (1, 0, 3)}


@pytest.mark.parametrize("alpha", [1e4, 1e2, 1.0, 1e-2])
def test_fixed_alpha_parity_on_cluster_spectra(alpha):
    """Both solvers reach the same A at every alpha from 1e4 down to 1e-2,
    to a relative 1e-10 (1 + 100 / alpha) on the A_j above 1e-6 of the peak:
    the Jacobian's smallest eigenvalue is alpha, so the rounding floor of the
    gradient moves A by about 1/alpha (measured 3e-13 at 1e4, 3e-9 at 1,
    1.1e-7 at 1e-2).  Where the data ask for lines sharper than the double
    range allows (alpha = 1e-2 at k = (pi, 0) and (pi, pi)), both report it."""
    tau, sig, draws = cluster_draws()
    w = np.linspace(-4.0, 4.0, 161)
    m = np.full(w.size, 1.0 / 8.0)
    for k, G in draws.items():
        if alpha < 0.1 and k != 0:
            with pytest.raises(bss.BssError) as err:
                bss.mem_spectrum(tau, G, sig, 2.0, w, m, alpha)
            assert err.value.status == bss.BSS_E_NUMERICAL
            with pytest.raises(RuntimeError):
                mem.spectrum(tau, G, sig, 2.0, w, m, alpha)
            continue
        Al, _, cl = bss.mem_spectrum(tau, G, sig, 2.0, w, m, alpha)
        Ao, _, co = mem.spectrum(tau, G, sig, 2.0, w, m, alpha)
        big = Ao > 1e-6 * Ao.max()
        tol = 1e-10 * (1.0 + 100.0 / alpha)
        assert np.max(np.abs(Al - Ao)[big] / Ao[big]) < tol, k
        assert np.max(np.abs(Al - Ao)) < tol * Ao.max(), k
        assert cl == pytest.approx(co, rel=1e-9)


def test_nonuniform_grids_and_per_point_errors():
    """A denser w grid near 0, tau points clustered at the ends (where
    G(tau) varies fastest) and errors that differ per point."""
    x = np.linspace(-1, 1, 101)
    w = 4.0 * np.sign(x) * np.abs(x) ** 1.5
    u = np.linspace(0, 1, 51)
    tau = BETA * (1 - np.cos(np.pi * u)) / 2
    from tests.mem_data import two_band_spectrum
    rng = np.random.default_rng(21)
    sig = 1e-4 * (1 + rng.uniform(0, 1, len(tau)))
    G = mem.green(tau, w, two_band_spectrum(w), BETA) + sig * rng.standard_normal(len(tau))
    m = np.exp(-w ** 2 / 8)
    compare(tau, G, sig, w, m / np.sum(mem.trapezoid_weights(w) * m), None)


@pytest.mark.parametrize("beta", [1.0, 40.0, 400.0])
def test_mem_green_parity(beta):
    """eq. (4) on the grid for a random positive A, including beta |w| up to
    1600 (no overflow on either side)."""
    w = np.linspace(-4, 4, 97)
    A = np.random.default_rng(3).uniform(0, 1, len(w))
    tau = np.linspace(0, beta, 37)
    got = bss.mem_green(beta, w, A, tau)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - mem.green(tau, w, A, beta))) < 1e-14


def test_historic_alpha_that_does_not_exist_is_numerical():
    """The oracle's pinned case: chi^2 cannot reach n_tau with A >= 0."""
    tau, G, sig, w, m = data(81, 121, 1e-4, 3)
    with pytest.raises(bss.BssError) as e:
        bss.mem_spectrum(tau, G, sig, BETA, w, m)
    assert e.value.status == bss.BSS_E_NUMERICAL


def test_mem_argument_errors():
    tau, G, sig, w, m = data(21, 41, 1e-3, 4)
    bad = [
        dict(sigma=np.where(np.arange(len(sig)) == 3, 0.0, sig)),
        dict(omega=w[::-1].copy()),
        dict(model=np.where(np.arange(len(m)) == 5, -1.0, m)),
        dict(tau=np.append(tau[:-1], BETA + 0.1)),
        dict(G=np.where(np.arange(len(G)) == 2, np.nan, G)),
        dict(alpha=np.inf),
    ]
    for b in bad:
        args = dict(tau=tau, G=G, sigma=sig, omega=w, model=m, alpha=1.0)
        args.update(b)
        with pytest.raises(bss.BssError) as e:
            bss.mem_spectrum(args["tau"], args["G"], args["sigma"], BETA, args["omega"], args["model"], args["alpha"])
        assert e.value.status == bss.BSS_E_INVALID_ARG, b.keys()
    with pytest.raises(bss.BssError):
        bss.mem_green(BETA, w[::-1].copy(), m, tau)
