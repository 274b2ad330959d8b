"""The host analysis pinned to physics on the 2 x 2 cluster at U = 2, with
references from the 256-state Fock space (tests/fock.py; no oracle code):

- the Trotter elimination (paper Sec. 3, Trotter bias): G(tau, k) of the
  Trotterised model, exact for each slice width, extrapolated pointwise to
  dtau -> 0 by the library (bss_trotter_extrapolate) and by the oracle,
  recovers the exact continuous-time G(tau, k) of H = H_t + H_U, while the
  single grids miss it by up to 4.5e-2;
- the Matsubara transform (eq. (5), read with e^{+i w_n tau}) and the Dyson
  equation (eq. (6)): the exact continuous-time G(tau, k) on a fine tau grid,
  transformed and inverted by the library and by the oracle, gives the
  G_k(i w_n) and Sigma_k(i w_n) of the Lehmann sums over the eigenstates of
  H, including Re Sigma = 0 at k = (pi, 0) (particle-hole symmetry);
- the maximum-entropy spectrum (Sec. 3, Trotter-bias paragraph, eq. (4)) of
  the exact G(tau, k) with noise added, at the historic alpha, by the library
  and by the oracle: its frequency moments keep the sum rules of A_k
  (weight 1, first moment eps_k, second eps_k^2 + U^2/4 at half filling),
  computed from the Fock space as anticommutator expectation values."""
import numpy as np
import pytest

import paper_1504_05090_amd as bss
from oracle import analysis as an
from oracle import mem as om
from tests.fock import Cluster
from tests.fock_gk import continuous_giw_k, continuous_gk, spectral_moments_k, trotterised_gk

BETA, U, T = 2.0, 2.0, 0.25


@pytest.mark.parametrize("dts,bound", [([0.5, 0.4, 0.25, 0.2], 1e-3), ([0.25, 0.2, 0.125, 0.1], 1e-4)])
def test_trotter_elimination_recovers_the_continuous_time_g(dts, bound):
    cl = Cluster(2, T, U)
    tau_f = np.linspace(0.0, BETA, 21)
    exact = continuous_gk(cl, BETA, tau_f)
    Gs = [trotterised_gk(cl, BETA, dt) for dt in dts]
    coarse = np.interp(tau_f, np.linspace(0.0, BETA, len(Gs[0])), Gs[0][:, 0])
    assert np.max(np.abs(coarse - exact[:, 0])) > 10 * bound     # the bias to be removed
    lib = bss.trotter_extrapolate(dts, Gs, BETA, tau_f)
    orc = an.trotter_extrapolate(list(dts), Gs, BETA, tau_f)
    print(f"dtau grids {dts}: max|lib - exact| {np.max(np.abs(lib - exact)):.2e}, "
          f"max|oracle - exact| {np.max(np.abs(orc - exact)):.2e}")
    assert np.max(np.abs(lib - exact)) < bound
    assert np.max(np.abs(orc - exact)) < bound


def test_matsubara_and_dyson_of_the_exact_g_give_the_lehmann_self_energy():
    import math
    cl = Cluster(2, T, U)
    tau = np.linspace(0.0, BETA, 401)
    G = continuous_gk(cl, BETA, tau)
    nf = 8
    exact = continuous_giw_k(cl, BETA, nf)
    w = an.matsubara_frequencies(BETA, nf)
    for k in range(4):
        kx, ky = math.pi * (k % 2), math.pi * (k // 2)
        eps = -2 * T * (math.cos(kx) + math.cos(ky))
        sig_exact = an.dyson(w, eps, 0.0, exact[:, k])
        g_lib = bss.matsubara(tau, G[:, k], BETA, nf)
        g_orc = an.matsubara(tau, G[:, k], BETA, nf)
        assert np.max(np.abs(g_lib - exact[:, k])) < 1e-9 and np.max(np.abs(g_orc - exact[:, k])) < 1e-9
        s_lib = bss.dyson(BETA, eps, 0.0, g_lib)
        s_orc = an.dyson(w, eps, 0.0, g_orc)
        assert np.max(np.abs(s_lib - sig_exact)) < 1e-8 and np.max(np.abs(s_orc - sig_exact)) < 1e-8
        assert np.max(np.abs(sig_exact.imag)) > 0.4          # an interacting self-energy
        if eps == 0.0:
            assert np.max(np.abs(sig_exact.real)) < 1e-12 and np.max(np.abs(s_lib.real)) < 1e-9


def test_mem_spectrum_of_the_exact_g_keeps_the_sum_rules():
    """A_k from G(tau, k) + N(0, 1e-4^2) on 41 points (flat default model on
    [-4, 4], 161 points): both implementations find the same historic alpha
    and spectrum, and its weight, first and second moments match the exact
    ones within 2e-3, 2e-2 and 6e-2 (the weight is fixed by G(0) + G(beta)
    through eq. (4), the higher moments less tightly by the data; measured
    errors 4e-4, 6e-3, 3e-2).  The noise draw for k = (0, 0) is the one on
    which the library's search stalled while its Newton steps were
    backtracked on |F|^2 instead of Q."""
    cl = Cluster(2, T, U)
    mom = spectral_moments_k(cl, BETA, 2)
    for k in range(4):
        eps = -2 * T * (np.cos(np.pi * (k % 2)) + np.cos(np.pi * (k // 2)))
        np.testing.assert_allclose(mom[:, k], [1.0, eps, eps ** 2 + U ** 2 / 4], atol=1e-12)
    tau = np.linspace(0.0, BETA, 41)
    G = continuous_gk(cl, BETA, tau)
    omega = np.linspace(-4.0, 4.0, 161)
    model = np.full(omega.size, 1.0 / 8.0)
    sig = np.full(tau.size, 1e-4)
    q = np.full(omega.size, omega[1] - omega[0])
    q[0] = q[-1] = q[0] / 2
    rng = np.random.default_rng(5)
    for k in (1, 0, 3):
        Gn = G[:, k] + sig * rng.standard_normal(tau.size)
        A, alpha, chi2 = bss.mem_spectrum(tau, Gn, sig, BETA, omega, model)
        A_o, alpha_o, chi2_o = om.spectrum(tau, Gn, sig, BETA, omega, model)
        assert chi2 == pytest.approx(tau.size, rel=1e-9) and chi2_o == pytest.approx(tau.size, rel=1e-9)
        assert alpha == pytest.approx(alpha_o, rel=1e-8)
        np.testing.assert_allclose(A, A_o, rtol=0, atol=1e-9 * np.max(A_o))
        for spec in (A, A_o):
            m = np.array([np.sum(q * spec * omega ** p) for p in range(3)])
            assert np.all(np.abs(m - mom[:, k]) <= [2e-3, 2e-2, 6e-2]), (k, m, mom[:, k])
