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
  H, including Re Sigma = 0 at k = (pi, 0) (particle-hole symmetry)."""
import numpy as np
import pytest

import paper_1504_05090_amd as bss
from oracle import analysis as an
from tests.fock import Cluster
from tests.fock_gk import continuous_giw_k, continuous_gk, trotterised_gk

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
