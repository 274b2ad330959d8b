"""Pins of the oracle's sweep mechanics against from-scratch linear algebra:
determinant ratios, rank-1 updates, wraps, stabilised recomputation (checked
against high-precision arithmetic) and detailed balance."""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

T = 0.25


def independent_b(L, U, dtau, field, l, spin):
    """B_l built without the oracle: K from the lattice, scipy expm, Hirsch lambda."""
    N = L * L
    K = np.zeros((N, N))
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                K[i, (x + dx) % L + L * ((y + dy) % L)] += -T
    lam = math.acosh(math.exp(dtau * U / 2))
    sg = 1.0 if spin == 0 else -1.0
    return sla.expm(-dtau * K) @ np.diag(np.exp(sg * lam * field[l - 1]))


def m_matrix(L, U, dtau, field, l, spin):
    """I + B_{l-1}..B_1 B_Lam..B_l (whose inverse is G at the start of slice l)."""
    lam = field.shape[0]
    N = L * L
    P = np.eye(N)
    order = list(range(l, lam + 1)) + list(range(1, l))
    for q in order:
        P = independent_b(L, U, dtau, field, q, spin) @ P
    return np.eye(N) + P


def test_ratio_and_update_against_scratch(orc):
    L, U, beta, dtau = 4, 2.0, 2.0, 0.5
    c = orc.Chain(L, U, T, beta, dtau, 77, 0, 0, 2)
    c.step_slices(1, forced=np.zeros(16, np.uint8))   # move to slice 2 without flips
    l = c.slice
    assert l == 2
    for i in (0, 5, 11):
        f = c.field()
        fl = f.copy()
        fl[l - 1, i] *= -1
        for spin in range(2):
            M0 = m_matrix(L, U, dtau, f, l, spin)
            M1 = m_matrix(L, U, dtau, fl, l, spin)
            want = np.linalg.det(M1) / np.linalg.det(M0)
            got = c.ratio(l, i)[spin]
            assert abs(got - want) < 1e-12 * max(1, abs(want))
            assert np.max(np.abs(c.green(spin) - np.linalg.inv(M0))) < 1e-12
        c.accept_update(l, i)
        assert np.array_equal(c.field(), fl)
        for spin in range(2):
            assert np.max(np.abs(c.green(spin) - np.linalg.inv(m_matrix(L, U, dtau, fl, l, spin)))) < 1e-11


def test_wrap_identity(orc):
    """G(l+1) = B_l G(l) B_l^{-1}."""
    L, U, beta, dtau = 4, 2.0, 3.0, 0.5
    c = orc.Chain(L, U, T, beta, dtau, 8, 0, 0, 6)
    f = c.field()
    for l in (1, 2, 3):
        c.wrap(l)
        for spin in range(2):
            want = np.linalg.inv(m_matrix(L, U, dtau, f, l + 1, spin))
            assert np.max(np.abs(c.green(spin) - want)) < 1e-12
            assert np.max(np.abs(c.green(spin) - c.fresh_green(l + 1, spin))) < 1e-12


def mp_inverse_chain(Bs, N, prec=80):
    """(I + B_Lam ... B_1)^{-1} and the B_l..B_1 (I+...)^{-1} products in
    `prec`-digit arithmetic from the float64 B matrices."""
    with mpmath.workdps(prec):
        Ms = [mpmath.matrix(B.tolist()) for B in Bs]
        P = mpmath.eye(N)
        partial = [P]
        for M in Ms:
            P = M * P
            partial.append(P)
        G0 = (mpmath.eye(N) + P) ** -1
        return [np.array((Pl * G0).tolist(), dtype=float) for Pl in partial]


@pytest.mark.parametrize("L,U,beta,dtau,n_stab", [(2, 2.0, 20.0, 0.5, 8), (2, 4.0, 40.0, 0.5, 4),
                                                   (4, 2.0, 10.0, 0.5, 5)])
def test_stabilised_green_against_high_precision(orc, L, U, beta, dtau, n_stab):
    """The UDV-stabilised G(0) and G(tau_l, 0) agree with the unstabilised
    formulas evaluated in 80-digit arithmetic (same float64 B matrices).
    The block length must keep each plain block product well conditioned in
    FP64 (at U = 4, beta = 40 the error grows from 1e-13 at n_stab = 4 to 1e-5
    at n_stab = 20), so n_stab is chosen accordingly."""
    c = orc.Chain(L, U, T, beta, dtau, 4, 0, 0, n_stab)
    N, lam = c.N, c.Lam
    for spin in range(2):
        Bs = [c.bmat(l, spin) for l in range(1, lam + 1)]
        ref = mp_inverse_chain(Bs, N)
        G0 = c.fresh_green(1, spin)
        tol = 1e-12 * max(1.0, np.max(np.abs(ref[0])))
        assert np.max(np.abs(G0 - ref[0])) < tol
        for l in sorted({0, 1, n_stab, lam // 2, lam - 1, lam}):
            tol_l = 1e-12 * max(1.0, np.max(np.abs(ref[l])))
            assert np.max(np.abs(c.gtau0(l, spin) - ref[l])) < tol_l, l


def test_recompute_replaces_wrapped_green(orc):
    """Every n_stab slices and at the end of the sweep G is recomputed from
    scratch; the wrapped and fresh matrices differ only by rounding."""
    c = orc.Chain(4, 2.0, T, 10.0, 0.5, 12, 0, 0, 5)
    c.sweep(2)
    st = c.stats()
    assert st["drift_count"] == 2 * 4
    assert 0 < st["drift_max"] < 1e-9
    assert c.slice == 1 and c.sweep_index == 2
    for spin in range(2):
        assert np.array_equal(c.green(spin), c.fresh_green(1, spin))


def test_forced_history_replays_decisions(orc):
    a = orc.Chain(4, 2.0, T, 4.0, 0.5, 99, 0, 0, 4)
    b = orc.Chain(4, 2.0, T, 4.0, 0.5, 99, 0, 0, 4)
    tr = a.sweep(3, record=True)
    b.sweep(3, forced=tr)
    assert np.array_equal(a.field(), b.field())
    assert np.array_equal(a.green(0), b.green(0))
    # flip every decision of the first sweep: the field history changes
    c = orc.Chain(4, 2.0, T, 4.0, 0.5, 99, 0, 0, 4)
    c.sweep(1, forced=1 - tr[: 8 * 16])
    assert not np.array_equal(c.field(), a.field())


def test_detailed_balance_chi2(orc):
    """2 x 2, Lam = 2: the histogram of fields visited at sweep ends follows
    W(h) / Z (all 2^8 fields, chi-square test on thinned samples)."""
    from scipy.stats import chi2

    L, U, beta, dtau = 2, 2.0, 1.0, 0.5
    c = orc.Chain(L, U, T, beta, dtau, 2024, 0, 0, 2)
    N, lam = c.N, c.Lam
    import itertools
    fields = [np.array(b, dtype=np.int8).reshape(lam, N) for b in itertools.product((1, -1), repeat=lam * N)]
    index = {f.tobytes(): n for n, f in enumerate(fields)}
    w = np.array([math.exp(c.log_det_M(0, f)[0] + c.log_det_M(1, f)[0]) for f in fields])
    p = w / w.sum()
    counts = np.zeros(len(fields))
    c.sweep(20)
    n_samp = 30000
    for _ in range(n_samp):
        c.sweep(4)
        counts[index[c.field().tobytes()]] += 1
    expected = n_samp * p
    stat = np.sum((counts - expected) ** 2 / expected)
    pval = chi2.sf(stat, len(fields) - 1)
    assert pval > 1e-3, (stat, pval)
    assert p.max() / p.min() > 2     # the target is far from uniform


def _numpy_uniform(key0, key1, s, pos):
    """u of the Metropolis test from numpy's own Philox4x64-10: word 0 of the
    block at counter (s, pos, 0, 0) under key (key0, key1), top 53 bits
    scaled by 2^-53.  numpy bumps the counter before producing a block, so
    its state starts one below."""
    words = [s, pos, 0, 0]
    for k in range(4):            # subtract one from the 256-bit counter
        if words[k] > 0:
            words[k] -= 1
            break
        words[k] = 2**64 - 1
    ctr = np.array(words, dtype=np.uint64)
    bg = np.random.Philox(key=np.array([key0, key1], dtype=np.uint64), counter=ctr)
    w0 = int(bg.random_raw(1)[0])
    return (w0 >> 11) * 2.0 ** -53


def test_metropolis_draw_against_numpy_philox(orc):
    """The accept decisions of a free-running chain are those of the
    Metropolis test u < R with u from numpy's Philox at counter
    (sweep, (l-1) N + i, 0, 0) and key (seed + chain, instance): the chain is
    replayed proposal by proposal with the oracle's own ratio, update, wrap
    and recomputation pieces and numpy's draws, over two sweeps (so the sweep
    index enters), on a chain whose acceptance is far from 0 and 1."""
    L, U, beta, dtau, n_stab, seed, inst, chain = 4, 2.0, 1.0, 0.5, 2, 4711, 3, 5
    a = orc.Chain(L, U, T, beta, dtau, seed, inst, chain, n_stab)
    want = a.sweep(2, record=True)
    b = orc.Chain(L, U, T, beta, dtau, seed, inst, chain, n_stab)
    N, lam = b.N, b.Lam
    got = []
    for s in range(2):
        for l in range(1, lam + 1):
            for i in range(N):
                ru, rd = b.ratio(l, i)
                u = _numpy_uniform(seed + chain, inst, s, (l - 1) * N + i)
                acc = u < ru * rd
                got.append(acc)
                if acc:
                    b.accept_update(l, i)
            b.wrap(l)
            if l % n_stab == 0 or l == lam:
                nxt = 1 if l == lam else l + 1
                fresh = [b.fresh_green(nxt, sp) for sp in range(2)]
                for sp in range(2):
                    b.set_green(sp, fresh[sp])
    got = np.array(got, dtype=np.uint8)
    assert 0.2 < got.mean() < 0.8
    assert np.array_equal(got, want)
    assert np.array_equal(a.field(), b.field())


def _broken_green_chain(orc, value):
    c = orc.Chain(4, 2.0, T, 2.0, 0.5, 31, 0, 0, 2)
    for sp in range(2):
        c.set_green(sp, np.eye(c.N) * value)
    return c


@pytest.mark.parametrize("value", [float("nan"), 5.0], ids=["nan", "negative_ratio"])
def test_bad_ratio_is_an_error_even_when_rejected(orc, value):
    """A Green function whose diagonal is NaN, or so large that R <= 0, is a
    numerical failure (every weight of eq. (3) is positive at half filling):
    the free-running chain stops with its error flag set at the first such
    proposal, although the Metropolis test would simply reject it."""
    c = _broken_green_chain(orc, value)
    with pytest.raises(FloatingPointError):
        c.step_slices(1)
    st = c.stats()
    assert st["error"] == 1 and st["proposals"] == 1 and st["accepted"] == 0
    if value == 5.0:
        ru, rd = c.ratio(1, 0)
        assert ru * rd < 0


def test_forced_negative_ratio_flips_the_sign_and_stops(orc):
    """A forced acceptance of a negative ratio multiplies the running sign by
    -1, and the chain stops there with the error flag set."""
    c = _broken_green_chain(orc, 5.0)
    with pytest.raises(FloatingPointError):
        c.step_slices(1, forced=np.ones(c.N, np.uint8))
    st = c.stats()
    assert st["error"] == 1 and st["accepted"] == 1 and st["sign"] == -1
    h = orc.Chain(4, 2.0, T, 2.0, 0.5, 31, 0, 0, 2)
    assert np.array_equal(c.field(), h.field())   # the bad flip was not applied
