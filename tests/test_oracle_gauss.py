"""Pins for the oracle with Gaussian couplings (Sec. 2.1: couplings from a
standard normal; Sec. 4.2's model), couplings on the 2^-16 grid.

The acceptance rule is checked against an independent 60-digit decimal
evaluation of r < 2^32 exp(-b u 2^-16) at the boundary values of r; energies
against numpy brute force; a gauge transformation must leave the trajectory
unchanged; the exchange acceptance rate and whole PT + Houdayer chains must
reproduce exact enumeration (3x3 and 4x4 with Gaussian couplings)."""
import decimal
import math

import numpy as np
import pytest

import exact
from paper_2003_04621_amd import workloads as W

UNIT = 2.0 ** -16


def _threshold(b, u):
    """The number of 32-bit r with r < 2^32 exp(-b u 2^-16), from decimal."""
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        y = decimal.Decimal(b) * decimal.Decimal(int(u)) / decimal.Decimal(65536)
        t = (-y).exp() * decimal.Decimal(2 ** 32)
        # r < t for r = 0 .. ceil(t) - 1 (t is never an integer here)
        return int(t.to_integral_value(rounding=decimal.ROUND_CEILING))


def test_gauss_accept_rule_against_decimal(orc):
    rng = np.random.default_rng(9)
    cases = [(0.5, 1), (1.7, 65536), (5.0, 300000), (0.01, 12345678), (2.3, 40 * 65536),
             (1e-6, 3), (3.0, 1 << 33)]
    for _ in range(300):
        cases.append((float(rng.uniform(0.01, 5.0)), int(rng.integers(1, 3_000_000))))
    for b, u in cases:
        n = _threshold(b, u)
        for r in {0, max(n - 1, 0), n, min(n + 1, 2 ** 32 - 1), 2 ** 32 - 1}:
            if r >= 2 ** 32:
                continue
            assert orc.gauss_accept(r, b, u) == int(r < n), (b, u, r, n)


def _brute(L, d, Jn, s):
    return exact.brute_energy(L, d, Jn, s)


@pytest.mark.parametrize("L,d", [(3, 2), (4, 2), (6, 2), (3, 3), (4, 3)])
def test_gauss_energy_and_local_field(orc, L, d):
    rng = np.random.default_rng(L + 10 * d)
    N = L ** d
    Jn = W.gauss_units(W.couplings_gauss(1, L, d, 5 + L)[0])
    for _ in range(10):
        s = rng.choice(np.array([-1, 1], np.int8), size=N)
        E = orc.gauss_energy(L, d, Jn, s)
        assert E == _brute(L, d, Jn, s)
        for i in rng.integers(0, N, size=5):
            t = s.copy()
            t[i] = -t[i]
            assert _brute(L, d, Jn, t) - E == 2 * orc.gauss_local_x(L, d, Jn, s, int(i))


def test_gauss_incremental_energies_equal_recompute(orc):
    for L, d, hou in [(6, 2, 1), (4, 3, 2), (8, 2, 2), (5, 3, 0)]:
        S, NT = 2, 4
        Jf = W.couplings_gauss(S, L, d, 40 + L)
        Jn = W.gauss_units(Jf)
        job = orc.OracleGaussJob(S, NT, L, d, Jn, W.geometric_betas(0.4, 2.0, NT), 7)
        for _ in range(6):
            job.mcs(1, houdayer=hou > 0, multi=hou == 2)
            sp, E = job.spins(), job.energies()
            for s in range(S):
                for r in range(2 * NT):
                    assert E[s, r] == _brute(L, d, Jn[s], sp[s, r])
            sot, tos = job.maps()
            for s in range(S):
                for c in range(2):
                    assert (tos[s, c][sot[s, c]] == np.arange(NT)).all()


def test_gauss_gauge_invariance(orc):
    """J'_ij = e_i e_j J_ij with s' = e s gives s'_t = e s_t, the same
    energies and the same exchange decisions (x = s_i h_i is gauge
    invariant, and so are q and the clusters)."""
    L, d, S, NT = 6, 2, 2, 4
    N = L * L
    rng = np.random.default_rng(3)
    Jn = W.gauss_units(W.couplings_gauss(S, L, d, 77))
    eps = rng.choice(np.array([-1, 1], np.int8), size=(S, N))
    Jg = Jn.copy()
    for s in range(S):
        for mu in range(d):
            nb = np.array([((i % L) + (1 if mu == 0 else 0)) % L + L * (((i // L) + (1 if mu == 1 else 0)) % L)
                           for i in range(N)])
            Jg[s, mu] = Jn[s, mu] * eps[s] * eps[s][nb]
    b = W.geometric_betas(0.5, 2.0, NT)
    a = orc.OracleGaussJob(S, NT, L, d, Jn, b, 11)
    g = orc.OracleGaussJob(S, NT, L, d, Jg, b, 11)
    g.set_spins(a.spins() * eps[:, None, :])
    for step in range(8):
        a.mcs(1, houdayer=True, measure=True, multi=step % 2 == 1)
        g.mcs(1, houdayer=True, measure=True, multi=step % 2 == 1)
        assert (g.spins() == a.spins() * eps[:, None, :]).all()
        assert (g.energies() == a.energies()).all()
        for x, y in zip(a.maps(), g.maps()):
            assert (x == y).all()


def _all_state_energies(L, d, Jn):
    N = L ** d
    states = ((np.arange(2 ** N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int8)
    s = 1 - 2 * states
    shp = (2 ** N,) + (L,) * d
    sg = s.reshape(shp).astype(np.int64)
    E = np.zeros(2 ** N, np.int64)
    for mu in range(d):
        axis = d - mu
        Jm = Jn[mu].reshape((L,) * d).astype(np.int64)
        E -= np.sum((Jm[None] * sg * np.roll(sg, -1, axis=axis)).reshape(2 ** N, -1), axis=1)
    return E


def test_gauss_state_energies_match_brute(orc):
    L, d = 3, 2
    Jn = W.gauss_units(W.couplings_gauss(1, L, d, 3)[0])
    E = _all_state_energies(L, d, Jn)
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2 ** 9, size=20):
        s = (1 - 2 * ((int(x) >> np.arange(9)) & 1)).astype(np.int8)
        assert E[x] == orc.gauss_energy(L, d, Jn, s)


def test_gauss_pt_acceptance_rate_matches_exact(orc):
    """Swap rate of the coldest pair on a 3x3 Gaussian sample after
    equilibration: sum over energy pairs of pi_0 pi_1 P(swap), P from the
    decimal thresholds."""
    L, d, S = 3, 2, 3000
    Jn = W.gauss_units(W.couplings_gauss(1, L, d, 21))
    Es = _all_state_energies(L, d, Jn[0])
    betas = np.array([1.0, 0.6])
    p0 = np.exp(-betas[0] * Es * UNIT - np.max(-betas[0] * Es * UNIT))
    p0 /= p0.sum()
    p1 = np.exp(-betas[1] * Es * UNIT - np.max(-betas[1] * Es * UNIT))
    p1 /= p1.sum()
    uE, inv = np.unique(Es, return_inverse=True)
    w0 = np.bincount(inv, weights=p0)
    w1 = np.bincount(inv, weights=p1)
    db = float(betas[0] - betas[1])
    expect = 0.0
    for i, Ex in enumerate(uE):
        for j, Ey in enumerate(uE):
            D = int(Ey - Ex)
            pa = 1.0 if D <= 0 else _threshold(db, D) / 2 ** 32
            expect += w0[i] * w1[j] * pa
    job = orc.OracleGaussJob(S, 2, L, d, np.repeat(Jn, S, axis=0), betas, 55)
    job.mcs(40)
    before = job.maps()[0].copy()
    job.sweep(1)
    job.exchange()
    acc = (job.maps()[0][:, :, 0] != before[:, :, 0]).mean()
    sigma = math.sqrt(expect * (1 - expect) / (2 * S))
    assert abs(acc - expect) < 5 * sigma, (acc, expect, sigma)


@pytest.mark.parametrize("multi", [False, True])
def test_gauss_4x4_pt_houdayer_matches_exact_moments(orc, multi):
    L, d, S = 4, 2, 64
    N = L * L
    Jn = W.gauss_units(W.couplings_gauss(1, L, d, 12))
    Es = _all_state_energies(L, d, Jn[0])
    Ef = Es.astype(np.float64) * UNIT
    betas = np.array([1.5, 1.0, 0.6, 0.3])
    job = orc.OracleGaussJob(S, len(betas), L, d, np.repeat(Jn, S, axis=0), betas, 3)
    job.mcs(400, houdayer=True, multi=multi)
    job.mcs(2000, houdayer=True, multi=multi, measure=True)
    ps, dis, n = job.observables()
    mom = job.moments()
    for k, beta in enumerate(betas):
        logw = -beta * Ef
        w = np.exp(logw - logw.max())
        w /= w.sum()
        e_ex = float(np.sum(w * Ef)) / N
        # <E^2> from the 128-bit sums of squared energies (units^2)
        e2_ex = float(np.sum(w * Ef ** 2))
        e2 = (mom["E2"][:, k, 0].astype(float) + mom["E2"][:, k, 1].astype(float) * 2.0 ** 64) \
            * UNIT ** 2 / (2.0 * n)
        se2 = e2.std(ddof=1) / math.sqrt(S)
        assert abs(e2.mean() - e2_ex) < 5 * se2, (beta, e2.mean(), e2_ex, se2)
        q2_ex, q4_ex, _ = exact.overlap_moments(Ef, N, beta)
        aq_ex = exact.abs_overlap(Ef, N, beta)
        for col, ex in [(0, e_ex), (1, 0.0), (2, aq_ex), (3, q2_ex), (4, q4_ex)]:
            v = ps[:, k, col]
            se = v.std(ddof=1) / math.sqrt(S)
            assert abs(v.mean() - ex) < 5 * se + 1e-12, (beta, col, v.mean(), ex, se)
