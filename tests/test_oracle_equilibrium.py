"""Equilibrium pins for the oracle: exact enumeration and closed forms.

  * 3x3 2D: the one-sweep transition matrix built from the oracle's own
    single-site rule (probed) and visiting order leaves the Boltzmann
    distribution stationary (Sec. 2.2); the oracle's seeded chain reproduces
    the exact finite-time energy distribution (chi-square).
  * 3x3x3 3D: exact <E> from the density of states.
  * 16x16 ferromagnet (J = +1, p = 1 in Eq. (2)): Kaufman's exact <E>.
  * 4x4 2D +-J with PT and Houdayer moves: exact <E>, <q^2>, <q^4>, <|q|> and
    the Binder parameter.
Errors of the simulated averages come from the spread over independent
samples that share one coupling set.
"""
import math

import numpy as np
import pytest

import exact
from paper_2003_04621_amd import workloads as W


def _states_spins(N):
    z = np.arange(1 << N, dtype=np.int64)
    return np.where((z[:, None] >> np.arange(N)) & 1, -1, 1).astype(np.int8)


def _flip_prob(orc, thr_row, x):
    """P(flip | x) of the oracle's rule, found by bisection over r."""
    if orc.metro_rule(x, 0xFFFFFFFF, thr_row):
        return 1.0
    lo, hi = 0, 0xFFFFFFFF          # rule(lo)=? , rule(hi)=0
    if not orc.metro_rule(x, 0, thr_row):
        return 0.0
    while hi - lo > 1:               # invariant: rule(lo)=1, rule(hi)=0
        mid = (lo + hi) // 2
        if orc.metro_rule(x, mid, thr_row):
            lo = mid
        else:
            hi = mid
    return hi / 2 ** 32


def _sweep_matrix(orc, L, d, J, beta, prob=None):
    N = L ** d
    S = _states_spins(N)
    E = np.array([exact.brute_energy(L, d, J, s) for s in S], np.int64)
    thr = orc.metro_thresholds([beta], d)[0]
    P = np.eye(1 << N)
    z = np.arange(1 << N)
    cache = {}
    for i in orc.sweep_order(L, d):
        zf = z ^ (1 << int(i))
        x = (E[zf] - E) // 2
        p = np.empty(len(z))
        for xv in np.unique(x):
            if prob is None:
                if xv not in cache:
                    cache[xv] = _flip_prob(orc, thr, int(xv))
                p[x == xv] = cache[xv]
            else:
                p[x == xv] = prob(int(xv))
        K = np.zeros((len(z), len(z)))
        K[z, z] = 1 - p
        K[z, zf] += p
        P = P @ K
    return P, E


def test_3x3_sweep_matrix_keeps_boltzmann_stationary(orc):
    L, d = 3, 2
    J = W.couplings_pm_j(1, L, d, 4)[0]
    for beta in (0.3, 0.8, 1.6):
        P, E = _sweep_matrix(orc, L, d, J, beta)
        pi = np.exp(-beta * (E - E.min()))
        pi /= pi.sum()
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        err = np.abs(pi @ P - pi).sum()
        assert err < 1e-8, err
    # negative control: a rule with the wrong energy scale is not stationary
    Pbad, E = _sweep_matrix(orc, L, d, J, 0.8, prob=lambda x: 1.0 if x <= 0 else math.exp(-0.8 * x))
    pi = np.exp(-0.8 * (E - E.min()))
    pi /= pi.sum()
    assert np.abs(pi @ Pbad - pi).sum() > 1e-3


def test_3x3_chain_matches_exact_finite_time_distribution(orc):
    L, d, S, sweeps = 3, 2, 1500, 12
    J1 = W.couplings_pm_j(1, L, d, 4)
    J = np.repeat(J1, S, axis=0)
    betas = np.array([1.2, 0.5])
    job = orc.OracleJob(S, 2, L, d, J, betas, 2024)
    job.sweep(sweeps)
    Efin = job.energies()                    # [S][4]; slot j of each set at T_j
    from exact import chi2_sf
    N = L * L
    for k, beta in enumerate(betas):
        P, E = _sweep_matrix(orc, L, d, J1[0], beta)
        p0 = np.full(1 << N, 1.0 / (1 << N))   # initial spins are uniform
        pt = p0 @ np.linalg.matrix_power(P, sweeps)
        levels = np.unique(E)
        expect = np.array([pt[E == e].sum() for e in levels])
        draws = np.concatenate([Efin[:, k], Efin[:, 2 + k]])
        obs = np.array([(draws == e).sum() for e in levels], float)
        exp_counts = expect * len(draws)
        # merge sparse bins into their neighbour
        o, e_ = [], []
        acc_o = acc_e = 0.0
        for oo, ee in zip(obs, exp_counts):
            acc_o += oo
            acc_e += ee
            if acc_e >= 5:
                o.append(acc_o)
                e_.append(acc_e)
                acc_o = acc_e = 0.0
        if acc_e > 0:
            o[-1] += acc_o
            e_[-1] += acc_e
        o, e_ = np.array(o), np.array(e_)
        chi2 = float(np.sum((o - e_) ** 2 / e_))
        assert chi2_sf(chi2, len(o) - 1) > 1e-4, (beta, chi2, len(o))


def _sample_means(per_sample, col):
    v = per_sample[:, :, col]
    return v.mean(axis=0), v.std(axis=0, ddof=1) / math.sqrt(v.shape[0])


def test_3x3x3_mean_energy_exact(orc):
    L, d, S = 3, 3, 48
    J1 = W.couplings_pm_j(1, L, d, 31)
    counts = orc.density_of_states(L, d, J1[0])
    assert int(counts.sum()) == 1 << 27
    betas = np.array([1.0, 0.75, 0.5, 0.3])
    job = orc.OracleJob(S, 4, L, d, np.repeat(J1, S, axis=0), betas, 9)
    job.mcs(200)
    job.mcs(500, measure=True)
    ps, _, n = job.observables()
    assert n == 500
    N = L ** d
    mean, se = _sample_means(ps, 0)
    for k, beta in enumerate(betas):
        ex = exact.mean_energy_from_dos(counts, d, N, beta)[0] / N
        assert abs(mean[k] - ex) < 5 * se[k] + 1e-12, (beta, mean[k], ex, se[k])


def test_kaufman_formula_matches_enumeration():
    import oracle
    L = 4
    counts = oracle.density_of_states(L, 2, np.ones((2, L * L), np.int8))
    for beta in (0.15, 0.3, 0.4407, 0.5, 0.9):
        e_enum = exact.mean_energy_from_dos(counts, 2, L * L, beta)[0]
        assert abs(exact.kaufman_mean_energy(L, beta) - e_enum) < 1e-6 * abs(e_enum)


def test_ferromagnet_16x16_matches_kaufman(orc):
    L, d, S = 16, 2, 8
    J = W.ferromagnet(S, L, d)
    betas = np.array([0.8, 0.65, 0.55, 0.35, 0.28, 0.22])
    job = orc.OracleJob(S, len(betas), L, d, J, betas, 77)
    job.mcs(300)
    job.mcs(900, measure=True)
    ps, _, _ = job.observables()
    mean, se = _sample_means(ps, 0)
    N = L * L
    for k, beta in enumerate(betas):
        ex = exact.kaufman_mean_energy(L, beta) / N
        assert abs(mean[k] - ex) < 5 * se[k] + 2e-4, (beta, mean[k], ex, se[k])


def test_4x4_pt_houdayer_matches_exact_moments(orc):
    L, d, S = 4, 2, 64
    N = L * L
    J1 = W.couplings_pm_j(1, L, d, 12)
    Es = orc.state_energies(L, d, J1[0])
    betas = np.array([1.5, 1.0, 0.6, 0.3])
    job = orc.OracleJob(S, len(betas), L, d, np.repeat(J1, S, axis=0), betas, 3)
    job.mcs(400, houdayer=True)
    job.mcs(2000, houdayer=True, measure=True)
    ps, dis, n = job.observables()
    mom = job.moments()
    for k, beta in enumerate(betas):
        logw = -beta * Es.astype(float)
        w = np.exp(logw - logw.max())
        w /= w.sum()
        e_ex = float(np.sum(w * Es)) / N
        q2_ex, q4_ex, norm = exact.overlap_moments(Es, N, beta)
        assert abs(norm - 1) < 1e-12
        aq_ex = exact.abs_overlap(Es, N, beta)
        checks = [(0, e_ex), (1, 0.0), (2, aq_ex), (3, q2_ex), (4, q4_ex)]
        for col, ex in checks:
            v = ps[:, k, col]
            se = v.std(ddof=1) / math.sqrt(S)
            assert abs(v.mean() - ex) < 5 * se + 1e-12, (beta, col, v.mean(), ex, se)
        # <E^2> from the raw moments (both replicas of the pair count)
        e2_ex = float(np.sum(w * Es.astype(float) ** 2))
        e2 = mom["E2"][:, k] / (2.0 * n)
        se2 = e2.std(ddof=1) / math.sqrt(S)
        assert abs(e2.mean() - e2_ex) < 5 * se2, (beta, e2.mean(), e2_ex, se2)
        # Binder parameter from pooled numerators, jackknife over samples
        q2s = mom["Q2"][:, k].astype(float)
        q4s = mom["Q4"][:, k, 0].astype(float) + mom["Q4"][:, k, 1].astype(float) * 2.0 ** 64
        def g_of(idx):
            a = q4s[idx].sum() / (len(idx) * n * N ** 4)
            b = q2s[idx].sum() / (len(idx) * n * N ** 2)
            return 0.5 * (3 - a / b ** 2)
        full = g_of(np.arange(S))
        jk = np.array([g_of(np.delete(np.arange(S), i)) for i in range(S)])
        se_g = math.sqrt((S - 1) / S * np.sum((jk - jk.mean()) ** 2))
        g_ex = 0.5 * (3 - q4_ex / q2_ex ** 2)
        assert abs(dis[k, 5] - full) < 1e-12
        assert abs(full - g_ex) < 5 * se_g + 1e-9, (beta, full, g_ex, se_g)
