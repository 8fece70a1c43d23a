"""Pins for the oracle's multi-cluster variant of the Houdayer move (proposed in
Sec. 3 and Sec. 5): every q = -1 cluster of the pair is exchanged,
independently, with probability 1/2, the cluster named by its lowest site.

Cluster identification is checked against a breadth-first labelling written
here, energies against brute-force recomputation, the coins for fairness and
independence, and a whole PT + multi-cluster chain against the exact 4x4
moments.  Detailed balance of the move follows from what these pin: the
outcome is the exchange on any union of clusters with probability 2^-n, the
clusters (the q field) are unchanged by it, the same coins undo it, and
E_a + E_b is conserved."""
import math
from collections import deque

import numpy as np
import pytest

import exact
from paper_2003_04621_amd import workloads as W


def _neighbours(L, d, i):
    x = [i % L, (i // L) % L, i // (L * L) if d == 3 else 0]
    out = []
    for mu in range(d):
        for dx in (1, -1):
            y = list(x)
            y[mu] = (y[mu] + dx) % L
            out.append(y[0] + L * y[1] + (L * L * y[2] if d == 3 else 0))
    return out


def _components(L, d, minus):
    """Connected components of the q = -1 sites: site -> lowest site of its
    component (-1 for q = +1 sites)."""
    N = L ** d
    rep = np.full(N, -1, np.int64)
    for i0 in range(N):
        if not minus[i0] or rep[i0] >= 0:
            continue
        comp = [i0]
        rep[i0] = i0
        dq = deque([i0])
        while dq:
            i = dq.popleft()
            for j in _neighbours(L, d, i):
                if minus[j] and rep[j] < 0:
                    rep[j] = i0
                    comp.append(j)
                    dq.append(j)
        assert min(comp) == i0
    return rep


@pytest.mark.parametrize("L,d", [(4, 2), (5, 2), (8, 2), (3, 3), (4, 3), (6, 3)])
def test_multi_move_exchanges_exactly_the_chosen_clusters(orc, L, d):
    rng = np.random.default_rng(100 * L + d)
    N = L ** d
    for trial in range(20):
        J = rng.choice(np.array([-1, 1], np.int8), size=(d, N))
        sa = rng.choice(np.array([-1, 1], np.int8), size=N)
        sb = rng.choice(np.array([-1, 1], np.int8), size=N)
        coin = rng.integers(0, 2, size=N).astype(np.uint8)
        q0 = sa * sb
        rep = _components(L, d, q0 < 0)
        want = np.array([rep[i] >= 0 and coin[rep[i]] == 1 for i in range(N)])
        Ea, Eb = exact.brute_energy(L, d, J, sa), exact.brute_energy(L, d, J, sb)
        a, b = sa.copy(), sb.copy()
        delta, fl, ncl = orc.houdayer_multi_move(L, d, J, a, b, coin)
        assert ncl == len(set(rep[rep >= 0].tolist()))
        assert (fl == want).all()
        assert (a * b == q0).all()                                     # q field unchanged
        assert (a[fl] == sb[fl]).all() and (b[fl] == sa[fl]).all()     # exchanged
        assert (a[~fl] == sa[~fl]).all() and (b[~fl] == sb[~fl]).all()
        Ea2, Eb2 = exact.brute_energy(L, d, J, a), exact.brute_energy(L, d, J, b)
        assert Ea2 - Ea == delta and Eb2 - Eb == -delta
        assert Ea2 + Eb2 == Ea + Eb
        # the same coins undo the move: the clusters and their lowest sites are
        # those of the q field, which the move leaves alone
        orc.houdayer_multi_move(L, d, J, a, b, coin)
        assert (a == sa).all() and (b == sb).all()


def test_multi_move_all_or_no_coins(orc):
    """Every coin set exchanges every q = -1 site: the two configurations
    trade places, delta = E_b - E_a.  No coin set: nothing moves."""
    rng = np.random.default_rng(5)
    for L, d in [(6, 2), (4, 3)]:
        N = L ** d
        J = rng.choice(np.array([-1, 1], np.int8), size=(d, N))
        sa = rng.choice(np.array([-1, 1], np.int8), size=N)
        sb = rng.choice(np.array([-1, 1], np.int8), size=N)
        Ea, Eb = exact.brute_energy(L, d, J, sa), exact.brute_energy(L, d, J, sb)
        a, b = sa.copy(), sb.copy()
        delta, _, _ = orc.houdayer_multi_move(L, d, J, a, b, np.ones(N, np.uint8))
        assert (a == sb).all() and (b == sa).all() and delta == Eb - Ea
        a, b = sa.copy(), sb.copy()
        delta, fl, _ = orc.houdayer_multi_move(L, d, J, a, b, np.zeros(N, np.uint8))
        assert delta == 0 and not fl.any() and (a == sa).all() and (b == sb).all()
        # identical replicas: no cluster at all
        a, b = sa.copy(), sa.copy()
        delta, fl, n = orc.houdayer_multi_move(L, d, J, a, b, np.ones(N, np.uint8))
        assert delta == 0 and n == 0 and not fl.any()


def test_multi_coins_are_fair_bits(orc):
    """Coins over many passes: each position is 1 half the time, and the
    coins of two positions are independent (2x2 table)."""
    N, T = 300, 4000
    c = np.array([orc.multi_coins(77, 3, 5, v, N) for v in range(T)], np.int64)
    p = c.mean(axis=0)
    assert np.abs(p - 0.5).max() < 5 * math.sqrt(0.25 / T) + 0.02
    for i, j in [(0, 1), (0, 127), (127, 128), (31, 32), (5, 299)]:
        tab = np.array([[np.sum((c[:, i] == x) & (c[:, j] == y)) for y in (0, 1)] for x in (0, 1)],
                       float)
        chi2 = float(np.sum((tab - T / 4) ** 2 / (T / 4)))
        assert exact.chi2_sf(chi2, 3) > 1e-4, (i, j, tab)
    # different temperatures, samples and seeds draw different coins
    base = orc.multi_coins(77, 3, 5, 0, N)
    for args in [(78, 3, 5, 0), (77, 4, 5, 0), (77, 3, 6, 0)]:
        assert (orc.multi_coins(*args, N) != base).any()


def test_multi_pass_outcomes_uniform_over_cluster_subsets(orc):
    """A job's multi-cluster pass on a fixed pair state: each of the 2^n
    unions of its n clusters comes out with probability 2^-n (chi-square over
    passes), and nothing else does."""
    L, d, NT = 6, 2, 2
    N = L * L
    J = W.ferromagnet(1, L, d)
    job = orc.OracleJob(1, NT, L, d, J, W.geometric_betas(1.0, 2.0, NT), 9)
    sp = job.spins()
    sp[0, :, :] = 1
    minus_sites = [0, 1, 8, 20, 21, 27, 33]       # clusters {0,1}, {8}, {20,21,27,33}
    rep = _components(L, d, np.isin(np.arange(N), minus_sites))
    roots = sorted(set(rep[rep >= 0].tolist()))
    assert len(roots) == 3
    hist = {}
    T = 4000
    for _ in range(T):
        s = sp.copy()
        s[0, NT + 0, minus_sites] = -1             # set 1, temperature 0 (identity maps)
        job.set_spins(s)
        job.houdayer(multi=True)
        out = job.spins()[0, 0]
        flipped = tuple(int(r) for r in roots if out[r] == -1)
        for r in roots:                            # whole clusters only
            members = np.flatnonzero(rep == r)
            assert len(set(out[members].tolist())) == 1
        hist[flipped] = hist.get(flipped, 0) + 1
    assert len(hist) == 8
    obs = np.array(list(hist.values()), float)
    chi2 = float(np.sum((obs - T / 8) ** 2 / (T / 8)))
    assert exact.chi2_sf(chi2, 7) > 1e-4, hist
    assert job.counters()["v"] == T


def test_4x4_pt_multicluster_matches_exact_moments(orc):
    """Metropolis + multi-cluster Houdayer + PT on 4x4 +-J samples reproduces
    the exact <e>, <|q|>, <q^2>, <q^4> (Walsh-Hadamard enumeration)."""
    L, d, S = 4, 2, 64
    N = L * L
    J1 = W.couplings_pm_j(1, L, d, 13)
    Es = orc.state_energies(L, d, J1[0])
    betas = np.array([1.5, 1.0, 0.6, 0.3])
    job = orc.OracleJob(S, len(betas), L, d, np.repeat(J1, S, axis=0), betas, 4)
    job.mcs(400, houdayer=True, multi=True)
    job.mcs(2000, houdayer=True, multi=True, measure=True)
    ps, dis, n = job.observables()
    for k, beta in enumerate(betas):
        logw = -beta * Es.astype(float)
        w = np.exp(logw - logw.max())
        w /= w.sum()
        e_ex = float(np.sum(w * Es)) / N
        q2_ex, q4_ex, norm = exact.overlap_moments(Es, N, beta)
        aq_ex = exact.abs_overlap(Es, N, beta)
        for col, ex in [(0, e_ex), (1, 0.0), (2, aq_ex), (3, q2_ex), (4, q4_ex)]:
            v = ps[:, k, col]
            se = v.std(ddof=1) / math.sqrt(S)
            assert abs(v.mean() - ex) < 5 * se + 1e-12, (beta, col, v.mean(), ex, se)
