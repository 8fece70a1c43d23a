"""Pins of the oracle's two-replica modes (spin-glass susceptibility and
correlation length; named in Sec. 3, defined by the usual formulas).

The oracle accumulates A(delta) = sum over axes mu of sum_x P_mu(x)
P_mu(x + delta), P_mu the plane sums of the overlap field q_i = s_i^a s_i^b.
Fixed here against
  * numpy's FFT: sum_delta cos(2 pi n delta / L) A(delta) equals the summed
    squared Fourier modes |sum_i q_i exp(2 pi i n x_mu / L)|^2 for every n, which
    determines every A(delta);
  * the sum rule sum_delta A(delta) = d Q^2 (Q = sum_i q_i), tying the modes to
    the overlap moment measured alongside;
  * closed forms: identical replicas (q = 1) and a staggered overlap;
  * the per-measurement accumulation over a run, recomputed from the spins;
  * a hand-worked correlation length.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2003_04621_amd import workloads


def _fft_power(q, L, d, n):
    """sum over axes of |sum_i q_i exp(2 pi i n x_mu / L)|^2 by numpy's FFT."""
    a = np.asarray(q, np.float64).reshape((L,) * d)  # C order: [x_{d-1}] ... [x0]
    tot = 0.0
    for mu in range(d):
        axis = d - 1 - mu
        others = tuple(ax for ax in range(d) if ax != axis)
        P = a.sum(axis=others)
        tot += abs(np.fft.fft(P)[n]) ** 2
    return tot


@pytest.mark.parametrize("L,d", [(4, 2), (5, 2), (6, 2), (8, 2), (3, 3), (4, 3), (6, 3)])
def test_modes_equal_fft(L, d):
    rng = np.random.default_rng(L * 10 + d)
    N = L ** d
    for _ in range(3):
        sa = rng.choice([-1, 1], N).astype(np.int8)
        sb = rng.choice([-1, 1], N).astype(np.int8)
        A = oracle.overlap_modes(L, d, sa, sb)
        q = sa.astype(int) * sb
        for n in range(L):
            want = _fft_power(q, L, d, n)
            assert oracle.mode_power(A, L, n) == pytest.approx(want, rel=1e-12, abs=1e-9)
        # sum rule: every delta of the autocorrelation adds up to the squared total
        Aext = [A[t] if t <= L // 2 else A[L - t] for t in range(L)]
        assert sum(int(x) for x in Aext) == d * int(q.sum()) ** 2


@pytest.mark.parametrize("L,d", [(4, 2), (8, 2), (4, 3), (6, 3)])
def test_modes_closed_forms(L, d):
    N = L ** d
    plane = L ** (d - 1)
    s = np.random.default_rng(1).choice([-1, 1], N).astype(np.int8)
    A = oracle.overlap_modes(L, d, s, s)  # q = 1 everywhere: P_mu(x) = L^(d-1)
    assert list(A) == [d * L * plane * plane] * (L // 2 + 1)
    assert oracle.mode_power(A, L, 1) == pytest.approx(0.0, abs=1e-6)
    x0 = np.arange(N) % L
    sb = (s * np.where(x0 % 2 == 0, 1, -1)).astype(np.int8)  # q = (-1)^x0
    A = oracle.overlap_modes(L, d, s, sb)
    assert list(A) == [L * plane * plane * (-1) ** t for t in range(L // 2 + 1)]


def test_modes_accumulate_over_a_run():
    S, NT, L, d, P = 2, 3, 6, 3, 7
    J = workloads.couplings_pm_j(S, L, d, seed=5)
    betas = workloads.geometric_betas(0.8, 2.0, NT)
    job = oracle.OracleJob(S, NT, L, d, J, betas, 99)
    job.mcs(2)  # not accumulated: before enabling
    job.enable_modes()
    want = np.zeros((S, NT, L // 2 + 1), np.int64)
    for _ in range(P):
        job.mcs(1, measure=True)
        spins, (sot, _) = job.spins(), job.maps()
        for s in range(S):
            for k in range(NT):
                a, b = spins[s, sot[s, 0, k]], spins[s, NT + sot[s, 1, k]]
                want[s, k] += oracle.overlap_modes(L, d, a, b)
    got = job.modes()
    np.testing.assert_array_equal(got, want)
    # the sum rule against the measured Q^2 moment
    Q2 = job.moments()["Q2"]
    ext = got.sum(axis=2) * 2 - got[:, :, 0] - got[:, :, L // 2]  # L even
    np.testing.assert_array_equal(ext, d * Q2)


def test_correlation_length_hand_value():
    L, d, S, n = 4, 2, 1, 1
    N = L ** d
    # chi(k_min) = (A0 - A2) / (d S n N) = 32 / 32 = 1; chi(0) = 80 / 16 = 5
    modes = np.array([[[64, 0, 32]]], np.int64)
    chi0, chik, xi = oracle.correlation_length(modes, [[80]], n, L, d)
    assert chi0[0] == 5.0 and chik[0] == 1.0
    assert xi[0] == pytest.approx(math.sqrt(4.0) / (2 * math.sin(math.pi / 4)), rel=1e-15)
    # no correlation beyond the site: chi(0) = chi(k_min) gives xi = 0
    chi0, chik, xi = oracle.correlation_length(np.array([[[32, 0, 0]]]), [[16]], n, L, d)
    assert chi0[0] == chik[0] == 1.0 and xi[0] == 0.0
    # identical replicas: chi(k_min) = 0, xi undefined
    _, chik, xi = oracle.correlation_length(np.array([[[128, 128, 128]]]), [[256]], n, L, d)
    assert chik[0] == 0.0 and np.isnan(xi[0])


def test_independent_replicas_have_unit_susceptibility():
    """At a vanishing inverse temperature every proposed flip is taken, both
    replicas flip every spin each sweep, and the overlap stays the product of
    two independent random initial states: chi_SG(k) = 1 on average for
    every k, so xi is near 0."""
    S, NT, L, d = 60, 2, 8, 2
    J = workloads.couplings_pm_j(S, L, d, seed=8)
    betas = np.array([1e-9, 0.5e-9])
    job = oracle.OracleJob(S, NT, L, d, J, betas, 3)
    job.enable_modes()
    job.mcs(4, measure=True)
    chi0, chik, xi = oracle.correlation_length(job.modes(), job.moments()["Q2"], 4, L, d)
    assert abs(chi0[0] - 1.0) < 0.35 and abs(chik[0] - 1.0) < 0.35
