"""Exact reference quantities used to pin the oracle (test-side helpers).

Everything here is independent of the oracle's simulation code: brute-force
energies with numpy, canonical averages from an exact density of states,
overlap moments of two independent replicas by a Walsh-Hadamard transform, and
Kaufman's closed-form partition function of the periodic square-lattice Ising
ferromagnet.
"""
from __future__ import annotations

import math

import numpy as np


def lattice_shape(L: int, d: int):
    # site i = x0 + L*x1 (+ L^2*x2): numpy C-order shape is reversed
    return (L,) * d


def brute_energy(L: int, d: int, J: np.ndarray, s: np.ndarray) -> int:
    """E = -sum_<ij> J_ij s_i s_j over the d*N bonds (i, i+e_mu), via np.roll."""
    shp = lattice_shape(L, d)
    sg = s.reshape(shp).astype(np.int64)
    E = 0
    for mu in range(d):
        axis = d - 1 - mu        # x0 is the last numpy axis
        Jm = J[mu].reshape(shp).astype(np.int64)
        E -= int(np.sum(Jm * sg * np.roll(sg, -1, axis=axis)))
    return E


def boltzmann_from_dos(counts: np.ndarray, d: int, N: int, beta: float):
    """Returns (energies, probabilities) of the canonical distribution."""
    E = np.arange(-d * N, d * N + 1, dtype=np.float64)
    c = counts.astype(np.float64)
    nz = c > 0
    E, c = E[nz], c[nz]
    logw = np.log(c) - beta * E
    logw -= logw.max()
    w = np.exp(logw)
    return E, w / w.sum()


def mean_energy_from_dos(counts, d, N, beta):
    E, p = boltzmann_from_dos(counts, d, N, beta)
    return float(np.sum(E * p)), float(np.sum(E * E * p))


def _wht(a: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along the only axis."""
    a = a.copy()
    h = 1
    n = a.shape[0]
    while h < n:
        a = a.reshape(-1, 2, h)
        x, y = a[:, 0, :].copy(), a[:, 1, :].copy()
        a[:, 0, :] = x + y
        a[:, 1, :] = x - y
        a = a.reshape(n)
        h *= 2
    return a


def overlap_moments(state_E: np.ndarray, N: int, beta: float):
    """Exact <q^2>, <q^4> for two independent replicas with the same couplings.

    q(x, y) = 1 - 2 popcount(x ^ y) / N depends only on z = x ^ y, so
    <q^p> = sum_z A(z) q(z)^p with A(z) = sum_x pi(x) pi(x ^ z), the XOR
    autocorrelation of pi, computed as WHT^-1(WHT(pi)^2)."""
    logw = -beta * state_E.astype(np.float64)
    logw -= logw.max()
    pi = np.exp(logw)
    pi /= pi.sum()
    F = _wht(pi)
    A = _wht(F * F) / len(pi)
    z = np.arange(len(pi), dtype=np.uint64)
    pop = np.zeros(len(pi), np.int64)
    for i in range(N):
        pop += ((z >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
    q = 1.0 - 2.0 * pop / N
    return float(np.sum(A * q * q)), float(np.sum(A * q ** 4)), float(np.sum(A))


def abs_overlap(state_E: np.ndarray, N: int, beta: float) -> float:
    """Exact <|q|> for two independent replicas (same construction as above)."""
    logw = -beta * state_E.astype(np.float64)
    logw -= logw.max()
    pi = np.exp(logw)
    pi /= pi.sum()
    F = _wht(pi)
    A = _wht(F * F) / len(pi)
    z = np.arange(len(pi), dtype=np.uint64)
    pop = np.zeros(len(pi), np.int64)
    for i in range(N):
        pop += ((z >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
    return float(np.sum(A * np.abs(1.0 - 2.0 * pop / N)))


def kaufman_log_z(L: int, K: float) -> float:
    """ln Z of the L x L periodic Ising ferromagnet at coupling K = beta J
    (Kaufman 1949): Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4) with
    Z1 = prod_r 2cosh(L g_{2r+1}/2), Z2 = prod_r 2sinh(L g_{2r+1}/2),
    Z3 = prod_r 2cosh(L g_{2r}/2),   Z4 = prod_r 2sinh(L g_{2r}/2),
    r = 0..L-1, cosh g_k = cosh 2K coth 2K - cos(pi k / L) for k >= 1 and
    g_0 = 2K + ln tanh K (which changes sign at the critical point)."""
    N = L * L

    def gamma(k):
        if k == 0:
            return 2 * K + math.log(math.tanh(K))
        c = math.cosh(2 * K) / math.tanh(2 * K) - math.cos(math.pi * k / L)
        return math.acosh(c)

    terms = []   # (sign, log|Z_i|)
    for parity, fn in ((1, "cosh"), (1, "sinh"), (0, "cosh"), (0, "sinh")):
        sign, logabs = 1.0, 0.0
        for r in range(L):
            a = L * gamma(2 * r + parity) / 2
            if fn == "cosh":       # ln(2 cosh a)
                logabs += abs(a) + math.log1p(math.exp(-2 * abs(a)))
            else:                  # ln|2 sinh a|, sign tracked separately
                if a == 0.0:
                    sign = 0.0
                    break
                logabs += abs(a) + math.log1p(-math.exp(-2 * abs(a)))
                if a < 0:
                    sign = -sign
        terms.append((sign, logabs))
    m = max(t[1] for t in terms if t[0] != 0.0)
    tot = sum(s * math.exp(la - m) for s, la in terms if s != 0.0)
    return math.log(0.5) + (N / 2) * math.log(2 * math.sinh(2 * K)) + m + math.log(tot)


def kaufman_mean_energy(L: int, beta: float, h: float = 1e-5) -> float:
    """<E> = -d ln Z / d beta (J = 1), central difference."""
    return -(kaufman_log_z(L, beta + h) - kaufman_log_z(L, beta - h)) / (2 * h)


def chi2_sf(x: float, k: int) -> float:
    """Survival function of the chi-square distribution with k dof."""
    from scipy.stats import chi2
    return float(chi2.sf(x, k))
