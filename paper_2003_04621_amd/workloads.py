"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module holds no arithmetic of the simulation method: it only draws the
quenched couplings (bimodal, Eq. (2) of the paper, p = 1/2 unless asked
otherwise) with numpy's PCG64 generator, builds temperature ladders (fixed
geometric ladder of Sec. 2.3 and the power-law family of Eqs. (6)-(7)), and
names the benchmark workloads.  Random numbers the method itself draws
(initial spins, Metropolis, exchange, Houdayer) are not made here.

Coupling layout: int8 [samples][dim][L^dim], value +1 or -1; entry
[s][mu][i] is the bond between site i and its neighbour i + e_mu (periodic),
with site i = x0 + L*x1 (+ L^2*x2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def couplings_pm_j(samples: int, L: int, dim: int, seed: int, p: float = 0.5) -> np.ndarray:
    """Bimodal couplings, Eq. (2): +1 with probability p, else -1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((samples, dim, L ** dim))
    return np.where(u < p, 1, -1).astype(np.int8)


# Gaussian couplings live on a fixed-point grid: J = n * GAUSS_UNIT, |J| <= GAUSS_MAX.
GAUSS_UNIT = 2.0 ** -16
GAUSS_MAX = 8.0


def couplings_gauss(samples: int, L: int, dim: int, seed: int) -> np.ndarray:
    """Gaussian couplings (Sec. 2.1: standard normal) as float32 [samples][dim][L^dim]:
    normal draws rounded to the nearest multiple of 2^-16 and clipped to [-8, 8]
    (the grid every value of which a float32 holds exactly)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((samples, dim, L ** dim))
    n = np.clip(np.rint(z / GAUSS_UNIT), -GAUSS_MAX / GAUSS_UNIT, GAUSS_MAX / GAUSS_UNIT)
    return (n * GAUSS_UNIT).astype(np.float32)


def gauss_units(J: np.ndarray) -> np.ndarray:
    """The integer grid units n = J / 2^-16 of float32 Gaussian couplings."""
    return np.rint(np.asarray(J, np.float64) / GAUSS_UNIT).astype(np.int32)


def ferromagnet(samples: int, L: int, dim: int) -> np.ndarray:
    """J = +1 everywhere (p = 1 in Eq. (2)): the pure Ising ferromagnet."""
    return np.ones((samples, dim, L ** dim), np.int8)


def geometric_betas(t_min: float, t_max: float, n: int) -> np.ndarray:
    """Geometric temperature ladder T_k = T_min (T_max/T_min)^(k/(n-1)).

    Returned as inverse temperatures, index 0 the coldest (largest beta)."""
    k = np.arange(n, dtype=np.float64)
    T = t_min * (t_max / t_min) ** (k / (n - 1))
    return 1.0 / T


def power_law_betas(t_min: float, t_max: float, n: int, phi: float) -> np.ndarray:
    """Power-law protocol, Eqs. (6)-(7): T_i = i^phi T_norm + T_min with
    T_norm = (T_max - T_min) / (n-1)^phi.  Returned as inverse temperatures."""
    i = np.arange(n, dtype=np.float64)
    t_norm = (t_max - t_min) / (n - 1) ** phi
    T = i ** phi * t_norm + t_min
    return 1.0 / T


def phi_star(L: int) -> float:
    """Linear fit of the optimal exponent, Eq. (8): a_phi + b_phi L with the
    constants printed for the 2D Gaussian model (a_phi = 0.406, b_phi = 0.014)."""
    return 0.406 + 0.014 * L


def n_t_star(L: int) -> int:
    """Linear fit of the optimal number of temperatures, Eq. (9):
    a_NT + b_NT L with the constants printed for the 2D Gaussian model
    (a_NT = 0.025, b_NT = 0.644), rounded to the nearest count and at least 2."""
    return max(2, int(round(0.025 + 0.644 * L)))


def optimized_betas(L: int, t_min: float, t_max: float) -> np.ndarray:
    """The power-law ladder of Eqs. (6)-(7) with the fitted phi*(L) and
    N_T*(L) of Eqs. (8)-(9): the paper's recipe for sizes not simulated
    directly (fitted on the 2D Gaussian model)."""
    return power_law_betas(t_min, t_max, n_t_star(L), phi_star(L))


@dataclass
class Workload:
    name: str
    dim: int
    L: int
    samples: int
    replicas: int          # N_T, temperatures per replica set
    betas: np.ndarray
    sweeps: int
    houdayer: bool
    couplings_seed: int = 1000
    seed: int = 2000
    notes: str = ""
    extra: dict = field(default_factory=dict)
    gauss: bool = False    # Gaussian couplings (float32 on the 2^-16 grid) instead of +-J

    @property
    def N(self) -> int:
        return self.L ** self.dim

    @property
    def flips_per_sweep(self) -> int:
        """Attempted single-spin updates per sweep of the whole job (Eq. (11)
        normaliser: N_T * N_C * samples * L^d with N_C = 2)."""
        return self.samples * 2 * self.replicas * self.N

    def couplings(self) -> np.ndarray:
        if self.gauss:
            return couplings_gauss(self.samples, self.L, self.dim, self.couplings_seed)
        return couplings_pm_j(self.samples, self.L, self.dim, self.couplings_seed)


def workload(name: str) -> Workload:
    """The named workloads.

    small3d : 3D +-J, L=8, 8 samples x 16 temperatures, T in [0.9, 2.0]
              geometric, 1000 sweeps with exchange every sweep.
    3d_l16  : 3D +-J, L=16, 1000 samples x 32 temperatures, T in [0.9, 2.0]
              geometric, 10^4 sweeps + exchange, observables over the second
              half.
    2d_l64  : 2D +-J, L=64, 500 samples x 24 temperatures, T in [0.2, 1.6]
              on the power-law ladder with phi = phi*(64), 5000 sweeps of
              Metropolis + Houdayer + exchange.
    3d_l48  : 3D +-J, L=48, 64 samples x 32 temperatures, T in [0.9, 2.0]
              geometric (the largest served size; each sample's 64
              configurations span several workgroups).
    3d_l32  : 3D +-J, L=32, 128 samples x 32 temperatures, T in [0.9, 2.0]
              geometric (served size, split over two workgroups).
    2d_l64_gauss : 2D with Gaussian couplings (Sec. 4.2's model), otherwise
              the 2d_l64 workload: L=64, 500 samples x 24 temperatures on the
              same power-law ladder, Metropolis + Houdayer + exchange.
    """
    if name == "small3d":
        return Workload(name, 3, 8, 8, 16, geometric_betas(0.9, 2.0, 16), 1000, False)
    if name == "3d_l16":
        return Workload(name, 3, 16, 1000, 32, geometric_betas(0.9, 2.0, 32), 10000, False)
    if name == "2d_l64":
        return Workload(name, 2, 64, 500, 24, power_law_betas(0.2, 1.6, 24, phi_star(64)),
                        5000, True)
    if name == "2d_l64_gauss":
        return Workload(name, 2, 64, 500, 24, power_law_betas(0.2, 1.6, 24, phi_star(64)),
                        5000, True, gauss=True)
    if name == "3d_l48":
        return Workload(name, 3, 48, 64, 32, geometric_betas(0.9, 2.0, 32), 10000, False)
    if name == "3d_l32":
        return Workload(name, 3, 32, 128, 32, geometric_betas(0.9, 2.0, 32), 10000, False)
    raise KeyError(name)
