"""CPU oracle for the parallel-tempering EA spin-glass path -- TEST INFRASTRUCTURE.

A plain, slow, single-threaded C implementation (``ea_oracle.c`` for bimodal
couplings, ``gauss_oracle.c`` for Gaussian ones) of what the GPU path
computes, plus an independent exact-enumeration helper (``enum.c``).
Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product library never does.

The arithmetic lives in C; this module only marshals numpy arrays through
ctypes.  Build with :func:`build` (gcc -O2, no fast-math, no intrinsics).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["ea_oracle.c", "enum.c", "gauss_oracle.c"]
_lib = None


def build() -> str:
    """Compile the oracle shared library (always recompiles)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fvisibility=hidden",
           "-o", tmp] + srcs + ["-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


P = C.c_void_p


def _declare(L):
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_philox4x32_10.restype = None
    L.or_philox_stream.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, P,
                                   C.c_int64, P]
    L.or_philox_stream.restype = None
    L.or_energy.argtypes = [C.c_int, C.c_int, P, P]
    L.or_energy.restype = C.c_int64
    L.or_local_x.argtypes = [C.c_int, C.c_int, P, P, C.c_int]
    L.or_local_x.restype = C.c_int
    L.or_metro_thresholds.argtypes = [P, C.c_int, C.c_int, P]
    L.or_metro_thresholds.restype = None
    L.or_pt_thresholds.argtypes = [P, C.c_int, C.c_int, C.c_int, P, C.c_int]
    L.or_pt_thresholds.restype = C.c_int
    L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, C.c_uint64, P]
    L.or_create.restype = P
    L.or_destroy.argtypes = [P]
    L.or_destroy.restype = None
    for name in ("or_exchange", "or_houdayer", "or_houdayer_multi", "or_measure",
                 "or_recompute_energies"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = None
    L.or_sweep.argtypes = [P, C.c_int]
    L.or_sweep.restype = None
    L.or_mcs.argtypes = [P, C.c_int, C.c_int, C.c_int]
    L.or_mcs.restype = None
    L.or_houdayer_move.argtypes = [C.c_int, C.c_int, P, P, P, C.c_uint64, P, P]
    L.or_houdayer_move.restype = C.c_int64
    L.or_houdayer_multi_move.argtypes = [C.c_int, C.c_int, P, P, P, P, P, P]
    L.or_houdayer_multi_move.restype = C.c_int64
    L.or_multi_coins.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, P]
    L.or_multi_coins.restype = None
    L.or_observables.argtypes = [P, P, P, P]
    L.or_observables.restype = None
    L.or_get_spins.argtypes = [P, P]
    L.or_set_spins.argtypes = [P, P]
    L.or_get_energies.argtypes = [P, P]
    L.or_get_maps.argtypes = [P, P, P]
    L.or_get_counters.argtypes = [P, P]
    L.or_get_moments.argtypes = [P, P, P, P, P, P, P]
    L.or_get_walk.argtypes = [P, P, P, P]
    L.or_overlap_modes.argtypes = [C.c_int, C.c_int, P, P, P]
    L.or_enable_modes.argtypes = [P]
    L.or_get_modes.argtypes = [P, P]
    L.or_set_measure_every.argtypes = [P, C.c_int]
    L.or_get_stats.argtypes = [P, P]
    L.or_pt_table_len.argtypes = [P]
    L.or_pt_table_len.restype = C.c_int
    L.or_get_pt_table.argtypes = [P, P]
    L.or_sweep_order.argtypes = [C.c_int, C.c_int, P]
    L.or_metro_rule.argtypes = [C.c_int, C.c_uint32, P]
    L.or_metro_rule.restype = C.c_int
    L.org_energy.argtypes = [C.c_int, C.c_int, P, P]
    L.org_energy.restype = C.c_int64
    L.org_local_x.argtypes = [C.c_int, C.c_int, P, P, C.c_int]
    L.org_local_x.restype = C.c_int64
    L.org_accept.argtypes = [C.c_uint32, C.c_double, C.c_int64]
    L.org_accept.restype = C.c_int
    L.org_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, C.c_uint64, P]
    L.org_create.restype = P
    L.org_destroy.argtypes = [P]
    L.org_destroy.restype = None
    for name in ("org_exchange", "org_measure", "org_recompute_energies"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = None
    L.org_sweep.argtypes = [P, C.c_int]
    L.org_houdayer.argtypes = [P, C.c_int]
    L.org_mcs.argtypes = [P, C.c_int, C.c_int, C.c_int]
    L.org_set_measure_every.argtypes = [P, C.c_int]
    L.org_observables.argtypes = [P, P, P, P]
    L.org_get_spins.argtypes = [P, P]
    L.org_set_spins.argtypes = [P, P]
    L.org_get_energies.argtypes = [P, P]
    L.org_get_maps.argtypes = [P, P, P]
    L.org_get_counters.argtypes = [P, P]
    L.org_get_moments.argtypes = [P, P, P, P, P, P, P]
    L.en_density_of_states.argtypes = [C.c_int, C.c_int, P, P]
    L.en_density_of_states.restype = C.c_int
    L.en_state_energies.argtypes = [C.c_int, C.c_int, P, P]
    L.en_state_energies.restype = C.c_int


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def nsites(L: int, d: int) -> int:
    return L ** d


# --------------------------------------------------------------------------
# Stateless helpers
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_stream(c0, c1, c2, c3, key, n) -> np.ndarray:
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros((n, 4), np.uint32)
    lib().or_philox_stream(c0, c1, c2, c3, _p(k), n, _p(out))
    return out


def energy(L: int, d: int, J: np.ndarray, spins: np.ndarray) -> int:
    J = np.ascontiguousarray(J, dtype=np.int8)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().or_energy(L, d, _p(J), _p(s)))


def local_x(L: int, d: int, J: np.ndarray, spins: np.ndarray, i: int) -> int:
    J = np.ascontiguousarray(J, dtype=np.int8)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().or_local_x(L, d, _p(J), _p(s), i))


def metro_thresholds(betas, d: int) -> np.ndarray:
    b = np.ascontiguousarray(betas, dtype=np.float64)
    out = np.zeros((len(b), d), np.uint32)
    lib().or_metro_thresholds(_p(b), len(b), d, _p(out))
    return out


def pt_thresholds(betas, d: int, N: int) -> np.ndarray:
    b = np.ascontiguousarray(betas, dtype=np.float64)
    M = lib().or_pt_thresholds(_p(b), len(b), d, N, None, 0)
    out = np.zeros((len(b) - 1, M), np.uint32)
    lib().or_pt_thresholds(_p(b), len(b), d, N, _p(out), M)
    return out


def metro_rule(x: int, r: int, thr_row: np.ndarray) -> int:
    t = np.ascontiguousarray(thr_row, dtype=np.uint32)
    return int(lib().or_metro_rule(int(x), int(r), _p(t)))


def sweep_order(L: int, d: int) -> np.ndarray:
    out = np.zeros(nsites(L, d), np.int32)
    lib().or_sweep_order(L, d, _p(out))
    return out


def houdayer_move(L, d, J, sa, sb, r64):
    """Applies one Houdayer move in place on int8 arrays sa, sb.

    Returns (delta, cluster_mask, cluster_size)."""
    J = np.ascontiguousarray(J, dtype=np.int8)
    assert sa.dtype == np.int8 and sb.dtype == np.int8
    assert sa.flags.c_contiguous and sb.flags.c_contiguous
    N = nsites(L, d)
    cl = np.zeros(N, np.int8)
    size = np.zeros(1, np.int32)
    delta = lib().or_houdayer_move(L, d, _p(J), _p(sa), _p(sb), C.c_uint64(r64),
                                   _p(cl), _p(size))
    return int(delta), cl.astype(bool), int(size[0])


def houdayer_multi_move(L, d, J, sa, sb, coin):
    """Applies one multi-cluster Houdayer move in place on int8 arrays sa, sb:
    the cluster whose lowest site is m is exchanged iff coin[m].

    Returns (delta, exchanged-site mask, number of clusters)."""
    J = np.ascontiguousarray(J, dtype=np.int8)
    assert sa.dtype == np.int8 and sb.dtype == np.int8
    assert sa.flags.c_contiguous and sb.flags.c_contiguous
    N = nsites(L, d)
    c = np.ascontiguousarray(coin, dtype=np.uint8)
    assert c.size == N
    fl = np.zeros(N, np.int8)
    n = np.zeros(1, np.int32)
    delta = lib().or_houdayer_multi_move(L, d, _p(J), _p(sa), _p(sb), _p(c), _p(fl), _p(n))
    return int(delta), fl.astype(bool), int(n[0])


def multi_coins(seed: int, sample: int, k: int, v: int, N: int) -> np.ndarray:
    """The coins of one multi-cluster move (pass v, temperature k, sample)."""
    out = np.zeros(N, np.uint8)
    lib().or_multi_coins(C.c_uint64(seed), sample, k, v, N, _p(out))
    return out


def density_of_states(L: int, d: int, J: np.ndarray) -> np.ndarray:
    N = nsites(L, d)
    J = np.ascontiguousarray(J, dtype=np.int8)
    out = np.zeros(2 * d * N + 1, np.uint64)
    rc = lib().en_density_of_states(L, d, _p(J), _p(out))
    assert rc == 0
    return out


def state_energies(L: int, d: int, J: np.ndarray) -> np.ndarray:
    N = nsites(L, d)
    J = np.ascontiguousarray(J, dtype=np.int8)
    out = np.zeros(1 << N, np.int32)
    rc = lib().en_state_energies(L, d, _p(J), _p(out))
    assert rc == 0
    return out


# --------------------------------------------------------------------------
# Job wrapper
# --------------------------------------------------------------------------
class OracleJob:
    """S samples x 2 replica sets x NT temperatures, as in the GPU library."""

    def __init__(self, samples, replicas, L, dim, couplings, betas, seed,
                 sample_keys=None):
        self.S, self.NT, self.L, self.d = int(samples), int(replicas), int(L), int(dim)
        self.N = nsites(self.L, self.d)
        self._J = np.ascontiguousarray(couplings, dtype=np.int8).reshape(
            self.S, self.d, self.N)
        self._b = np.ascontiguousarray(betas, dtype=np.float64)
        keys = None
        if sample_keys is not None:
            self._keys = np.ascontiguousarray(sample_keys, dtype=np.uint32)
            keys = _p(self._keys)
        self._h = lib().or_create(self.S, self.NT, self.L, self.d, _p(self._J),
                                  _p(self._b), C.c_uint64(seed), keys)
        if not self._h:
            raise ValueError("oracle rejected the job arguments")

    def close(self):
        if self._h:
            lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        lib().or_sweep(self._h, int(n))

    def exchange(self):
        lib().or_exchange(self._h)

    def houdayer(self, multi=False):
        """One Houdayer pass; multi=True: the multi-cluster variant."""
        if multi:
            lib().or_houdayer_multi(self._h)
        else:
            lib().or_houdayer(self._h)

    def measure(self):
        lib().or_measure(self._h)

    def mcs(self, n, houdayer=False, measure=False, multi=False):
        """n Monte Carlo steps; multi=True makes the Houdayer moves the
        multi-cluster variant."""
        h = (2 if multi else 1) if houdayer else 0
        lib().or_mcs(self._h, int(n), h, int(bool(measure)))

    def spins(self) -> np.ndarray:
        out = np.zeros((self.S, 2 * self.NT, self.N), np.int8)
        lib().or_get_spins(self._h, _p(out))
        return out

    def set_spins(self, spins):
        s = np.ascontiguousarray(spins, dtype=np.int8).reshape(self.S, 2 * self.NT, self.N)
        lib().or_set_spins(self._h, _p(s))

    def energies(self) -> np.ndarray:
        out = np.zeros((self.S, 2 * self.NT), np.int64)
        lib().or_get_energies(self._h, _p(out))
        return out

    def maps(self):
        sot = np.zeros((self.S, 2, self.NT), np.int32)
        tos = np.zeros((self.S, 2, self.NT), np.int32)
        lib().or_get_maps(self._h, _p(sot), _p(tos))
        return sot, tos

    def counters(self):
        out = np.zeros(4, np.uint64)
        lib().or_get_counters(self._h, _p(out))
        return dict(t=int(out[0]), u=int(out[1]), v=int(out[2]), n_meas=int(out[3]))

    def moments(self):
        ST = (self.S, self.NT)
        arrs = [np.zeros(ST, np.int64) for _ in range(5)]
        q4 = np.zeros(ST + (2,), np.uint64)
        lib().or_get_moments(self._h, *[_p(a) for a in arrs], _p(q4))
        names = ["E", "E2", "Q", "AQ", "Q2"]
        out = dict(zip(names, arrs))
        out["Q4"] = q4
        return out

    def pt_table(self) -> np.ndarray:
        M = lib().or_pt_table_len(self._h)
        out = np.zeros((self.NT - 1, M), np.uint32)
        lib().or_get_pt_table(self._h, _p(out))
        return out

    def walk(self):
        """Replica-walk state after the last exchange pass (Sec. 2.3): slot
        labels [S][2NT] (0 none, 1 going up, 2 going down), the pass at which
        each slot's current round trip began [S][2NT], and the round-trip bins
        [S][32][3] (trips ended in passes [2^b, 2^(b+1)): count, sum of
        lengths, sum of squared lengths)."""
        lab = np.zeros((self.S, 2 * self.NT), np.int32)
        beg = np.zeros((self.S, 2 * self.NT), np.uint32)
        trips = np.zeros((self.S, 32, 3), np.uint64)
        lib().or_get_walk(self._h, _p(lab), _p(beg), _p(trips))
        return lab, beg, trips

    def stats(self):
        """Run diagnostics [S][NT][24] (int64): accepted Metropolis flips at
        temperature k, accepted exchanges of (k, k+1), Houdayer passes at k
        that exchanged sites, the sites they exchanged, and a histogram of the
        exchanged sites per pass by floor(log2) (20 bins)."""
        out = np.zeros((self.S, self.NT, 24), np.int64)
        lib().or_get_stats(self._h, _p(out))
        return out

    def set_measure_every(self, every):
        """mcs() measures only after sweeps whose count is a multiple of every."""
        lib().or_set_measure_every(self._h, int(every))

    def enable_modes(self):
        """Accumulate the two-replica modes at every later measurement."""
        lib().or_enable_modes(self._h)

    def modes(self) -> np.ndarray:
        """Accumulated plane-sum autocorrelations A(delta), [S][NT][L/2+1]."""
        out = np.zeros((self.S, self.NT, self.L // 2 + 1), np.int64)
        lib().or_get_modes(self._h, _p(out))
        return out

    def observables(self):
        ps = np.zeros((self.S, self.NT, 5), np.float64)
        dis = np.zeros((self.NT, 6), np.float64)
        n = np.zeros(1, np.int64)
        lib().or_observables(self._h, _p(ps), _p(dis), _p(n))
        return ps, dis, int(n[0])


# --------------------------------------------------------------------------
# Round-trip time summary (Sec. 2.3)
# --------------------------------------------------------------------------
def tunnel_summary(trips, passes):
    """Round-trip time estimates from round-trip bins.

    trips: integer array [..., 32, 3] (count, sum of lengths, sum of squared
    lengths per logarithmic bin b of the pass at which a trip ended); every
    leading index is pooled.  passes: exchange passes done so far.

    Returns (tau_b[32], err_b[32], tau, equilibrated):
      tau_b = sum of lengths / count of bin b (nan when empty);
      err_b = standard error of that mean, sqrt((C Q - D^2) / (C^2 (C - 1)))
              with C, D, Q the bin's count, sum and sum of squares (nan when
              C < 2);
      tau   = all lengths over all trips (nan when there is none);
      equilibrated = 1 when the last three complete bins (bin b is complete
              once passes >= 2^(b+1) - 1) each hold two or more trips and
              every two of them differ by at most twice the root sum of
              squares of their errors -- the logarithmic-binning check, read
              as agreement of the last three bins within two standard errors.
    """
    t = np.asarray(trips, dtype=np.uint64).reshape(-1, 32, 3)
    C = [0] * 32
    D = [0] * 32
    Q = [0] * 32
    for row in t:
        for b in range(32):
            C[b] += int(row[b][0])
            D[b] += int(row[b][1])
            Q[b] += int(row[b][2])
    tau_b = np.full(32, np.nan)
    err_b = np.full(32, np.nan)
    for b in range(32):
        if C[b] > 0:
            tau_b[b] = D[b] / C[b]
        if C[b] > 1:
            num = C[b] * Q[b] - D[b] * D[b]
            err_b[b] = math.sqrt(float(num) / (float(C[b]) * float(C[b]) * float(C[b] - 1)))
    ctot, dtot = sum(C), sum(D)
    tau = dtot / ctot if ctot > 0 else float("nan")
    top = -1
    while top + 1 < 32 and (1 << (top + 2)) - 1 <= passes:
        top += 1
    eq = 0
    if top >= 2:
        last = [top - 2, top - 1, top]
        eq = 1
        for b in last:
            if C[b] < 2:
                eq = 0
        if eq:
            for i in range(3):
                for j in range(i + 1, 3):
                    a, b = last[i], last[j]
                    lim = 2.0 * math.sqrt(err_b[a] ** 2 + err_b[b] ** 2)
                    if abs(tau_b[a] - tau_b[b]) > lim:
                        eq = 0
    return tau_b, err_b, tau, eq


# --------------------------------------------------------------------------
# Two-replica modes: spin-glass susceptibility and correlation length
# --------------------------------------------------------------------------
def overlap_modes(L: int, d: int, sa, sb) -> np.ndarray:
    """A(delta), delta = 0 .. L/2, of one pair of configurations: the sum over
    the d axes of the autocorrelation of the overlap's plane sums."""
    a = np.ascontiguousarray(sa, dtype=np.int8)
    b = np.ascontiguousarray(sb, dtype=np.int8)
    out = np.zeros(L // 2 + 1, np.int64)
    lib().or_overlap_modes(int(L), int(d), _p(a), _p(b), _p(out))
    return out


def _cos_frac(m: int, L: int) -> float:
    """cos(2 pi m / L), exact where it is 0 or +-1."""
    m %= L
    if m == 0:
        return 1.0
    if 2 * m == L:
        return -1.0
    if 4 * m == L or 4 * m == 3 * L:
        return 0.0
    return math.cos(2.0 * math.pi * m / L)


def mode_power(A, L: int, n: int) -> float:
    """sum over the d axes of |sum_i q_i exp(2 pi i n x_mu / L)|^2 from A(0..L/2):
    sum_{delta=0}^{L-1} cos(2 pi n delta / L) A(delta), with A(L - delta) = A(delta),
    summed in increasing delta."""
    tot = 0.0
    for delta in range(L):
        a = A[delta] if delta <= L // 2 else A[L - delta]
        tot += _cos_frac(n * delta, L) * float(a)
    return tot


def correlation_length(modes, Q2, n_meas: int, L: int, d: int):
    """Per temperature, disorder-averaged (integer sums over samples first):
    chi_SG(0) = [sum Q^2] / (S n_meas N), chi_SG(k_min) = [sum_mu |q(k_mu)|^2 N^2]
    / (d S n_meas N) with k_min = 2 pi / L along each axis, and the second-moment
    correlation length xi = sqrt(chi(0)/chi(k_min) - 1) / (2 sin(pi / L))
    (nan where the ratio is below 1 or chi(k_min) is 0).

    modes: [S][NT][L/2+1] accumulated A(delta); Q2: [S][NT] accumulated Q^2."""
    m = np.asarray(modes, dtype=np.int64)
    S, NT = m.shape[0], m.shape[1]
    N = L ** d
    chi0 = np.zeros(NT)
    chik = np.zeros(NT)
    xi = np.full(NT, np.nan)
    for k in range(NT):
        A = [int(sum(int(m[s, k, j]) for s in range(S))) for j in range(L // 2 + 1)]
        q2 = int(sum(int(Q2[s][k]) for s in range(S)))
        chi0[k] = q2 / (S * n_meas * N)
        chik[k] = mode_power(A, L, 1) / (d * S * n_meas * N)
        if chik[k] > 0 and chi0[k] / chik[k] >= 1.0:
            xi[k] = math.sqrt(chi0[k] / chik[k] - 1.0) / (2.0 * math.sin(math.pi / L))
    return chi0, chik, xi


# --------------------------------------------------------------------------
# Gaussian couplings (gauss_oracle.c)
# --------------------------------------------------------------------------
GAUSS_UNIT = 2.0 ** -16


def gauss_energy(L: int, d: int, Jn: np.ndarray, spins: np.ndarray) -> int:
    """Eq. (1) in 2^-16 units for coupling units Jn [d][N]."""
    J = np.ascontiguousarray(Jn, dtype=np.int32)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().org_energy(L, d, _p(J), _p(s)))


def gauss_local_x(L: int, d: int, Jn: np.ndarray, spins: np.ndarray, i: int) -> int:
    J = np.ascontiguousarray(Jn, dtype=np.int32)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return int(lib().org_local_x(L, d, _p(J), _p(s), i))


def gauss_accept(r: int, b: float, u: int) -> int:
    """1 iff r < 2^32 exp(-b u 2^-16) (b > 0, u > 0 units of 2^-16)."""
    return int(lib().org_accept(int(r), float(b), int(u)))


class OracleGaussJob:
    """S samples x 2 replica sets x NT temperatures with Gaussian couplings
    given as integer units Jn [S][d][N] of 2^-16; energies in the same units."""

    def __init__(self, samples, replicas, L, dim, couplings_units, betas, seed, sample_keys=None):
        self.S, self.NT, self.L, self.d = int(samples), int(replicas), int(L), int(dim)
        self.N = nsites(self.L, self.d)
        self._J = np.ascontiguousarray(couplings_units, dtype=np.int32).reshape(self.S, self.d, self.N)
        self._b = np.ascontiguousarray(betas, dtype=np.float64)
        keys = None
        if sample_keys is not None:
            self._keys = np.ascontiguousarray(sample_keys, dtype=np.uint32)
            keys = _p(self._keys)
        self._h = lib().org_create(self.S, self.NT, self.L, self.d, _p(self._J), _p(self._b),
                                   C.c_uint64(seed), keys)
        if not self._h:
            raise ValueError("oracle rejected the job arguments")

    def close(self):
        if self._h:
            lib().org_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        lib().org_sweep(self._h, int(n))

    def exchange(self):
        lib().org_exchange(self._h)

    def houdayer(self, multi=False):
        lib().org_houdayer(self._h, int(bool(multi)))

    def measure(self):
        lib().org_measure(self._h)

    def mcs(self, n, houdayer=False, measure=False, multi=False):
        h = (2 if multi else 1) if houdayer else 0
        lib().org_mcs(self._h, int(n), h, int(bool(measure)))

    def set_measure_every(self, every):
        lib().org_set_measure_every(self._h, int(every))

    def spins(self):
        out = np.zeros((self.S, 2 * self.NT, self.N), np.int8)
        lib().org_get_spins(self._h, _p(out))
        return out

    def set_spins(self, spins):
        s = np.ascontiguousarray(spins, dtype=np.int8).reshape(self.S, 2 * self.NT, self.N)
        lib().org_set_spins(self._h, _p(s))

    def energies(self):
        out = np.zeros((self.S, 2 * self.NT), np.int64)
        lib().org_get_energies(self._h, _p(out))
        return out

    def maps(self):
        sot = np.zeros((self.S, 2, self.NT), np.int32)
        tos = np.zeros((self.S, 2, self.NT), np.int32)
        lib().org_get_maps(self._h, _p(sot), _p(tos))
        return sot, tos

    def counters(self):
        out = np.zeros(4, np.uint64)
        lib().org_get_counters(self._h, _p(out))
        return dict(t=int(out[0]), u=int(out[1]), v=int(out[2]), n_meas=int(out[3]))

    def moments(self):
        ST = (self.S, self.NT)
        E, Q, AQ, Q2 = (np.zeros(ST, np.int64) for _ in range(4))
        E2 = np.zeros(ST + (2,), np.uint64)
        Q4 = np.zeros(ST + (2,), np.uint64)
        lib().org_get_moments(self._h, _p(E), _p(E2), _p(Q), _p(AQ), _p(Q2), _p(Q4))
        return dict(E=E, E2=E2, Q=Q, AQ=AQ, Q2=Q2, Q4=Q4)

    def observables(self):
        ps = np.zeros((self.S, self.NT, 5), np.float64)
        dis = np.zeros((self.NT, 6), np.float64)
        n = np.zeros(1, np.int64)
        lib().org_observables(self._h, _p(ps), _p(dis), _p(n))
        return ps, dis, int(n[0])
