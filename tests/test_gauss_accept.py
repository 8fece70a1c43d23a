"""The exact acceptance decision of the Gaussian-coupling model (Sec. 2.1
couplings from a standard normal; Metropolis rule of Sec. 2.2, Eq. (5)):
r < 2^32 exp(-b u 2^-16) for a 32-bit word r, a double b > 0 and an integer
u > 0 of 2^-16 units.  The library's double-double evaluation, run on the
host, must agree with a 60-digit decimal evaluation at the boundary words
(r = ceil(t) - 1 accepts, r = ceil(t) rejects) and with the oracle; the
inputs also exercise the large-u and tiny-b ends of the range."""
import decimal

import numpy as np
import pytest

import oracle


def _ceil_threshold(b, u):
    """ceil(2^32 exp(-b u 2^-16)) from decimal arithmetic: r accepts iff r < it
    (t is never an integer: exp of a non-zero rational is irrational)."""
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        y = decimal.Decimal(b) * decimal.Decimal(int(u)) / decimal.Decimal(65536)
        t = (-y).exp() * decimal.Decimal(2 ** 32)
        return int(t.to_integral_value(rounding=decimal.ROUND_CEILING))


def boundary_cases(seed, n):
    """(b, u) pairs spread over the Metropolis and exchange ranges."""
    rng = np.random.default_rng(seed)
    cases = [(0.5, 2), (1.7, 65536), (5.0, 300000), (0.01, 12345678), (2.3, 40 * 65536),
             (1e-6, 3), (3.0, 1 << 33), (0.05, 1), (4.9, (1 << 24) - 1), (1e-3, 1 << 40)]
    for _ in range(n):
        cases.append((float(rng.uniform(0.01, 5.0)), int(rng.integers(1, 1 << 24))))
    for _ in range(n // 4):  # t close to 2^32 (tiny b u)
        cases.append((float(rng.uniform(1e-7, 1e-4)), int(rng.integers(1, 1 << 20))))
    for _ in range(n // 4):  # exchange energy differences
        cases.append((float(rng.uniform(1e-3, 0.2)), int(rng.integers(1 << 20, 1 << 34))))
    return cases


def boundary_words(cases):
    r, b, u, want = [], [], [], []
    for bb, uu in cases:
        n = _ceil_threshold(bb, uu)
        for rr in sorted({0, n - 2, n - 1, n, n + 1, 2 ** 32 - 1}):
            if 0 <= rr < 2 ** 32:
                r.append(rr)
                b.append(bb)
                u.append(uu)
                want.append(int(rr < n))
    return (np.array(r, np.uint32), np.array(b, np.float64), np.array(u, np.int64),
            np.array(want, np.int32))


@pytest.fixture(scope="module")
def ptlib():
    from paper_2003_04621_amd import pt
    pt.lib()
    return pt


def test_host_double_double_matches_decimal_and_oracle(ptlib):
    r, b, u, want = boundary_words(boundary_cases(3, 400))
    got = np.array([ptlib.pt_gauss_accept_host(int(x), float(y), int(z)) for x, y, z in zip(r, b, u)])
    assert (got == want).all(), np.flatnonzero(got != want)[:10]
    orc = np.array([oracle.gauss_accept(int(x), float(y), int(z)) for x, y, z in zip(r, b, u)])
    assert (orc == want).all()


def test_host_double_double_random_words(ptlib):
    rng = np.random.default_rng(11)
    for _ in range(3000):
        r = int(rng.integers(0, 2 ** 32))
        b = float(rng.uniform(0.01, 5.0))
        u = int(rng.integers(1, 1 << 24))
        assert ptlib.pt_gauss_accept_host(r, b, u) == oracle.gauss_accept(r, b, u), (r, b, u)


def test_host_rejects_bad_arguments(ptlib):
    from paper_2003_04621_amd.pt import PTError
    for b, u in [(0.0, 5), (-1.0, 5), (float("nan"), 5), (1.0, 0), (1.0, -3), (1.0, (1 << 52) + 1)]:
        with pytest.raises(PTError):
            ptlib.pt_gauss_accept_host(7, b, u)
