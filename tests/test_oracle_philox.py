"""Pins for the oracle's Philox4x32-10 (Salmon et al., SC'11; cited in Sec. 3).

The published known-answer vectors are not available here, so the generator
is pinned by (i) an independently written inverse of the Philox bijection,
which must recover every counter from the oracle's output, (ii) the Weyl key
increments derived from sqrt(5) and sqrt(3), and (iii) simple statistics.
Exact agreement with an external reference implementation is unpinned.
"""
import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
MASK = 0xFFFFFFFF


def _weyl():
    # (sqrt(5) - 1)/2 and sqrt(3) - 1 as 32-bit fractions
    w0 = int(((math.sqrt(5.0) - 1.0) / 2.0) * 2 ** 32)
    w1 = int((math.sqrt(3.0) - 1.0) * 2 ** 32)
    return w0, w1


def _inverse_philox(y, key, rounds=10):
    """Undo `rounds` Philox rounds.  Round r maps (x0,x1,x2,x3) with key
    (k0,k1) to (hi(M1 x2)^x1^k0, lo(M1 x2), hi(M0 x0)^x3^k1, lo(M0 x0)); since
    M0, M1 are odd the low products are invertible mod 2^32."""
    w0, w1 = _weyl()
    inv0, inv1 = pow(M0, -1, 2 ** 32), pow(M1, -1, 2 ** 32)
    y0, y1, y2, y3 = (int(v) for v in y)
    for r in reversed(range(rounds)):
        k0 = (int(key[0]) + r * w0) & MASK
        k1 = (int(key[1]) + r * w1) & MASK
        x2 = (y1 * inv1) & MASK
        x0 = (y3 * inv0) & MASK
        hi1 = (M1 * x2) >> 32
        hi0 = (M0 * x0) >> 32
        x1 = y0 ^ hi1 ^ k0
        x3 = y2 ^ hi0 ^ k1
        y0, y1, y2, y3 = x0, x1, x2, x3
    return [y0, y1, y2, y3]


def test_weyl_constants_from_irrationals():
    assert _weyl() == (0x9E3779B9, 0xBB67AE85)


def test_inverse_recovers_counter(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        out = orc.philox4x32_10(ctr, key)
        assert _inverse_philox(out, key) == [int(c) for c in ctr]
    # edge counters and keys
    for ctr, key in (([0, 0, 0, 0], [0, 0]), ([MASK] * 4, [MASK, MASK])):
        out = orc.philox4x32_10(ctr, key)
        assert _inverse_philox(out, key) == ctr


def test_stream_equals_single_calls(orc):
    key = [123, 456]
    st = orc.philox_stream(10, 2, 3, 4, key, 16)
    for i in range(16):
        assert (st[i] == orc.philox4x32_10([10 + i, 2, 3, 4], key)).all()


def test_bit_frequencies_and_byte_chi2(orc):
    n = 1 << 20                          # 2^22 words
    w = orc.philox_stream(0, 7, 1, (3 << 28) | 5, [0xDEADBEEF, 0x12345678], n).ravel()
    bits = np.unpackbits(w.view(np.uint8)).reshape(-1, 32).astype(np.int64)
    freq = bits.mean(axis=0)
    sigma = 0.5 / math.sqrt(w.size)
    assert np.all(np.abs(freq - 0.5) < 6 * sigma)
    counts = np.bincount(w.view(np.uint8), minlength=256).astype(np.float64)
    exp = w.size * 4 / 256
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    from exact import chi2_sf
    assert chi2_sf(chi2, 255) > 1e-4
    # top-bit fraction drives the initial spins and the couplings draw
    top = (w >> 31).mean()
    assert abs(top - 0.5) < 6 * sigma


def test_counter_words_distinct(orc):
    # changing any counter word or the key changes all four outputs
    base = orc.philox4x32_10([1, 2, 3, 4], [5, 6])
    for pos in range(4):
        c = [1, 2, 3, 4]
        c[pos] ^= 1
        assert np.all(orc.philox4x32_10(c, [5, 6]) != base)
    assert np.all(orc.philox4x32_10([1, 2, 3, 4], [5, 7]) != base)
