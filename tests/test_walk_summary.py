"""The library's host-side round-trip summary (pt_tunnel_summary) against the
oracle's, on seeded bins: same means and errors within 1e-13 relative, the
same equilibration decision.  Host code only: no GPU is touched."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def pt():
    from paper_2003_04621_amd import pt as _pt
    _pt.lib()
    return _pt


def _random_bins(rng, rows, passes, lengths):
    t = np.zeros((rows, 32, 3), np.uint64)
    for r in range(rows):
        for _ in range(int(rng.integers(0, 40))):
            end = int(rng.integers(1, passes + 1))
            n = int(rng.integers(lengths[0], lengths[1]))
            b = end.bit_length() - 1
            t[r, b] += np.array([1, n, n * n], np.uint64)
    return t


@pytest.mark.parametrize("seed", range(12))
def test_summary_matches_oracle(pt, seed):
    rng = np.random.default_rng(seed)
    passes = int(rng.integers(1, 5000))
    rows = int(rng.integers(1, 6))
    t = _random_bins(rng, rows, passes, (2, 400))
    got = pt.pt_tunnel_summary(t, passes)
    want = oracle.tunnel_summary(t, passes)
    for g, w in zip(got[:2], want[:2]):
        np.testing.assert_allclose(g, w, rtol=1e-13, atol=0, equal_nan=True)
    if np.isnan(want[2]):
        assert np.isnan(got[2])
    else:
        assert got[2] == pytest.approx(want[2], rel=1e-13)
    assert got[3] == want[3]


def test_summary_flag_cases(pt):
    def bins(values):
        t = np.zeros((32, 3), np.uint64)
        for b, lens in values.items():
            t[b] = [len(lens), sum(lens), sum(x * x for x in lens)]
        return t
    agree = bins({3: [4, 6], 4: [5, 7], 5: [4, 5, 6, 7]})
    for passes, want in [(62, 0), (63, 1), (126, 1), (127, 0)]:
        assert pt.pt_tunnel_summary(agree, passes)[3] == want
        assert oracle.tunnel_summary(agree, passes)[3] == want
    drift = bins({3: [4, 6], 4: [5, 7], 5: [20, 22, 21, 23]})
    assert pt.pt_tunnel_summary(drift, 63)[3] == 0


def test_summary_rejects_bad_arguments(pt):
    with pytest.raises(pt.PTError):
        pt.pt_tunnel_summary(np.zeros((0, 32, 3), np.uint64), 10)
