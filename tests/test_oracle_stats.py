"""Pins for the oracle's run diagnostics (acceptance rates, Sec. 2.3; the
spread of cluster sizes, Sec. 3): every counter is recounted here from the
states before and after each step, not from the oracle's own bookkeeping."""
import numpy as np
import pytest

from paper_2003_04621_amd import workloads as W


def _accepted_swaps(m0, m1):
    """Decisions of one ascending exchange pass over one ladder, from the maps
    before (m0) and after (m1): after step k position k is never touched
    again, so step k swapped iff position k did not already hold its final
    configuration."""
    cur = list(m0)
    acc = np.zeros(len(m0), np.int64)
    for k in range(len(m0) - 1):
        if cur[k] != m1[k]:
            cur[k], cur[k + 1] = cur[k + 1], cur[k]
            acc[k] = 1
    assert cur == list(m1)
    return acc


@pytest.mark.parametrize("L,d,multi", [(6, 2, False), (4, 3, True), (5, 2, True)])
def test_stats_recounted_step_by_step(orc, L, d, multi):
    S, NT = 3, 5
    job = orc.OracleJob(S, NT, L, d, W.couplings_pm_j(S, L, d, 3 + L),
                        W.geometric_betas(0.4, 2.0, NT), 12)
    want = np.zeros((S, NT, 24), np.int64)
    for step in range(12):
        # sweep: flipped sites of each configuration, at its temperature
        sp0 = job.spins()
        _, tos = job.maps()
        job.sweep(1)
        sp1 = job.spins()
        for s in range(S):
            for r in range(2 * NT):
                k = tos[s, r // NT, r % NT]
                want[s, k, 0] += int(np.sum(sp0[s, r] != sp1[s, r]))
        # Houdayer: sites exchanged in each pair
        sot, _ = job.maps()
        sp0 = job.spins()
        job.houdayer(multi=multi)
        sp1 = job.spins()
        for s in range(S):
            for k in range(NT):
                a = sot[s, 0, k]
                n = int(np.sum(sp0[s, a] != sp1[s, a]))
                if n:
                    want[s, k, 2] += 1
                    want[s, k, 3] += n
                    want[s, k, 4 + int(np.floor(np.log2(n)))] += 1
        # exchange: decisions reconstructed from the maps
        m0, _ = job.maps()
        job.exchange()
        m1, _ = job.maps()
        for s in range(S):
            for c in range(2):
                want[s, :, 1] += _accepted_swaps(m0[s, c], m1[s, c])
    assert (job.stats() == want).all()
    assert want[..., 0].sum() > 0 and want[..., 1].sum() > 0 and want[..., 2].sum() > 0
