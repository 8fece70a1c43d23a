"""GPU parity of measurements at intervals (Sec. 3): a step measures when its
1-based sweep number is a multiple of the job's interval, on every path and
across launch boundaries, with the interval changed mid-run; against the
oracle, every bit of the moments, the modes and the counters."""
import numpy as np
import pytest

import oracle
from paper_2003_04621_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_04621_amd import pt as _pt
    _pt.lib()
    return _pt


def say(*a):
    print(*a, flush=True)


CASES = [
    # (name, dim, L, samples, replicas, houdayer, how)
    ("fused 3D L=8", 3, 8, 2, 4, False, "mcs"),
    ("fused 2D L=16 Houdayer", 2, 16, 2, 4, True, "mcs"),
    ("per-step 3D L=6", 3, 6, 2, 3, False, "plain"),
    ("split 3D L=32", 3, 32, 1, 24, False, "mcs"),
    ("batch 3D L=8", 3, 8, 2, 4, False, "batch"),
]


@pytest.mark.parametrize("name,d,L,S,NT,hou,how", CASES)
def test_interval_vs_oracle(pt, name, d, L, S, NT, hou, how):
    say(f"interval case {name}")
    J = W.couplings_pm_j(S, L, d, 70 + L)
    b = W.geometric_betas(0.8, 2.0, NT)
    job = pt.pt_init(S, NT, L, d, J, b, 91, modes=True)
    ref = oracle.OracleJob(S, NT, L, d, J, b, 91)
    ref.enable_modes()
    batch = pt.pt_batch_create([job]) if how == "batch" else None
    big = L >= 32
    for every, chunks in ((3, (4, 7) if big else (10, 11)), (5, (6,) if big else (12,)),
                          (1, (2,))):
        pt.pt_set_measure_interval(job, every)
        ref.set_measure_every(every)
        for n in chunks:
            if batch is not None:
                pt.pt_batch_run(batch, n, houdayer=hou, measure=True)
            else:
                pt.pt_mcs(job, n, houdayer=hou, measure=True, plain=how == "plain")
            ref.mcs(n, houdayer=hou, measure=True)
        assert pt.pt_get_counters(job) == ref.counters(), (name, every)
        gm, rm = pt.pt_get_moments(job), ref.moments()
        for k in rm:
            assert (np.asarray(gm[k]) == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), k
        assert (pt.pt_get_modes(job) == ref.modes()).all()
    if batch is not None:
        pt.pt_batch_destroy(batch)


def test_interval_rejects_zero(pt):
    job = pt.pt_init(1, 2, 4, 3, W.couplings_pm_j(1, 4, 3, 1), W.geometric_betas(1, 2, 2), 1)
    with pytest.raises(pt.PTError):
        pt.pt_set_measure_interval(job, 0)
