"""GPU parity of split samples: jobs whose 2 N_T configurations do not fit one
workgroup run each sample on several workgroups that meet once per step.
Spins, energies, maps, counters and integer moments must be bit-identical to
the CPU oracle, alone, inside a mixed batch, and under graph replay."""
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


def matches_oracle(pt, job, ref, what):
    assert (pt.pt_get_spins(job) == ref.spins()).all(), f"{what}: spins"
    assert (pt.pt_get_energies(job) == ref.energies()).all(), f"{what}: energies"
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a == b).all(), f"{what}: maps"
    assert pt.pt_get_counters(job) == ref.counters(), what
    gm, rm = pt.pt_get_moments(job), ref.moments()
    for k in rm:
        assert (np.asarray(gm[k]) == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), (what, k)
    if job.walk:
        for x, y in zip(pt.pt_get_walk(job), ref.walk()):
            assert (x == y).all(), f"{what}: replica walk"


SPLIT_CASES = [
    # (dim, L, samples, replicas, layout, expected parts)
    (3, 32, 2, 24, 0, 2),    # couplings in LDS, one replica set per part
    (3, 32, 1, 36, 1, 3),    # parts that straddle the two replica sets
    (3, 48, 1, 8, 0, 2),     # couplings read from global memory
    (3, 24, 1, 48, 1, 2),    # two fields per word
    (2, 64, 1, 160, 0, 2),   # 2D
    (3, 48, 1, 48, 1, 12),   # the largest served shape: 12 parts of 8
    (3, 64, 1, 4, 0, 2),     # the largest L: one row field per word, couplings in global memory
    (3, 64, 1, 2, 1, 1),     # one part holding all four configurations
]


def _job(pt, d, L, S, NT, layout, seed0, walk=False):
    J = W.couplings_pm_j(S, L, d, seed0 + L)
    b = W.geometric_betas(0.9, 2.0, NT) if d == 3 else W.geometric_betas(0.6, 5.0, NT)
    seed = 0xABCD_0000 + 31 * L + NT
    return (pt.pt_init(S, NT, L, d, J, b, seed, layout=layout, walk=walk),
            oracle.OracleJob(S, NT, L, d, J, b, seed))


@pytest.mark.parametrize("d,L,S,NT,layout,parts", SPLIT_CASES)
def test_split_matches_oracle(pt, d, L, S, NT, layout, parts):
    say(f"split case d={d} L={L} S={S} NT={NT} layout={layout}")
    job, ref = _job(pt, d, L, S, NT, layout, 300, walk=layout == 0)
    plan = pt.pt_get_plan(job, measure=True)
    assert plan["mode"] == 3 and plan["parts"] == parts, plan
    assert plan["lds_bytes"] <= 160 * 1024
    pt.pt_mcs(job, 2)
    ref.mcs(2)
    matches_oracle(pt, job, ref, "burn-in")
    pt.pt_mcs(job, 3, measure=True)
    ref.mcs(3, measure=True)
    matches_oracle(pt, job, ref, "measured")
    # a second measuring launch (an even step count) adds to the sums
    pt.pt_mcs(job, 2, measure=True)
    ref.mcs(2, measure=True)
    matches_oracle(pt, job, ref, "measured again")
    ps, dis, n = pt.pt_observables(job)
    rps, rdis, rn = ref.observables()
    assert n == rn == 5
    np.testing.assert_allclose(ps, rps, rtol=1e-12, atol=0)
    np.testing.assert_allclose(dis, rdis, rtol=1e-12, atol=0)
    pt.pt_destroy(job)


def test_3d_l64_per_step_kernels(pt):
    """The largest 3D lattice (L = 64, N = 262144) through the per-step kernels,
    Houdayer moves included (one workgroup per pair), against the oracle."""
    say("3D L=64 per-step sweep + Houdayer + exchange + measure")
    job, ref = _job(pt, 3, 64, 1, 3, 0, 410)
    assert pt.pt_get_plan(job, houdayer=True, measure=True)["mode"] == -1
    pt.pt_mcs(job, 2, houdayer=True, measure=True, plain=True)
    ref.mcs(2, houdayer=True, measure=True)
    matches_oracle(pt, job, ref, "per-step")
    pt.pt_mcs(job, 1, measure=True)
    ref.mcs(1, measure=True)
    matches_oracle(pt, job, ref, "split after per-step")
    ps, dis, n = pt.pt_observables(job)
    rps, rdis, rn = ref.observables()
    assert n == rn == 3
    np.testing.assert_allclose(dis, rdis, rtol=1e-12, atol=0)
    pt.pt_destroy(job)


def test_split_plain_steps_agree(pt):
    """The split plan and the per-step kernels interleave on one job."""
    say("split vs plain interleaved")
    job, ref = _job(pt, 3, 32, 1, 24, 0, 400)
    pt.pt_mcs(job, 2, measure=True)
    pt.pt_mcs(job, 1, measure=True, plain=True)
    pt.pt_mcs(job, 2)
    ref.mcs(3, measure=True)
    ref.mcs(2)
    matches_oracle(pt, job, ref, "interleaved")


@pytest.mark.parametrize("graph", [False, True])
def test_split_in_mixed_batch(pt, graph):
    """Split samples share one persistent launch with resident ones."""
    say(f"split in batch graph={graph}")
    shapes = [(32, 1, 24, 0), (8, 3, 4, 1), (24, 1, 48, 0), (16, 2, 6, 1), (12, 2, 3, 0)]
    jobs, refs = [], []
    for n, (L, S, NT, layout) in enumerate(shapes):
        j, r = _job(pt, 3, L, S, NT, layout, 500 + n)
        jobs.append(j)
        refs.append(r)
    assert pt.pt_get_plan(jobs[0], measure=True)["mode"] == 3
    assert pt.pt_get_plan(jobs[1], measure=True)["mode"] == 0
    batch = pt.pt_batch_create(jobs)
    for rnd in range(2):
        pt.pt_batch_run(batch, 2, measure=True, graph=graph)
        for r in refs:
            r.mcs(2, measure=True)
        for j, r in zip(jobs, refs):
            matches_oracle(pt, j, r, f"round {rnd}")
    pt.pt_batch_destroy(batch)



def test_plan_query_matches_jobs_and_byte_bound(pt):
    """pt_plan_query (host only) reports the plan a created job takes, and
    pt_job_bytes bounds what the job allocates."""
    import torch
    sizes = []

    def alloc(size, ctx):
        sizes.append(int(size))
        return torch.cuda.caching_allocator_alloc(int(size))

    def free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    pt.pt_set_allocator(alloc, free)
    try:
        for d, L, S, NT, layout in [(3, 16, 3, 8, 0), (3, 32, 2, 24, 1), (3, 48, 1, 48, 0),
                                    (2, 64, 2, 24, 0), (2, 12, 4, 5, 1), (3, 64, 1, 8, 0)]:
            say(f"plan/bytes d={d} L={L} S={S} NT={NT} layout={layout}")
            J = W.couplings_pm_j(S, L, d, 7)
            b = W.geometric_betas(0.9, 2.0, NT)
            sizes.clear()
            job = pt.pt_init(S, NT, L, d, J, b, 11, layout=layout)
            assert sum(sizes) <= pt.pt_job_bytes(S, NT, L, d, b, layout=layout)
            for hou, meas in [(False, False), (False, True), (True, True)]:
                assert pt.pt_get_plan(job, houdayer=hou, measure=meas) == \
                    pt.pt_plan_query(d, L, NT, houdayer=hou, measure=meas)
            pt.pt_destroy(job)
    finally:
        pt.pt_set_allocator(None, None)
