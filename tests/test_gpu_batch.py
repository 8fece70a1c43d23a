"""GPU tests of the batched form: jobs of mixed shape in one persistent launch
must reproduce, bit for bit, each job run alone and the CPU oracle."""
import os
import tempfile

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


def state(pt, job):
    return (pt.pt_get_spins(job), pt.pt_get_energies(job), *pt.pt_get_maps(job),
            tuple(sorted(pt.pt_get_counters(job).items())),
            {k: np.asarray(v).copy() for k, v in pt.pt_get_moments(job).items()},
            pt.pt_get_walk(job) if job.walk else ())


def same_state(a, b):
    for x, y in zip(a[:4], b[:4]):
        if not (np.asarray(x) == np.asarray(y)).all():
            return False
    if a[4] != b[4]:
        return False
    if not all((x == y).all() for x, y in zip(a[6], b[6])):
        return False
    return all((a[5][k] == b[5][k]).all() for k in a[5])


def matches_oracle(pt, job, ref):
    assert (pt.pt_get_spins(job) == ref.spins()).all()
    assert (pt.pt_get_energies(job) == ref.energies()).all()
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a == b).all()
    assert pt.pt_get_counters(job) == ref.counters()
    gm, rm = pt.pt_get_moments(job), ref.moments()
    for k in rm:
        assert (np.asarray(gm[k]) == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), k
    if job.walk:
        for x, y in zip(pt.pt_get_walk(job), ref.walk()):
            assert (x == y).all()


SHAPES_3D = [  # (L, samples, replicas, layout)
    (4, 2, 3, 0), (6, 1, 4, 1), (8, 3, 5, 0), (12, 2, 3, 1), (16, 1, 6, 0), (8, 1, 2, 1),
]


def make_jobs(pt, shapes, dim, seed0=10):
    jobs, refs = [], []
    for n, (L, S, NT, layout) in enumerate(shapes):
        J = W.couplings_pm_j(S, L, dim, seed0 + n)
        b = W.geometric_betas(0.5, 2.2, NT)
        jobs.append(pt.pt_init(S, NT, L, dim, J, b, 1000 + n, layout=layout))
        refs.append(oracle.OracleJob(S, NT, L, dim, J, b, 1000 + n))
    return jobs, refs


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle_3d(pt, graph):
    say(f"batch 3d graph={graph}")
    jobs, refs = make_jobs(pt, SHAPES_3D, 3)
    batch = pt.pt_batch_create(jobs)
    for rnd in range(3):
        pt.pt_batch_run(batch, 4, measure=True, graph=graph)
        for r in refs:
            r.mcs(4, measure=True)
        for j, r in zip(jobs, refs):
            matches_oracle(pt, j, r)
    pt.pt_batch_destroy(batch)


def test_batch_houdayer_2d(pt):
    shapes = [(16, 2, 4, 0), (8, 3, 3, 1), (64, 1, 3, 0), (6, 2, 2, 1)]
    jobs, refs = make_jobs(pt, shapes, 2, seed0=50)
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 5, houdayer=True, measure=True, graph=True)
    pt.pt_batch_run(batch, 5, houdayer=True, measure=True, graph=True)
    for r in refs:
        r.mcs(10, houdayer=True, measure=True)
    for j, r in zip(jobs, refs):
        matches_oracle(pt, j, r)


@pytest.mark.parametrize("cfg", [(1024, 1, 0), (512, 2, 1), (256, 1, 1), (256, 2, 0), (0, 2, 0),
                                 (768, 2, 0), (320, 2, 1), (448, 1, 0), (64, 2, 0)])
def test_batch_configs_agree(pt, cfg):
    say(f"batch config {cfg}")
    jobs, refs = make_jobs(pt, SHAPES_3D, 3, seed0=70)
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_set_config(batch, *cfg)
    pt.pt_batch_run(batch, 6)
    for r in refs:
        r.mcs(6)
    for j, r in zip(jobs, refs):
        matches_oracle(pt, j, r)


def test_launch_shape(pt):
    """The automatic grid: whole multiples of four wavefronts per workgroup,
    every workgroup resident at once, the largest size when items <= CUs,
    and for the 3D L=16 x 32-temperature workload shape at least two
    workgroups and 16 wavefronts per CU."""
    import torch
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"launch shape, {ncu} CUs")
    jobs, _ = make_jobs(pt, SHAPES_3D, 3, seed0=130)
    batch = pt.pt_batch_create(jobs)
    assert pt.pt_batch_launch_shape(batch) == {"blocks": 0, "threads": 0, "per_cu": 0}
    pt.pt_batch_run(batch, 1)
    shape = pt.pt_batch_launch_shape(batch)
    items = sum(j.S for j in jobs)
    assert items <= ncu and shape["threads"] == 1024 and shape["blocks"] == items
    for bad in (32, 100, 1088, -64):
        with pytest.raises(pt.PTError):
            pt.pt_batch_set_config(batch, bad, 2, 0)
    pt.pt_batch_set_config(batch, 320, 2, 0)
    pt.pt_batch_run(batch, 1)
    assert pt.pt_batch_launch_shape(batch)["threads"] == 320
    pt.pt_batch_destroy(batch)
    S = 4 * ncu
    J = W.couplings_pm_j(S, 16, 3, 5)
    big = pt.pt_init(S, 32, 16, 3, J, W.geometric_betas(0.9, 2.0, 32), 3)
    batch = pt.pt_batch_create([big])
    pt.pt_batch_run(batch, 1, measure=True)
    shape = pt.pt_batch_launch_shape(batch)
    say(f"3D L=16 x 32, {S} samples: {shape}")
    assert shape["threads"] % 256 == 0 and shape["per_cu"] >= 2
    assert shape["per_cu"] * shape["threads"] // 64 >= 16
    assert shape["blocks"] == min(S, ncu * shape["per_cu"])
    pt.pt_batch_destroy(batch)
    pt.pt_destroy(big)


def test_batch_equals_alone(pt):
    """The same job gives the same result alone and inside a mixed batch."""
    shapes = [(8, 2, 4, 0), (16, 1, 3, 1), (12, 3, 5, 0)]
    jobs, _ = make_jobs(pt, shapes, 3, seed0=90)
    alone, _ = make_jobs(pt, shapes, 3, seed0=90)
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 7, measure=True, graph=True)
    for a in alone:
        pt.pt_mcs(a, 7, measure=True)
    for j, a in zip(jobs, alone):
        assert same_state(state(pt, j), state(pt, a))


def test_tuner_restores_state_and_caches(pt):
    jobs, refs = make_jobs(pt, SHAPES_3D, 3, seed0=110)
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 2)
    for r in refs:
        r.mcs(2)
    before = [state(pt, j) for j in jobs]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        cfg = pt.pt_batch_tune(batch, 2, cache_path=path)
        assert cfg[0] in (256, 512, 768, 1024) and cfg[1] in (1, 2) and cfg[2] in (0, 1)
        assert os.path.exists(path) and "threads" in open(path).read()
        for j, s0 in zip(jobs, before):
            assert same_state(state(pt, j), s0)
        pt.pt_batch_set_config(batch, 256, 1, 1)
        assert pt.pt_batch_tune(batch, 2, cache_path=path) == cfg   # cache hit
    pt.pt_batch_run(batch, 3, graph=True)
    for r in refs:
        r.mcs(3)
    for j, r in zip(jobs, refs):
        matches_oracle(pt, j, r)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_runs_unplanned_jobs_per_step(pt, graph):
    """Houdayer moves on a 3D sample whose two sets do not fit one workgroup
    (L = 32, 4 temperatures: no fused plan) run through the per-step kernels
    beside the launch; every job matches the oracle, before and after steps
    without Houdayer moves (where that job is fused, a split sample)."""
    shapes = [(32, 1, 4, 0), (8, 2, 4, 1), (12, 1, 3, 0)]
    jobs, refs = make_jobs(pt, shapes, 3, seed0=130)
    assert pt.pt_get_plan(jobs[0], houdayer=True, measure=True)["mode"] == -1
    batch = pt.pt_batch_create(jobs)
    say(f"unplanned job in a batch, graph={graph}")
    pt.pt_batch_run(batch, 2, measure=True, graph=graph)
    for r in refs:
        r.mcs(2, measure=True)
    pt.pt_batch_run(batch, 3, houdayer=True, measure=True, graph=graph)
    for r in refs:
        r.mcs(3, houdayer=True, measure=True)
    pt.pt_batch_run(batch, 2, measure=True, graph=graph)
    for r in refs:
        r.mcs(2, measure=True)
    for j, r in zip(jobs, refs):
        matches_oracle(pt, j, r)


def test_batch_rejects_mixed_dims(pt):
    j2 = pt.pt_init(1, 2, 8, 2, W.couplings_pm_j(1, 8, 2, 1), np.array([1.0, 0.5]), 1)
    j3 = pt.pt_init(1, 2, 8, 3, W.couplings_pm_j(1, 8, 3, 1), np.array([1.0, 0.5]), 1)
    with pytest.raises(pt.PTError):
        pt.pt_batch_create([j2, j3])
    with pytest.raises(pt.PTError):
        pt.pt_batch_create([j2, j2])


def test_full_size_batched_mix_sampled(pt):
    """The batched workload at full size (2000 one-sample jobs, 400 each at
    L = 8, 12, 16, 24, 32, 24 temperatures) in one persistent launch replayed
    from a graph; two jobs of each L re-run by the oracle."""
    Ls, per_L, NT = [8, 12, 16, 24, 32], 400, 24
    b = W.geometric_betas(0.9, 2.0, NT)
    jobs, picks = [], []
    n = 0
    for L in Ls:
        for i in range(per_L):
            jobs.append(pt.pt_init(1, NT, L, 3, W.couplings_pm_j(1, L, 3, 1000 + n), b, 2000 + n))
            if i in (0, per_L - 1):
                picks.append(n)
            n += 1
    say(f"batched mix: {len(jobs)} jobs")
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 3, graph=True)
    pt.pt_batch_run(batch, 3, graph=True)
    for n in picks:
        L = Ls[n // per_L]
        ref = oracle.OracleJob(1, NT, L, 3, W.couplings_pm_j(1, L, 3, 1000 + n), b, 2000 + n)
        ref.mcs(6)
        say(f"check job {n} (L={L})")
        matches_oracle(pt, jobs[n], ref)
    pt.pt_batch_destroy(batch)
    for j in jobs:
        pt.pt_destroy(j)


def test_tuner_restores_walk_and_modes(pt):
    """Tuning trials run on a snapshot: the replica walk, its round-trip sums
    and the two-replica modes are restored with everything else, so a tuned
    batch of jobs keeping them continues bit-exactly (graph-replayed too)."""
    shapes = [(4, 2, 5, 0), (8, 1, 4, 1), (6, 2, 3, 0)]
    jobs, refs = [], []
    for n, (L, S, NT, layout) in enumerate(shapes):
        J = W.couplings_pm_j(S, L, 3, 300 + n)
        b = W.geometric_betas(1.6, 2.4, NT)
        jobs.append(pt.pt_init(S, NT, L, 3, J, b, 3000 + n, layout=layout, walk=True, modes=True))
        r = oracle.OracleJob(S, NT, L, 3, J, b, 3000 + n)
        r.enable_modes()
        refs.append(r)
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 30, measure=True)
    for r in refs:
        r.mcs(30, measure=True)
    before = [state(pt, j) for j in jobs]
    modes_before = [pt.pt_get_modes(j) for j in jobs]
    with tempfile.TemporaryDirectory() as d:
        pt.pt_batch_tune(batch, 7, measure=True, cache_path=os.path.join(d, "tune.jsonl"))
    for j, s0, m0 in zip(jobs, before, modes_before):
        assert same_state(state(pt, j), s0)
        assert (pt.pt_get_modes(j) == m0).all()
    pt.pt_batch_run(batch, 40, measure=True, graph=True)
    for r in refs:
        r.mcs(40, measure=True)
    for j, r in zip(jobs, refs):
        matches_oracle(pt, j, r)
        assert (pt.pt_get_modes(j) == r.modes()).all()
    assert sum(int(pt.pt_get_walk(j)[2][..., 0].sum()) for j in jobs) > 0
