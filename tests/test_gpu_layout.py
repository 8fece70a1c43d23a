"""GPU tests of moving a job between the two spin layouts (Sec. 2.2): the
conversion kernel keeps the configuration exactly, so later steps match the
oracle bit for bit, alone, in a batch whose work list and graph were built
before the move, and under the autotuner's layout axis."""
import json
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


def pm_job(pt, L, S, NT, dim, layout, seed):
    J = W.couplings_pm_j(S, L, dim, seed)
    b = W.geometric_betas(0.5, 2.2, NT)
    return (pt.pt_init(S, NT, L, dim, J, b, 500 + seed, layout=layout),
            oracle.OracleJob(S, NT, L, dim, J, b, 500 + seed))


def same_as_oracle(pt, job, ref, what):
    assert (pt.pt_get_spins(job) == ref.spins()).all(), f"{what}: spins"
    assert (pt.pt_get_energies(job) == ref.energies()).all(), f"{what}: energies"
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a == b).all(), f"{what}: maps"
    assert pt.pt_get_counters(job) == ref.counters(), what
    gm, rm = pt.pt_get_moments(job), ref.moments()
    for k in rm:
        assert (np.asarray(gm[k]) == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), \
            f"{what}: {k}"


# (dim, L, samples, replicas): several words per colour, ragged word counts
# (L = 6, 12, 10) and a lattice of one word row
SHAPES = [(3, 6, 2, 3), (3, 12, 1, 4), (3, 16, 2, 2), (2, 10, 3, 3), (2, 64, 1, 2), (2, 4, 2, 2)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "d%d_L%d_S%d_NT%d" % s)
@pytest.mark.parametrize("start", [0, 1])
def test_set_layout_keeps_state_and_steps(pt, shape, start):
    d, L, S, NT = shape
    say(f"layout move: d={d} L={L} S={S} NT={NT} from layout {start}")
    job, ref = pm_job(pt, L, S, NT, d, start, 7 * L + NT + start)
    pt.pt_mcs(job, 3, houdayer=True, measure=True)
    ref.mcs(3, houdayer=True, measure=True)
    spins = pt.pt_get_spins(job)
    pt.pt_set_layout(job, 1 - start)
    assert pt.pt_get_layout(job) == 1 - start
    assert (pt.pt_get_spins(job) == spins).all()
    same_as_oracle(pt, job, ref, "after the move")
    pt.pt_mcs(job, 4, houdayer=True, measure=True)
    ref.mcs(4, houdayer=True, measure=True)
    same_as_oracle(pt, job, ref, "steps after the move")
    pt.pt_set_layout(job, start)
    pt.pt_set_layout(job, start)  # already there: no change
    pt.pt_mcs(job, 2, plain=True, measure=True)
    ref.mcs(2, measure=True)
    same_as_oracle(pt, job, ref, "per-step kernels after the move back")


@pytest.mark.parametrize("start", [0, 1])
def test_set_layout_split_sample(pt, start):
    """A sample split over two workgroups (3D L = 32, 24 temperatures): fused
    measuring steps before and after the move."""
    job, ref = pm_job(pt, 32, 1, 24, 3, start, 91 + start)
    assert pt.pt_get_plan(job, measure=True)["mode"] == 3
    pt.pt_mcs(job, 3, measure=True)
    ref.mcs(3, measure=True)
    pt.pt_set_layout(job, 1 - start)
    pt.pt_mcs(job, 4, measure=True)
    ref.mcs(4, measure=True)
    same_as_oracle(pt, job, ref, "split sample after the move")


def test_set_layout_gauss(pt):
    d, L, S, NT = 2, 12, 2, 3
    Jf = W.couplings_gauss(S, L, d, 41)
    b = W.geometric_betas(0.2, 1.6, NT)
    job = pt.pt_init_gauss(S, NT, L, d, Jf, b, 77, layout=0)
    ref = oracle.OracleGaussJob(S, NT, L, d, W.gauss_units(Jf), b, 77)
    pt.pt_mcs(job, 3, houdayer=True, measure=True)
    ref.mcs(3, houdayer=True, measure=True)
    pt.pt_set_layout(job, 1)
    pt.pt_mcs(job, 3, houdayer=True, measure=True)
    ref.mcs(3, houdayer=True, measure=True)
    assert (pt.pt_get_spins(job) == ref.spins()).all()
    assert (pt.pt_get_energies64(job) == ref.energies()).all()
    assert pt.pt_get_counters(job) == ref.counters()


def test_set_layout_rejects_unknown(pt):
    job, _ = pm_job(pt, 4, 1, 2, 2, 0, 3)
    with pytest.raises(pt.PTError):
        pt.pt_set_layout(job, 2)
    assert pt.pt_get_layout(job) == 0


@pytest.mark.parametrize("graph", [False, True])
def test_batch_rebuilds_after_move(pt, graph):
    shapes = [(8, 2, 4, 0), (12, 1, 3, 1), (6, 3, 2, 0)]
    pairs = [pm_job(pt, L, S, NT, 3, lay, 20 + n) for n, (L, S, NT, lay) in enumerate(shapes)]
    jobs, refs = [p[0] for p in pairs], [p[1] for p in pairs]
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 3, houdayer=True, measure=True, graph=graph)
    for r in refs:
        r.mcs(3, houdayer=True, measure=True)
    pt.pt_set_layout(jobs[0], 1)
    pt.pt_set_layout(jobs[1], 0)
    pt.pt_batch_run(batch, 3, houdayer=True, measure=True, graph=graph)
    for r in refs:
        r.mcs(3, houdayer=True, measure=True)
    for n, (j, r) in enumerate(zip(jobs, refs)):
        same_as_oracle(pt, j, r, f"job {n}")


def test_tuner_layout_axis(pt):
    shapes = [(8, 2, 4, 0), (16, 1, 3, 1), (12, 2, 2, 0)]
    pairs = [pm_job(pt, L, S, NT, 3, lay, 60 + n) for n, (L, S, NT, lay) in enumerate(shapes)]
    jobs, refs = [p[0] for p in pairs], [p[1] for p in pairs]
    batch = pt.pt_batch_create(jobs)
    pt.pt_batch_run(batch, 2, measure=True)
    for r in refs:
        r.mcs(2, measure=True)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        cfg = pt.pt_batch_tune(batch, 2, measure=True, cache_path=path, layouts=True)
        lines = [json.loads(x) for x in open(path)]
        assert len(lines) == 1 and lines[0]["layout"] in (0, 1)
        chosen = lines[0]["layout"]
        say(f"tuned: {cfg}, layout {chosen}")
        assert all(pt.pt_get_layout(j) == chosen == j.layout for j in jobs)
        for n, (j, r) in enumerate(zip(jobs, refs)):
            same_as_oracle(pt, j, r, f"restored job {n}")
        # a cache hit for the same starting layouts applies the cached layout
        for j, (_, _, _, lay) in zip(jobs, shapes):
            pt.pt_set_layout(j, lay)
        pt.pt_batch_set_config(batch, 256, 1, 1)
        assert pt.pt_batch_tune(batch, 2, measure=True, cache_path=path, layouts=True) == cfg
        assert all(pt.pt_get_layout(j) == chosen for j in jobs)
        assert len(open(path).readlines()) == 1
    pt.pt_batch_run(batch, 3, measure=True, graph=True)
    for r in refs:
        r.mcs(3, measure=True)
    for n, (j, r) in enumerate(zip(jobs, refs)):
        same_as_oracle(pt, j, r, f"job {n} after tuning")


def test_checkpoint_restores_only_into_its_layout(pt):
    """A checkpoint names its layout: refused after a move, accepted after the
    move back, and the restored job continues as the oracle does."""
    job, ref = pm_job(pt, 8, 2, 3, 3, 0, 5)
    pt.pt_mcs(job, 3, measure=True)
    ref.mcs(3, measure=True)
    ck = pt.pt_get_state(job)
    pt.pt_mcs(job, 2, measure=True)
    pt.pt_set_layout(job, 1)
    with pytest.raises(pt.PTError):
        pt.pt_set_state(job, ck)
    pt.pt_set_layout(job, 0)
    pt.pt_set_state(job, ck)
    same_as_oracle(pt, job, ref, "restored")
    pt.pt_mcs(job, 2, measure=True)
    ref.mcs(2, measure=True)
    same_as_oracle(pt, job, ref, "after the restore")
