"""GPU parity of the multi-cluster Houdayer move (Sec. 3 / Sec. 5 variant):
the per-pair kernel (pt_houdayer_multi, PT_MCS_PLAIN), the fused step, the
batched and the served forms must be bit-identical to the CPU oracle."""
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


def make(pt, d, L, S, NT, layout, seed0):
    J = W.couplings_pm_j(S, L, d, seed0)
    b = W.geometric_betas(0.9, 2.0, NT) if d == 3 else W.geometric_betas(0.3, 1.6, NT)
    seed = 0x5EED_0000 + 97 * L + NT + seed0
    return (pt.pt_init(S, NT, L, d, J, b, seed, layout=layout),
            oracle.OracleJob(S, NT, L, d, J, b, seed), J, b, seed)


SHAPES = [  # (dim, L, samples, replicas, layout)
    (2, 64, 2, 6, 0),
    (2, 16, 3, 5, 1),
    (2, 6, 4, 3, 0),
    (3, 8, 3, 6, 1),
    (3, 16, 2, 8, 0),
    (3, 6, 2, 4, 1),
    (3, 24, 1, 4, 0),
]


@pytest.mark.parametrize("d,L,S,NT,layout", SHAPES)
def test_multicluster_fused_and_per_step_match_oracle(pt, d, L, S, NT, layout):
    say(f"multi-cluster d={d} L={L} S={S} NT={NT} layout={layout}")
    job, ref, *_ = make(pt, d, L, S, NT, layout, 11 * L + d)
    assert pt.pt_get_plan(job, houdayer=True, measure=True, multi=True)["mode"] == 1
    pt.pt_mcs(job, 3, houdayer=True, multi=True, plain=True)
    ref.mcs(3, houdayer=True, multi=True)
    matches_oracle(pt, job, ref, "per-step")
    pt.pt_mcs(job, 4, houdayer=True, multi=True, measure=True)
    ref.mcs(4, houdayer=True, multi=True, measure=True)
    matches_oracle(pt, job, ref, "fused")
    # single- and multi-cluster passes share the pass counter
    pt.pt_mcs(job, 2, houdayer=True, measure=True)
    ref.mcs(2, houdayer=True, measure=True)
    pt.pt_houdayer_multi(job)
    ref.houdayer(multi=True)
    matches_oracle(pt, job, ref, "mixed")
    _, dis, n = pt.pt_observables(job)
    _, rdis, rn = ref.observables()
    assert n == rn == 6
    np.testing.assert_allclose(dis, rdis, rtol=1e-12, atol=0)
    pt.pt_destroy(job)


def test_multicluster_largest_lattice_per_step(pt):
    """3D L = 32 (32768 sites, the most the labels name): the per-pair kernel;
    the fused plan does not hold such a pair."""
    say("multi-cluster 3D L=32 per-step")
    job, ref, *_ = make(pt, 3, 32, 1, 3, 0, 5)
    assert pt.pt_get_plan(job, houdayer=True, multi=True)["mode"] == -1
    pt.pt_mcs(job, 3, houdayer=True, multi=True, measure=True)
    ref.mcs(3, houdayer=True, multi=True, measure=True)
    matches_oracle(pt, job, ref, "L=32")
    big, *_ = make(pt, 3, 34, 1, 2, 0, 6)
    with pytest.raises(pt.PTError) as e:
        pt.pt_mcs(big, 1, houdayer=True, multi=True)
    assert e.value.code == pt.PT_EINVAL
    with pytest.raises(pt.PTError):
        pt.pt_mcs(job, 1, multi=True)       # needs houdayer


@pytest.mark.parametrize("d,L", [(2, 64), (3, 16), (2, 10)])
def test_multicluster_edge_states(pt, d, L):
    """Pairs with no q = -1 site, with every site q = -1 (one cluster covering
    the lattice: full rows and full overlaps), and with whole rows alternating."""
    S, NT = 1, 4
    say(f"multi-cluster edge states d={d} L={L}")
    for layout in (0, 1):
        job, ref, *_ = make(pt, d, L, S, NT, layout, 70 + L)
        sp = pt.pt_get_spins(job)
        N = L ** d
        sp[0, NT + 0] = sp[0, 0]                 # k = 0: identical replicas
        sp[0, NT + 1] = -sp[0, 1]                # k = 1: every site q = -1
        rows = (np.arange(N) // L) % 2 == 0      # k = 2: every other row q = -1
        sp[0, NT + 2] = np.where(rows, -sp[0, 2], sp[0, 2])
        pt.pt_set_spins(job, sp)
        ref.set_spins(sp)
        for rep in range(3):
            pt.pt_houdayer_multi(job)
            ref.houdayer(multi=True)
            matches_oracle(pt, job, ref, f"edge per-step {rep}")
        pt.pt_set_spins(job, sp)
        ref.set_spins(sp)
        # the fused form on the same states (sweep first: the states change a little)
        pt.pt_mcs(job, 2, houdayer=True, multi=True)
        ref.mcs(2, houdayer=True, multi=True)
        matches_oracle(pt, job, ref, "edge fused")
        pt.pt_destroy(job)


def test_multicluster_batched_and_graph(pt):
    """Jobs of mixed shape with multi-cluster moves in one persistent launch,
    replayed from a captured graph."""
    shapes = [(3, 8, 2, 6, 0), (3, 16, 1, 8, 1), (3, 12, 2, 4, 0)]
    jobs, refs = [], []
    for n, (d, L, S, NT, layout) in enumerate(shapes):
        j, r, *_ = make(pt, d, L, S, NT, layout, 200 + n)
        jobs.append(j)
        refs.append(r)
    batch = pt.pt_batch_create(jobs)
    for rnd in range(3):
        say(f"multi-cluster batch round {rnd}")
        pt.pt_batch_run(batch, 2, houdayer=True, measure=True, graph=rnd > 0, multi=True)
        for r in refs:
            r.mcs(2, houdayer=True, measure=True, multi=True)
        for j, r in zip(jobs, refs):
            matches_oracle(pt, j, r, f"batch round {rnd}")
    pt.pt_batch_destroy(batch)


def test_multicluster_served_matches_oracle(pt):
    import time
    srv = pt.pt_server_start(1 << 28, steps_per_round=3)
    specs = [(2, 32, 4, 2, 9, 3), (3, 8, 5, 1, 8, 2), (3, 32, 2, 1, 5, 1)]
    tickets = {}
    inputs = {}
    for n, (d, L, NT, S, sweeps, burn) in enumerate(specs):
        J = W.couplings_pm_j(S, L, d, 300 + n)
        b = W.geometric_betas(0.5, 2.0, NT)
        inputs[n] = (J, b, 400 + n)
        tickets[n] = pt.pt_server_submit(srv, d, L, NT, S, b, J, 400 + n, sweeps, burn,
                                         houdayer=True, multi=True)
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for n, t in tickets.items():
            if n not in out:
                r = pt.pt_server_poll(srv, t)
                if r is not None:
                    out[n] = r
        assert time.time() - t0 < 120
        time.sleep(0.01)
    pt.pt_server_stop(srv)
    for n, (d, L, NT, S, sweeps, burn) in enumerate(specs):
        J, b, seed = inputs[n]
        ref = oracle.OracleJob(S, NT, L, d, J, b, seed)
        ref.mcs(burn, houdayer=True, multi=True)
        ref.mcs(sweeps - burn, houdayer=True, multi=True, measure=True)
        _, rdis, rn = ref.observables()
        assert out[n]["status"] == 0 and out[n]["n_meas"] == rn
        np.testing.assert_allclose(out[n]["disorder"], rdis, rtol=1e-12, atol=0)


def test_full_size_2d_l64_multicluster_sampled(pt):
    """The benchmark's multi-cluster workload at full size (2D L = 64, 500
    samples x 2 x 24 temperatures, fused launch), a few Monte Carlo steps with
    multi-cluster moves and measurements; sampled samples re-run by the
    oracle under their own sample keys, and the run diagnostics of a sampled
    job with PT_TRACK_STATS (per-step kernels) against the oracle's."""
    wl = W.workload("2d_l64")
    say(f"case {wl.name} multi-cluster S={wl.samples} NT={wl.replicas} L={wl.L}")
    J = wl.couplings()
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed)
    assert pt.pt_get_plan(job, houdayer=True, measure=True, multi=True)["mode"] == 1
    pt.pt_mcs(job, 5, houdayer=True, measure=True, multi=True)
    picks = [0, 211, wl.samples - 1]
    ref = oracle.OracleJob(len(picks), wl.replicas, wl.L, wl.dim, J[picks], wl.betas, wl.seed,
                           sample_keys=picks)
    ref.mcs(5, houdayer=True, measure=True, multi=True)
    assert (pt.pt_get_spins(job)[picks] == ref.spins()).all()
    assert (pt.pt_get_energies(job)[picks] == ref.energies()).all()
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a[picks] == b).all()
    mom, rmom = pt.pt_get_moments(job), ref.moments()
    for key in rmom:
        assert (np.asarray(mom[key])[picks] == np.asarray(rmom[key])).all(), key
    pt.pt_destroy(job)
    # the same first steps of the sampled samples with the diagnostics kept
    sj = pt.pt_init(len(picks), wl.replicas, wl.L, wl.dim, J[picks], wl.betas, wl.seed, stats=True)
    ref2 = oracle.OracleJob(len(picks), wl.replicas, wl.L, wl.dim, J[picks], wl.betas, wl.seed)
    pt.pt_mcs(sj, 3, houdayer=True, measure=True, multi=True)
    ref2.mcs(3, houdayer=True, measure=True, multi=True)
    assert (pt.pt_get_stats(sj) == ref2.stats()).all()
    pt.pt_destroy(sj)
