"""GPU parity: the gfx950 library against the CPU oracle on the same seeded
inputs.  Spins, integer energies, temperature maps, counters and integer
moments must be bit-identical; FP64 observables agree within 1e-12
relative (same integer numerators, one division each)."""
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


def compare(pt, job, ref, what=""):
    gs, rs = pt.pt_get_spins(job), ref.spins()
    assert (gs == rs).all(), f"{what}: spins differ at {np.argwhere(gs != rs)[:5]}"
    ge, re_ = pt.pt_get_energies(job), ref.energies()
    assert (ge == re_).all(), f"{what}: energies differ {ge} vs {re_}"
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a == b).all(), f"{what}: maps differ"
    assert pt.pt_get_counters(job) == ref.counters(), what
    gm, rm = pt.pt_get_moments(job), ref.moments()
    for k in rm:
        assert (np.asarray(gm[k]) == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), (what, k)
    if job.walk:
        for x, y, name in zip(pt.pt_get_walk(job), ref.walk(), ("labels", "begins", "trips")):
            assert (x == y).all(), f"{what}: replica walk {name} differ"


def compare_observables(pt, job, ref):
    ps, dis, n = pt.pt_observables(job)
    rps, rdis, rn = ref.observables()
    assert n == rn
    np.testing.assert_allclose(ps, rps, rtol=1e-12, atol=0)
    np.testing.assert_allclose(dis, rdis, rtol=1e-12, atol=0)


CASES = [
    # (dim, L, samples, replicas, layout)
    (2, 4, 2, 2, 0), (2, 6, 3, 3, 0), (2, 8, 2, 4, 1), (2, 10, 2, 3, 1), (2, 64, 2, 3, 0),
    (3, 4, 2, 3, 0), (3, 6, 2, 2, 1), (3, 8, 3, 5, 0), (3, 12, 2, 3, 0), (3, 12, 2, 3, 1),
    (3, 16, 2, 4, 0), (3, 16, 1, 2, 1), (3, 24, 1, 2, 0),
]


@pytest.mark.parametrize("d,L,S,NT,layout", CASES)
def test_mcs_parity(pt, d, L, S, NT, layout):
    walk = CASES.index((d, L, S, NT, layout)) % 2 == 1  # every other case keeps the walk
    say(f"case d={d} L={L} S={S} NT={NT} layout={layout} walk={walk}")
    J = W.couplings_pm_j(S, L, d, 100 + L)
    betas = W.geometric_betas(0.5, 2.5, NT)
    seed = 0x1234_5678_9ABC + L
    job = pt.pt_init(S, NT, L, d, J, betas, seed, layout=layout, walk=walk)
    ref = oracle.OracleJob(S, NT, L, d, J, betas, seed)
    compare(pt, job, ref, "init")
    pt.pt_sweep(job, 1)
    ref.sweep(1)
    compare(pt, job, ref, "sweep 1")
    pt.pt_sweep(job, 3)
    ref.sweep(3)
    compare(pt, job, ref, "sweep 3")
    pt.pt_exchange(job)
    ref.exchange()
    compare(pt, job, ref, "exchange")
    pt.pt_houdayer(job)
    ref.houdayer()
    compare(pt, job, ref, "houdayer")
    pt.pt_mcs(job, 6, houdayer=True, measure=True)
    ref.mcs(6, houdayer=True, measure=True)
    compare(pt, job, ref, "mcs")
    compare_observables(pt, job, ref)
    pt.pt_destroy(job)


def test_layouts_agree(pt):
    d, L, S, NT = 3, 8, 2, 4
    J = W.couplings_pm_j(S, L, d, 7)
    b = W.geometric_betas(0.9, 2.0, NT)
    a = pt.pt_init(S, NT, L, d, J, b, 99, layout=0)
    p = pt.pt_init(S, NT, L, d, J, b, 99, layout=1)
    for job in (a, p):
        pt.pt_mcs(job, 20, houdayer=True, measure=True)
    assert (pt.pt_get_spins(a) == pt.pt_get_spins(p)).all()
    assert (pt.pt_get_energies(a) == pt.pt_get_energies(p)).all()


def test_zero_sweeps_and_bad_n(pt):
    J = W.couplings_pm_j(1, 4, 2, 1)
    job = pt.pt_init(1, 2, 4, 2, J, np.array([1.0, 0.5]), 3)
    s0 = pt.pt_get_spins(job)
    pt.pt_sweep(job, 0)
    assert (pt.pt_get_spins(job) == s0).all() and pt.pt_get_counters(job)["t"] == 0
    with pytest.raises(pt.PTError):
        pt.pt_sweep(job, -1)
    with pytest.raises(pt.PTError):
        pt.pt_set_spins(job, np.zeros((1, 4, 16), np.int8))


def test_houdayer_identical_replicas_is_noop(pt):
    d, L, S, NT = 2, 8, 2, 3
    J = W.couplings_pm_j(S, L, d, 5)
    b = W.geometric_betas(0.5, 1.5, NT)
    job = pt.pt_init(S, NT, L, d, J, b, 17)
    sp = pt.pt_get_spins(job)
    sp[:, NT:, :] = sp[:, :NT, :]
    pt.pt_set_spins(job, sp)
    pt.pt_houdayer(job)
    assert (pt.pt_get_spins(job) == sp).all()
    assert pt.pt_get_counters(job)["v"] == 1


def test_zero_temperature_quench(pt):
    d, L, S = 3, 8, 2
    J = W.couplings_pm_j(S, L, d, 3)
    job = pt.pt_init(S, 2, L, d, J, np.array([60.0, 50.0]), 5)
    ref = oracle.OracleJob(S, 2, L, d, J, np.array([60.0, 50.0]), 5)
    prev = pt.pt_get_energies(job)
    for _ in range(10):
        pt.pt_sweep(job, 1)
        ref.sweep(1)
        E = pt.pt_get_energies(job)
        assert (E <= prev).all()
        prev = E
    compare(pt, job, ref, "quench")


def test_gauge_invariance_on_gpu(pt):
    d, L, S, NT = 3, 8, 2, 3
    N = L ** d
    J = W.couplings_pm_j(S, L, d, 8)
    rng = np.random.default_rng(3)
    eps = rng.choice(np.array([-1, 1], np.int8), size=(S, N))
    idx = np.arange(N).reshape((L,) * d)
    Jg = np.empty_like(J)
    for mu in range(d):
        nbr = np.roll(idx, -1, axis=d - 1 - mu).ravel()
        Jg[:, mu, :] = eps * eps[:, nbr] * J[:, mu, :]
    b = W.geometric_betas(0.8, 2.0, NT)
    a = pt.pt_init(S, NT, L, d, J, b, 42)
    g = pt.pt_init(S, NT, L, d, Jg, b, 42, layout=1)
    pt.pt_set_spins(g, pt.pt_get_spins(a) * eps[:, None, :])
    for job in (a, g):
        pt.pt_mcs(job, 15, houdayer=True, measure=True)
    assert (pt.pt_get_spins(g) == pt.pt_get_spins(a) * eps[:, None, :]).all()
    assert (pt.pt_get_energies(g) == pt.pt_get_energies(a)).all()
    for m1, m2 in zip(pt.pt_get_maps(g), pt.pt_get_maps(a)):
        assert (m1 == m2).all()


def test_checkpoint_restore_is_bit_exact(pt):
    d, L, S, NT = 2, 16, 3, 4
    J = W.couplings_pm_j(S, L, d, 21)
    b = W.geometric_betas(0.4, 1.6, NT)
    a = pt.pt_init(S, NT, L, d, J, b, 8)
    pt.pt_mcs(a, 10, houdayer=True, measure=True)
    state = pt.pt_get_state(a)
    pt.pt_mcs(a, 10, houdayer=True, measure=True)
    pt.pt_destroy(a)
    b2 = pt.pt_init(S, NT, L, d, J, b, 8)
    pt.pt_set_state(b2, state)
    pt.pt_mcs(b2, 10, houdayer=True, measure=True)
    ref = oracle.OracleJob(S, NT, L, d, J, b, 8)
    ref.mcs(20, houdayer=True, measure=True)
    compare(pt, b2, ref, "restored")


def test_full_size_3d_l16_sampled(pt):
    """1000 samples x 32 temperatures, 3D L=16, in the benchmark's launch
    configuration; three samples re-run by the oracle."""
    wl = W.workload("3d_l16")
    say(f"case {wl.name} S={wl.samples} NT={wl.replicas} L={wl.L}")
    J = wl.couplings()
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed, walk=True)
    pt.pt_mcs(job, 12, measure=True)
    picks = [0, 517, wl.samples - 1]
    ref = oracle.OracleJob(len(picks), wl.replicas, wl.L, wl.dim, J[picks], wl.betas, wl.seed,
                           sample_keys=picks)
    ref.mcs(12, measure=True)
    assert (pt.pt_get_spins(job)[picks] == ref.spins()).all()
    assert (pt.pt_get_energies(job)[picks] == ref.energies()).all()
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a[picks] == b).all()
    gm, rm = pt.pt_get_moments(job), ref.moments()
    for k in rm:
        assert (np.asarray(gm[k])[picks] == np.asarray(rm[k]).astype(np.asarray(gm[k]).dtype)).all(), k
    for x, y in zip(pt.pt_get_walk(job), ref.walk()):
        assert (x[picks] == y).all()
    ps, _, n = pt.pt_observables(job)
    rps, _, rn = ref.observables()
    assert n == rn == 12
    np.testing.assert_allclose(ps[picks], rps, rtol=1e-12, atol=0)


def test_full_size_2d_l64_houdayer_sampled(pt):
    wl = W.workload("2d_l64")
    say(f"case {wl.name} S={wl.samples} NT={wl.replicas} L={wl.L}")
    J = wl.couplings()
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed, walk=True)
    pt.pt_mcs(job, 6, houdayer=True, measure=True)
    picks = [3, wl.samples - 2]
    ref = oracle.OracleJob(len(picks), wl.replicas, wl.L, wl.dim, J[picks], wl.betas, wl.seed,
                           sample_keys=picks)
    ref.mcs(6, houdayer=True, measure=True)
    assert (pt.pt_get_spins(job)[picks] == ref.spins()).all()
    assert (pt.pt_get_energies(job)[picks] == ref.energies()).all()
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a[picks] == b).all()
    for x, y in zip(pt.pt_get_walk(job), ref.walk()):
        assert (x[picks] == y).all()


@pytest.mark.parametrize("layout", [0, 1])
def test_3d_l16_long(pt, layout):
    """3D L=16 (the shape whose sweep runs with compile-time geometry) for 300
    steps of sweep, exchange and measurement at 8 temperatures across the
    workload's range; every bit of the state and the observables against the
    oracle."""
    S, NT = 2, 8
    betas = W.geometric_betas(0.9, 2.0, NT)
    J = W.couplings_pm_j(S, 16, 3, 1616)
    say(f"case 3d L=16 S={S} NT={NT} layout={layout}, 300 steps")
    job = pt.pt_init(S, NT, 16, 3, J, betas, 5150 + layout, layout=layout)
    ref = oracle.OracleJob(S, NT, 16, 3, J, betas, 5150 + layout)
    for n in (100, 200):
        pt.pt_mcs(job, n, measure=True)
        ref.mcs(n, measure=True)
        compare(pt, job, ref, f"after {n}")
    compare_observables(pt, job, ref)
    pt.pt_destroy(job)


def test_2d_l64_houdayer_long_cold(pt):
    """2D L=64 at the workload's lowest temperatures for 300 steps of sweep,
    Houdayer move, exchange and measurement: overlap clusters grow large and
    cross the periodic boundary in both directions, which exercises every
    branch of the in-register cluster fill."""
    S, NT = 2, 8
    betas = W.power_law_betas(0.2, 0.6, NT, W.phi_star(64))
    J = W.couplings_pm_j(S, 64, 2, 4242)
    say(f"case 2d L=64 S={S} NT={NT} cold, 300 steps")
    job = pt.pt_init(S, NT, 64, 2, J, betas, 99)
    ref = oracle.OracleJob(S, NT, 64, 2, J, betas, 99)
    for n in (150, 150):
        pt.pt_mcs(job, n, houdayer=True, measure=True)
        ref.mcs(n, houdayer=True, measure=True)
        compare(pt, job, ref, f"after {n}")
    compare_observables(pt, job, ref)
    pt.pt_destroy(job)


@pytest.mark.parametrize("d,L,S,NT,layout,hou,meas", [
    (3, 8, 3, 5, 0, False, True), (3, 16, 2, 6, 1, True, True), (2, 64, 2, 5, 0, True, True),
    (2, 6, 3, 3, 1, True, False), (3, 12, 2, 4, 0, False, False), (2, 16, 4, 7, 0, True, True),
])
def test_fused_steps_equal_plain_and_oracle(pt, d, L, S, NT, layout, hou, meas):
    say(f"fused case d={d} L={L} S={S} NT={NT} layout={layout} hou={hou} meas={meas}")
    J = W.couplings_pm_j(S, L, d, 300 + L)
    betas = W.geometric_betas(0.3, 2.0, NT)
    fused = pt.pt_init(S, NT, L, d, J, betas, 77, layout=layout)
    plain = pt.pt_init(S, NT, L, d, J, betas, 77, layout=layout)
    ref = oracle.OracleJob(S, NT, L, d, J, betas, 77)
    for n in (1, 4, 7):
        pt.pt_mcs(fused, n, houdayer=hou, measure=meas)
        pt.pt_mcs(plain, n, houdayer=hou, measure=meas, plain=True)
        ref.mcs(n, houdayer=hou, measure=meas)
        compare(pt, fused, ref, f"fused after {n}")
        compare(pt, plain, ref, f"plain after {n}")


def test_full_run_small3d(pt):
    """The whole 3D L=8 workload: 8 samples x 16 temperatures, 1000 steps of
    sweep + exchange, measured over the second half; every bit of the final
    state and the observables against the oracle."""
    wl = W.workload("small3d")
    say(f"case {wl.name} S={wl.samples} NT={wl.replicas} L={wl.L} sweeps={wl.sweeps}")
    J = wl.couplings()
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed)
    ref = oracle.OracleJob(wl.samples, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed)
    half = wl.sweeps // 2
    pt.pt_mcs(job, half)
    pt.pt_mcs(job, wl.sweeps - half, measure=True)
    ref.mcs(half)
    ref.mcs(wl.sweeps - half, measure=True)
    compare(pt, job, ref, "small3d full run")
    compare_observables(pt, job, ref)
    pt.pt_destroy(job)


@pytest.mark.parametrize("NT", [2, 31, 32, 33, 63, 64, 65])
def test_exchange_ladder_sizes(pt, NT):
    """The exchange walk at the ladder sizes where its form changes: decision
    rows of one or two words (N_T = 32 / 33), the last ladder one wavefront
    walks by ballots (64) and the first one walked serially (65); every bit
    of the state and the walk against the oracle after fused and per-step
    steps, with narrow spacing so that most exchanges are accepted and long
    chains form."""
    d, L, S = 2, 4, 2
    J = W.couplings_pm_j(S, L, d, 900 + NT)
    betas = W.geometric_betas(1.0, 1.6, NT)
    say(f"ladder case NT={NT}")
    job = pt.pt_init(S, NT, L, d, J, betas, 31 + NT, walk=True)
    ref = oracle.OracleJob(S, NT, L, d, J, betas, 31 + NT)
    pt.pt_mcs(job, 25, measure=True)
    ref.mcs(25, measure=True)
    compare(pt, job, ref, "fused")
    pt.pt_mcs(job, 5, measure=True, plain=True)
    ref.mcs(5, measure=True)
    compare(pt, job, ref, "per-step")
    pt.pt_destroy(job)
