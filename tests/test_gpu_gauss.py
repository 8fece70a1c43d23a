"""GPU parity of the Gaussian-coupling model (Sec. 2.1: couplings from a
standard normal; the 2D Gaussian workload of Sec. 4.2): the exact acceptance
decision on the device in all its tiers, and every step (sweep, exchange,
single- and multi-cluster Houdayer moves, measurement, Monte Carlo steps)
bit-identical to the CPU oracle in spins, 64-bit energies, maps, counters and
moments, FP64 observables within 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2003_04621_amd import workloads as W
from test_gauss_accept import boundary_cases, boundary_words

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


def oracle_moments8(ref):
    m = ref.moments()
    out = np.zeros((ref.S, ref.NT, 8), np.int64)
    out[..., 0] = m["E"]
    out[..., 1] = m["E2"][..., 0].astype(np.int64)
    out[..., 2] = m["Q"]
    out[..., 3] = m["AQ"]
    out[..., 4] = m["Q2"]
    out[..., 5] = m["Q4"][..., 0].astype(np.int64)
    out[..., 6] = m["Q4"][..., 1].astype(np.int64)
    out[..., 7] = m["E2"][..., 1].astype(np.int64)
    return out


def matches(pt, job, ref, what, obs=False):
    assert (pt.pt_get_spins(job) == ref.spins()).all(), f"{what}: spins"
    assert (pt.pt_get_energies64(job) == ref.energies()).all(), f"{what}: energies"
    for a, b in zip(pt.pt_get_maps(job), ref.maps()):
        assert (a == b).all(), f"{what}: maps"
    assert pt.pt_get_counters(job) == ref.counters(), what
    assert (pt.pt_get_moments8(job) == oracle_moments8(ref)).all(), f"{what}: moments"
    if obs:
        ps, dis, n = pt.pt_observables(job)
        rps, rdis, rn = ref.observables()
        assert n == rn
        np.testing.assert_allclose(ps, rps, rtol=1e-12, atol=0)
        np.testing.assert_allclose(dis, rdis, rtol=1e-12, atol=0)


def make(pt, d, L, S, NT, layout, seed0, betas=None):
    Jf = W.couplings_gauss(S, L, d, seed0)
    Jn = W.gauss_units(Jf)
    b = betas if betas is not None else (W.geometric_betas(0.5, 2.0, NT) if d == 3
                                         else W.geometric_betas(0.2, 1.6, NT))
    seed = 0x6A55_0000 + 31 * L + NT + seed0
    return (pt.pt_init_gauss(S, NT, L, d, Jf, b, seed, layout=layout),
            oracle.OracleGaussJob(S, NT, L, d, Jn, b, seed))


def test_device_acceptance_all_tiers(pt):
    """Boundary words around 2^32 exp(-b u 2^-16) from a 60-digit decimal
    evaluation: the Metropolis path (float32 -> double -> double-double), the
    exchange path (double -> double-double) and double-double alone."""
    cases = boundary_cases(5, 4000)
    r, b, u, want = boundary_words(cases)
    say(f"acceptance: {r.size} words")
    for mode in (1, 2):
        got = pt.pt_gauss_accept_test(r, b, u, mode)
        assert (got == want).all(), (mode, np.flatnonzero(got != want)[:10])
    m = u < (1 << 24)
    got = pt.pt_gauss_accept_test(r[m], b[m], u[m], 0)
    assert (got == want[m]).all(), np.flatnonzero(got != want[m])[:10]
    # random words against the oracle in every mode
    rng = np.random.default_rng(17)
    n = 200_000
    rr = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    bb = rng.uniform(0.01, 5.0, size=n)
    uu = rng.integers(1, 1 << 24, size=n).astype(np.int64)
    ref = np.array([oracle.gauss_accept(int(x), float(y), int(z))
                    for x, y, z in zip(rr[:20000], bb[:20000], uu[:20000])], np.int32)
    for mode in (0, 1, 2):
        got = pt.pt_gauss_accept_test(rr[:20000], bb[:20000], uu[:20000], mode)
        assert (got == ref).all(), mode
    # the three paths agree with each other on many more words
    g0 = pt.pt_gauss_accept_test(rr, bb, uu, 0)
    g2 = pt.pt_gauss_accept_test(rr, bb, uu, 2)
    assert (g0 == g2).all()


SHAPES = [  # (dim, L, samples, replicas, layout)
    (2, 4, 2, 3, 0),
    (2, 6, 2, 4, 1),
    (2, 12, 3, 5, 0),
    (2, 16, 2, 4, 1),
    (2, 64, 2, 5, 0),
    (3, 4, 2, 3, 1),
    (3, 6, 2, 4, 0),
    (3, 8, 2, 6, 1),
    (3, 12, 1, 4, 0),
    (3, 16, 2, 3, 0),
]


@pytest.mark.parametrize("d,L,S,NT,layout", SHAPES)
def test_gauss_steps_match_oracle(pt, d, L, S, NT, layout):
    say(f"gauss d={d} L={L} S={S} NT={NT} layout={layout}")
    job, ref = make(pt, d, L, S, NT, layout, 7 * L + d)
    matches(pt, job, ref, "init")
    # separate entry points
    pt.pt_sweep(job, 2)
    ref.sweep(2)
    matches(pt, job, ref, "sweep x2")
    pt.pt_exchange(job)
    ref.exchange()
    matches(pt, job, ref, "exchange")
    pt.pt_houdayer(job)
    ref.houdayer()
    matches(pt, job, ref, "houdayer")
    if L ** d <= 32768:
        pt.pt_houdayer_multi(job)
        ref.houdayer(multi=True)
        matches(pt, job, ref, "houdayer multi")
    pt.pt_measure(job)
    ref.measure()
    matches(pt, job, ref, "measure", obs=True)
    # Monte Carlo steps: Metropolis + Houdayer + exchange + measure
    pt.pt_mcs(job, 6, houdayer=True, measure=True)
    ref.mcs(6, houdayer=True, measure=True)
    matches(pt, job, ref, "mcs houdayer", obs=True)
    if L ** d <= 32768:
        pt.pt_mcs(job, 5, houdayer=True, measure=True, multi=True)
        ref.mcs(5, houdayer=True, measure=True, multi=True)
        matches(pt, job, ref, "mcs multi", obs=True)
    pt.pt_set_measure_interval(job, 3)
    ref.set_measure_every(3)
    pt.pt_mcs(job, 7, measure=True)
    ref.mcs(7, measure=True)
    matches(pt, job, ref, "mcs interval 3", obs=True)
    pt.pt_destroy(job)


FUSED_SHAPES = [  # (dim, L, samples, replicas, layout)
    (2, 8, 3, 4, 0),
    (2, 12, 2, 5, 1),
    (2, 64, 2, 24, 1),
    (3, 6, 2, 3, 0),
    (3, 8, 2, 6, 1),
    (3, 16, 2, 8, 0),
]


def same_state(pt, x, y, what):
    assert (pt.pt_get_spins(x) == pt.pt_get_spins(y)).all(), f"{what}: spins"
    assert (pt.pt_get_energies64(x) == pt.pt_get_energies64(y)).all(), f"{what}: energies"
    for a, b in zip(pt.pt_get_maps(x), pt.pt_get_maps(y)):
        assert (a == b).all(), f"{what}: maps"
    assert pt.pt_get_counters(x) == pt.pt_get_counters(y), what
    assert (pt.pt_get_moments8(x) == pt.pt_get_moments8(y)).all(), f"{what}: moments"


@pytest.mark.parametrize("d,L,S,NT,layout", FUSED_SHAPES)
def test_gauss_fused_matches_per_step_and_oracle(pt, d, L, S, NT, layout):
    """Fused Gaussian steps (one workgroup per sample with all its
    configurations in LDS, n steps per launch) against the per-step kernels
    (PT_MCS_PLAIN) and the oracle: spins, 64-bit energies, maps, counters and
    moments bit for bit, with and without Houdayer moves and measurements, at
    a measurement interval, and across launches of more than 500 steps."""
    say(f"gauss fused d={d} L={L} S={S} NT={NT} layout={layout}")
    job, ref = make(pt, d, L, S, NT, layout, 300 + L)
    plain, _ = make(pt, d, L, S, NT, layout, 300 + L)
    plan = pt.pt_get_plan(job, houdayer=True, measure=True)
    assert plan["mode"] == 0 and plan["parts"] == 1 and plan["per_part"] == 2 * NT
    assert pt.pt_get_plan(job, houdayer=True, measure=True, plain=True)["mode"] == -1
    assert pt.pt_get_plan(job, houdayer=True, measure=True, multi=True)["mode"] == -1
    for n, hou, meas in ((7, True, True), (5, False, True), (4, True, False), (3, False, False)):
        pt.pt_mcs(job, n, houdayer=hou, measure=meas)
        pt.pt_mcs(plain, n, houdayer=hou, measure=meas, plain=True)
        ref.mcs(n, houdayer=hou, measure=meas)
        same_state(pt, job, plain, f"{n} steps houdayer={hou} measure={meas}")
    matches(pt, job, ref, "fused steps", obs=True)
    pt.pt_set_measure_interval(job, 3)
    pt.pt_set_measure_interval(plain, 3)
    ref.set_measure_every(3)
    pt.pt_mcs(job, 8, houdayer=True, measure=True)
    pt.pt_mcs(plain, 8, houdayer=True, measure=True, plain=True)
    ref.mcs(8, houdayer=True, measure=True)
    same_state(pt, job, plain, "interval 3")
    matches(pt, job, ref, "interval 3", obs=True)
    if L ** d <= 512:
        # a call longer than one launch (500 steps)
        pt.pt_mcs(job, 520, houdayer=True, measure=True)
        pt.pt_mcs(plain, 520, houdayer=True, measure=True, plain=True)
        same_state(pt, job, plain, "520 steps")
    pt.pt_destroy(job)
    pt.pt_destroy(plain)


def test_gauss_long_cold_2d(pt):
    """A long run at low temperatures (most moves decided by the threshold
    comparison), 2D L = 16 with both Houdayer variants alternating."""
    job, ref = make(pt, 2, 16, 2, 6, 0, 99, betas=W.geometric_betas(0.1, 1.0, 6))
    for rep in range(10):
        multi = rep % 2 == 1
        pt.pt_mcs(job, 20, houdayer=True, measure=True, multi=multi)
        ref.mcs(20, houdayer=True, measure=True, multi=multi)
    matches(pt, job, ref, "long cold", obs=True)


def test_gauss_set_spins_and_symmetry(pt):
    """pt_set_spins recomputes the 64-bit energies; the global flip leaves
    every energy and the whole trajectory's maps unchanged."""
    d, L, S, NT = 3, 6, 2, 4
    job, ref = make(pt, d, L, S, NT, 1, 5)
    rng = np.random.default_rng(3)
    spins = rng.choice(np.array([-1, 1], np.int8), size=(S, 2 * NT, L ** d))
    pt.pt_set_spins(job, spins)
    ref.set_spins(spins)
    matches(pt, job, ref, "set_spins")
    job2, _ = make(pt, d, L, S, NT, 0, 5)
    pt.pt_set_spins(job2, -spins)
    assert (pt.pt_get_energies64(job2) == pt.pt_get_energies64(job)).all()
    pt.pt_mcs(job, 4, houdayer=True)
    ref.mcs(4, houdayer=True)
    matches(pt, job, ref, "after set_spins")


def test_gauss_checkpoint_resume(pt):
    """Checkpoint after n steps, keep going, restore and redo: the continuation
    is bit-identical (spins, 64-bit energies, maps, counters, moments), and the
    oracle run for 2n steps agrees; a +-J job's state is refused."""
    d, L, S, NT = 2, 16, 2, 4
    job, ref = make(pt, d, L, S, NT, 0, 9)
    pt.pt_mcs(job, 6, houdayer=True, measure=True)
    state = pt.pt_get_state(job)
    pt.pt_mcs(job, 5, houdayer=True, measure=True, multi=True)
    after = (pt.pt_get_spins(job), pt.pt_get_energies64(job), pt.pt_get_moments8(job),
             pt.pt_get_counters(job))
    pt.pt_set_state(job, state)
    pt.pt_mcs(job, 5, houdayer=True, measure=True, multi=True)
    again = (pt.pt_get_spins(job), pt.pt_get_energies64(job), pt.pt_get_moments8(job),
             pt.pt_get_counters(job))
    for x, y in zip(after[:3], again[:3]):
        assert (x == y).all()
    assert after[3] == again[3]
    ref.mcs(6, houdayer=True, measure=True)
    ref.mcs(5, houdayer=True, measure=True, multi=True)
    matches(pt, job, ref, "restored and continued")
    other = pt.pt_init(S, NT, L, d, W.couplings_pm_j(S, L, d, 3), W.geometric_betas(0.5, 1.0, NT), 1)
    with pytest.raises(pt.PTError):
        pt.pt_set_state(other, state)
    pt.pt_destroy(other)
    pt.pt_destroy(job)


def test_gauss_refusals(pt):
    d, L, S, NT = 2, 8, 1, 3
    job, _ = make(pt, d, L, S, NT, 0, 1)
    for fn in (lambda: pt.pt_get_energies(job), lambda: pt.pt_get_moments(job),
               lambda: pt.pt_batch_create([job])):
        with pytest.raises(pt.PTError):
            fn()
    Jf = W.couplings_gauss(S, L, d, 1)
    Jf[0, 0, 0] = np.float32(0.1)  # not a multiple of 2^-16
    with pytest.raises(pt.PTError):
        pt.pt_init_gauss(S, NT, L, d, Jf, W.geometric_betas(0.5, 1.0, NT), 1)


def test_full_size_2d_l64_gauss_sampled(pt):
    """The 2D Gaussian workload at full size (2D L = 64, 500 samples x 2 x 24
    temperatures, the power-law ladder of the +-J 2D workload), a few Monte
    Carlo steps with Houdayer moves and measurements; sampled samples
    re-run by the oracle under their own sample keys."""
    wl = W.workload("2d_l64_gauss")
    Jf = wl.couplings()
    say(f"full size gauss: S={wl.samples} NT={wl.replicas} L={wl.L}")
    job = pt.pt_init_gauss(wl.samples, wl.replicas, wl.L, wl.dim, Jf, wl.betas, wl.seed)
    pt.pt_mcs(job, 3, houdayer=True, measure=True)
    sp, E, (sot, tos) = pt.pt_get_spins(job), pt.pt_get_energies64(job), pt.pt_get_maps(job)
    mom = pt.pt_get_moments8(job)
    Jn = W.gauss_units(Jf)
    for s in (0, 1, 137, wl.samples - 1):
        ref = oracle.OracleGaussJob(1, wl.replicas, wl.L, wl.dim, Jn[[s]], wl.betas, wl.seed,
                                    sample_keys=[s])
        ref.mcs(3, houdayer=True, measure=True)
        assert (sp[s] == ref.spins()[0]).all(), s
        assert (E[s] == ref.energies()[0]).all(), s
        rs, rt = ref.maps()
        assert (sot[s] == rs[0]).all() and (tos[s] == rt[0]).all(), s
        assert (mom[s] == oracle_moments8(ref)[0]).all(), s
    pt.pt_destroy(job)
