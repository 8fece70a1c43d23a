"""pt_mcs_noalloc (the work list in the library's static scratch, no device
allocation) against pt_mcs on twin jobs: spins, energies, maps, counters and
integer moments bit for bit, for two calls in a row (the second with a smaller
job), a split sample, a Houdayer job, a call longer than one launch, the
per-step fallback and a Gaussian-coupling job (fused steps that use no
scratch); a launch beyond the scratch's item limit is refused before anything
runs."""
import numpy as np
import pytest

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


def twins(pt, d, L, S, NT, seed, layout=0):
    J = W.couplings_pm_j(S, L, d, 700 + L + S)
    b = W.geometric_betas(0.9, 2.0, NT) if d == 3 else W.geometric_betas(0.3, 1.6, NT)
    return (pt.pt_init(S, NT, L, d, J, b, seed, layout=layout),
            pt.pt_init(S, NT, L, d, J, b, seed, layout=layout))


def same_state(pt, a, b, what):
    assert (pt.pt_get_spins(a) == pt.pt_get_spins(b)).all(), f"{what}: spins"
    assert (pt.pt_get_energies(a) == pt.pt_get_energies(b)).all(), f"{what}: energies"
    for x, y in zip(pt.pt_get_maps(a), pt.pt_get_maps(b)):
        assert (x == y).all(), f"{what}: maps"
    assert pt.pt_get_counters(a) == pt.pt_get_counters(b), what
    ma, mb = pt.pt_get_moments(a), pt.pt_get_moments(b)
    for k in ma:
        assert (np.asarray(ma[k]) == np.asarray(mb[k])).all(), (what, k)


# (dim, L, samples, N_T, steps, houdayer, layout): the first is the larger
# launch, the second a smaller one run right after it on the same scratch
CASES = [
    (3, 16, 40, 8, 30, False, 0),    # 40 items, both sets per workgroup
    (3, 8, 3, 4, 12, True, 1),       # 3 items, Houdayer room, packed spins
    (3, 32, 2, 32, 8, False, 0),     # split samples (parts of one sample consecutive)
    (2, 64, 4, 24, 10, True, 0),     # 2D L = 64 with Houdayer moves in registers
    (3, 8, 2, 4, 620, False, 0),     # more steps than one launch holds
]


def test_noalloc_matches_pt_mcs_call_after_call(pt):
    for d, L, S, NT, n, hou, layout in CASES:
        say(f"pt_mcs_noalloc d={d} L={L} S={S} NT={NT} steps={n} houdayer={hou} layout={layout}")
        a, b = twins(pt, d, L, S, NT, 0x5EED + 7 * L + NT, layout)
        pt.pt_mcs_noalloc(a, n, houdayer=hou, measure=True)
        pt.pt_mcs(b, n, houdayer=hou, measure=True)
        same_state(pt, a, b, f"d={d} L={L} S={S} NT={NT}")
        # a second call on the same job continues the streams
        pt.pt_mcs_noalloc(a, 3, houdayer=hou, measure=True)
        pt.pt_mcs(b, 3, houdayer=hou, measure=True)
        same_state(pt, a, b, f"d={d} L={L} S={S} NT={NT}, second call")
        pt.pt_destroy(a)
        pt.pt_destroy(b)


def test_noalloc_per_step_fallback_and_limit(pt):
    # a 3D Houdayer job whose two sets exceed one workgroup: per-step kernels
    say("pt_mcs_noalloc per-step fallback 3D L=32 NT=4 Houdayer")
    a, b = twins(pt, 3, 32, 1, 4, 99)
    assert pt.pt_get_plan(a, houdayer=True, measure=True)["mode"] == -1
    pt.pt_mcs_noalloc(a, 4, houdayer=True, measure=True)
    pt.pt_mcs(b, 4, houdayer=True, measure=True)
    same_state(pt, a, b, "per-step fallback")
    pt.pt_destroy(a)
    pt.pt_destroy(b)
    # more work items than the scratch holds: refused, nothing changes
    S = pt.PT_NOALLOC_MAX_ITEMS + 1
    say(f"pt_mcs_noalloc refusal S={S}")
    J = np.ones((S, 2, 16), np.int8)
    job = pt.pt_init(S, 2, 4, 2, J, np.array([1.0, 0.5]), 5)
    before = pt.pt_get_spins(job)
    with pytest.raises(pt.PTError) as ei:
        pt.pt_mcs_noalloc(job, 2, measure=True)
    assert ei.value.code == pt.PT_EINVAL
    assert pt.pt_get_counters(job)["t"] == 0
    assert (pt.pt_get_spins(job) == before).all()
    pt.pt_mcs(job, 1)  # the job still works
    assert pt.pt_get_counters(job)["t"] == 1
    pt.pt_destroy(job)


def test_noalloc_gauss(pt):
    """Gaussian jobs: pt_mcs_noalloc takes the same fused steps as pt_mcs (one
    workgroup per sample, no scratch), twice in a row."""
    d, L, S, NT = 2, 16, 3, 6
    say(f"pt_mcs_noalloc gauss d={d} L={L} S={S} NT={NT}")
    Jf = W.couplings_gauss(S, L, d, 41)
    b = W.geometric_betas(0.2, 1.6, NT)
    a = pt.pt_init_gauss(S, NT, L, d, Jf, b, 17)
    c = pt.pt_init_gauss(S, NT, L, d, Jf, b, 17)
    assert pt.pt_get_plan(a, houdayer=True, measure=True)["mode"] == 0
    for n in (9, 4):
        pt.pt_mcs_noalloc(a, n, houdayer=True, measure=True)
        pt.pt_mcs(c, n, houdayer=True, measure=True)
        assert (pt.pt_get_spins(a) == pt.pt_get_spins(c)).all()
        assert (pt.pt_get_energies64(a) == pt.pt_get_energies64(c)).all()
        for x, y in zip(pt.pt_get_maps(a), pt.pt_get_maps(c)):
            assert (x == y).all()
        assert pt.pt_get_counters(a) == pt.pt_get_counters(c)
        assert (pt.pt_get_moments8(a) == pt.pt_get_moments8(c)).all()
    pt.pt_destroy(a)
    pt.pt_destroy(c)
