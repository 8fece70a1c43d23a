"""GPU parity of the replica walk and its round trips (Sec. 2.3).

Every exchange path (fused with both replica sets per workgroup, one set per
workgroup, split samples, the per-step kernels, batches) updates the walk
labels, trip beginnings and round-trip bins; they must equal the oracle's bit
for bit on small runs with many round trips, equal the closed form of the
all-accepted exchange pass at larger sizes, and obey the walk's invariants at
the full 3D L=16 size in the benchmark's launch configuration."""
import numpy as np
import pytest

import oracle
from paper_2003_04621_amd import workloads as W
from walk_forms import expected_rotation

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


def same_walk(pt, job, ref, what):
    sot, tos = pt.pt_get_maps(job)
    rsot, rtos = ref.maps()
    assert (sot == rsot).all() and (tos == rtos).all(), f"{what}: maps"
    for x, y, name in zip(pt.pt_get_walk(job), ref.walk(), ("labels", "begins", "trips")):
        assert (x == y).all(), f"{what}: {name}"
    assert (pt.pt_get_energies(job) == ref.energies()).all(), f"{what}: energies"


@pytest.mark.parametrize("path", ["fused", "plain", "one_set", "houdayer", "batch"])
def test_walk_long_vs_oracle(pt, path):
    """Narrow ladders at high temperature, so that replicas diffuse fast and
    make many round trips; several launches, so that the walk state and the
    trip sums survive between them."""
    d, L, S, NT = (2, 16, 2, 5) if path == "houdayer" else (3, 8, 3, 5)
    betas = W.geometric_betas(1.8, 2.6, NT)
    J = W.couplings_pm_j(S, L, d, 77)
    seed = 4040 + len(path)
    say(f"walk case {path}: d={d} L={L} S={S} NT={NT}")
    job = pt.pt_init(S, NT, L, d, J, betas, seed, walk=True)
    ref = oracle.OracleJob(S, NT, L, d, J, betas, seed)
    hou = path == "houdayer"
    batch = None
    if path in ("one_set", "batch"):
        other = pt.pt_init(1, 3, 6, d, W.couplings_pm_j(1, 6, d, 5), W.geometric_betas(1.0, 2.0, 3), 9)
        batch = pt.pt_batch_create([job, other] if path == "batch" else [job])
        if path == "one_set":
            pt.pt_batch_set_config(batch, 0, 1, 0)
    for n in (150, 250):
        if batch is not None:
            pt.pt_batch_run(batch, n, measure=True)
        else:
            pt.pt_mcs(job, n, houdayer=hou, measure=True, plain=path == "plain")
        ref.mcs(n, houdayer=hou, measure=True)
        same_walk(pt, job, ref, f"{path} after {n}")
    trips = pt.pt_get_walk(job)[2]
    assert int(trips[..., 0].sum()) > 20, "too few round trips to test anything"
    assert pt.pt_tunnel_summary(trips, 400)[2] == oracle.tunnel_summary(ref.walk()[2], 400)[2]
    if batch is not None:
        pt.pt_batch_destroy(batch)


ROTATION = [
    # (name, dim, L, samples, replicas, steps per call, calls, how)
    ("fused 3D L=16", 3, 16, 64, 32, 500, 2, "mcs"),
    ("plain 3D L=8", 3, 8, 4, 6, 40, 3, "plain"),
    ("one set 3D L=16", 3, 16, 8, 16, 90, 2, "one_set"),
    ("split 3D L=32", 3, 32, 2, 24, 100, 3, "mcs"),
    ("split 2D L=64", 2, 64, 1, 160, 200, 2, "mcs"),
    ("split 3D L=48, 12 parts", 3, 48, 1, 48, 60, 2, "mcs"),
    ("houdayer 2D L=64", 2, 64, 4, 24, 70, 2, "houdayer"),
]


@pytest.mark.parametrize("name,d,L,S,NT,n,calls,how", ROTATION)
def test_walk_rotation_closed_form(pt, name, d, L, S, NT, n, calls, how):
    """Numerically equal temperatures: every exchange is accepted (a word of
    all ones, probability 2^-32 per decision, aside), slot j sits at
    temperature (j - m) mod NT after pass m, and every round trip lasts NT
    passes."""
    betas = 0.5 - 1e-13 * np.arange(NT)
    J = W.couplings_pm_j(S, L, d, 31)
    say(f"rotation case {name}: S={S} NT={NT}, {calls} x {n} steps")
    job = pt.pt_init(S, NT, L, d, J, betas, 12345, walk=True)
    batch = None
    if how == "one_set":
        batch = pt.pt_batch_create([job])
        pt.pt_batch_set_config(batch, 0, 1, 0)
    for _ in range(calls):
        if batch is not None:
            pt.pt_batch_run(batch, n)
        else:
            pt.pt_mcs(job, n, houdayer=how == "houdayer", measure=True, plain=how == "plain")
    P = n * calls
    assert pt.pt_get_counters(job)["u"] == P
    _, tos = pt.pt_get_maps(job)
    want = np.array([(j - P) % NT for j in range(NT)], np.int32)
    assert (tos == want).all(), "an exchange was rejected"
    lab, beg, trips = pt.pt_get_walk(job)
    elab, ebeg, ebins = expected_rotation(NT, P)
    assert (lab == np.tile(elab, 2)).all()
    assert (beg == np.tile(ebeg, 2)).all()
    assert (trips == 2 * ebins).all()
    if batch is not None:
        pt.pt_batch_destroy(batch)


def test_walk_full_size_invariants(pt):
    """3D L=16, 1000 samples x 2 x 32 temperatures, 1000 measured steps in the
    benchmark's launches of 500: what must hold at any size."""
    wl = W.workload("3d_l16")
    say(f"case {wl.name} S={wl.samples} NT={wl.replicas}, 1000 steps")
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas, wl.seed,
                     walk=True)
    pt.pt_mcs(job, 500, measure=True)
    pt.pt_mcs(job, 500, measure=True)
    P, NT = 1000, wl.replicas
    lab, beg, trips = pt.pt_get_walk(job)
    _, tos = pt.pt_get_maps(job)
    tos = tos.reshape(wl.samples, 2 * NT)
    assert set(np.unique(lab)) <= {0, 1, 2}
    assert (lab[tos == 0] == 1).all()  # just seen at the lowest temperature
    assert np.isin(lab[tos == NT - 1], [0, 2]).all()
    assert (beg[lab == 0] == 0).all()
    assert ((beg[lab > 0] >= 1) & (beg[lab > 0] <= P)).all()
    C, D, Q = (trips[..., i].astype(object) for i in range(3))
    assert C.sum() > 0
    assert (D >= NT * C).all() and (Q >= NT * D).all() and (C * Q >= D * D).all()
    assert (C[:, P.bit_length():] == 0).all()  # no trip ends after pass P
    tau_b, err_b, tau, eq = pt.pt_tunnel_summary(trips, P)
    assert tau >= NT
    say(f"tau_tunnel {tau:.1f} passes over {int(C.sum())} round trips, equilibrated {eq}")


def test_walk_is_opt_in(pt):
    """A job created without the walk has none to report, keeps a smaller
    checkpoint, and a checkpoint of one kind does not restore into the other;
    a walk job's checkpoint continues bit-exactly, walk included."""
    d, L, S, NT = 3, 8, 2, 4
    J = W.couplings_pm_j(S, L, d, 3)
    b = W.geometric_betas(1.8, 2.6, NT)
    plain_job = pt.pt_init(S, NT, L, d, J, b, 6)
    with pytest.raises(pt.PTError):
        pt.pt_get_walk(plain_job)
    a = pt.pt_init(S, NT, L, d, J, b, 6, walk=True)
    pt.pt_mcs(a, 70, measure=True)
    pt.pt_mcs(plain_job, 70, measure=True)
    assert (pt.pt_get_spins(a) == pt.pt_get_spins(plain_job)).all()  # the walk changes nothing else
    st, st_plain = pt.pt_get_state(a), pt.pt_get_state(plain_job)
    assert len(st) > len(st_plain)
    with pytest.raises(pt.PTError):
        pt.pt_set_state(plain_job, st)
    pt.pt_mcs(a, 80, measure=True)
    c = pt.pt_init(S, NT, L, d, J, b, 6, walk=True)
    pt.pt_set_state(c, st)
    pt.pt_mcs(c, 80, measure=True)
    ref = oracle.OracleJob(S, NT, L, d, J, b, 6)
    ref.mcs(150, measure=True)
    same_walk(pt, c, ref, "restored")
    for x, y in zip(pt.pt_get_walk(a), pt.pt_get_walk(c)):
        assert (x == y).all()
    assert pt.pt_plan_query(d, L, NT, measure=True, walk=True)["lds_bytes"] > \
        pt.pt_plan_query(d, L, NT, measure=True)["lds_bytes"]
