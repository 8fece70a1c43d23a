"""GPU tests of the served form: requests admitted by HBM budget, advanced in
continuous batches, must give the same observables as the same job run alone
(bit-identical FP64 values from identical integer moments)."""
import time

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


REQUESTS = [  # (dim, L, replicas, samples, sweeps, burn_in, houdayer, layout)
    (3, 8, 4, 2, 30, 10, False, 0),
    (3, 16, 6, 1, 25, 12, False, 1),
    (2, 64, 3, 1, 20, 5, True, 0),
    (3, 12, 5, 3, 17, 0, False, 0),
    (3, 48, 8, 1, 9, 4, False, 0),      # too large for one workgroup: a split sample
    (2, 16, 4, 2, 33, 11, True, 1),
    (3, 8, 3, 1, 0, 0, False, 0),        # nothing to do
    (3, 24, 4, 1, 14, 7, False, 1),
]


def _inputs(n, spec):
    dim, L, NT, S, sweeps, burn, hou, layout = spec
    J = W.couplings_pm_j(S, L, dim, 500 + n)
    b = W.geometric_betas(0.6, 2.0, NT)
    return J, b, 900 + n


def _alone(pt, n, spec):
    dim, L, NT, S, sweeps, burn, hou, layout = spec
    J, b, seed = _inputs(n, spec)
    job = pt.pt_init(S, NT, L, dim, J, b, seed, layout=layout)
    pt.pt_mcs(job, burn, houdayer=hou)
    pt.pt_mcs(job, sweeps - burn, houdayer=hou, measure=True)
    _, dis, nm = pt.pt_observables(job)
    pt.pt_destroy(job)
    return dis, nm


def _wait(pt, srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for n, t in tickets.items():
            if n in out:
                continue
            r = pt.pt_server_poll(srv, t)
            if r is not None:
                out[n] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.01)
    return out


def test_server_matches_alone_and_respects_budget(pt):
    budget = 24 << 20
    srv = pt.pt_server_start(budget, steps_per_round=7)
    tickets = {}
    for n, spec in enumerate(REQUESTS):
        dim, L, NT, S, sweeps, burn, hou, layout = spec
        J, b, seed = _inputs(n, spec)
        say(f"submit {spec}")
        tickets[n] = pt.pt_server_submit(srv, dim, L, NT, S, b, J, seed, sweeps, burn, hou, layout)
    res = _wait(pt, srv, tickets)
    stats = pt.pt_server_stats(srv)
    pt.pt_server_stop(srv)
    assert stats["peak_bytes"] <= budget
    assert stats["completed"] == len(REQUESTS)
    for n, spec in enumerate(REQUESTS):
        r = res[n]
        assert r["status"] == 0, (spec, r["status"])
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        dis, nm = _alone(pt, n, spec)
        assert r["n_meas"] == nm == spec[4] - spec[5]
        if nm > 0:
            assert np.array_equal(r["disorder"], dis), spec


ORACLE_REQUESTS = [  # (dim, L, replicas, samples, sweeps, burn_in, houdayer, layout, plan)
    (3, 32, 4, 1, 9, 3, True, 0, -1),     # 3D Houdayer too large for a workgroup: side stream
    (3, 48, 4, 1, 8, 3, False, 1, 3),     # a split sample
    (2, 16, 5, 2, 13, 4, True, 0, 1),     # 2D Houdayer, resident
    (3, 8, 6, 3, 11, 0, False, 1, 0),     # measured from the first step
    (3, 12, 3, 2, 10, 10, True, 0, 1),    # burn-in only: nothing measured
]


def test_server_results_match_the_oracle(pt):
    """Each finished request re-run by the CPU oracle from its inputs: the
    number of measurements exactly and the disorder averages within 1e-12
    (Sec. 2.4 steps, Eqs. (3)-(5), (10)), for the per-step side stream, a split
    sample and resident jobs served together."""
    srv = pt.pt_server_start(64 << 20, steps_per_round=4)
    tickets = {}
    for n, spec in enumerate(ORACLE_REQUESTS):
        dim, L, NT, S, sweeps, burn, hou, layout, plan = spec
        assert pt.pt_plan_query(dim, L, NT, houdayer=hou, measure=True)["mode"] == plan
        J, b, seed = _inputs(40 + n, spec[:8])
        say(f"submit {spec}")
        tickets[n] = pt.pt_server_submit(srv, dim, L, NT, S, b, J, seed, sweeps, burn, hou, layout)
    res = _wait(pt, srv, tickets, timeout=240.0)
    pt.pt_server_stop(srv)
    for n, spec in enumerate(ORACLE_REQUESTS):
        dim, L, NT, S, sweeps, burn, hou, layout, plan = spec
        r = res[n]
        assert r["status"] == 0, (spec, r["status"])
        J, b, seed = _inputs(40 + n, spec[:8])
        ref = oracle.OracleJob(S, NT, L, dim, J, b, seed)
        ref.mcs(burn, houdayer=hou)
        ref.mcs(sweeps - burn, houdayer=hou, measure=True)
        _, rdis, rn = ref.observables()
        say(f"oracle {spec}: n_meas {rn}")
        assert r["n_meas"] == rn == sweeps - burn
        if rn > 0:
            np.testing.assert_allclose(r["disorder"], rdis, rtol=1e-12, atol=0)


def test_server_same_result_alone_and_in_mix(pt):
    spec = (3, 16, 6, 2, 21, 9, False, 0)
    J, b, seed = _inputs(77, spec)
    dim, L, NT, S, sweeps, burn, hou, layout = spec
    alone = pt.pt_server_start(1 << 30, steps_per_round=5)
    t = pt.pt_server_submit(alone, dim, L, NT, S, b, J, seed, sweeps, burn, hou, layout)
    r_alone = _wait(pt, alone, {0: t})[0]
    pt.pt_server_stop(alone)
    mix = pt.pt_server_start(8 << 20, steps_per_round=4)
    tickets = {}
    for n, other in enumerate(REQUESTS[:6]):
        Jo, bo, so = _inputs(n, other)
        tickets[n] = pt.pt_server_submit(mix, other[0], other[1], other[2], other[3], bo, Jo, so,
                                         other[4], other[5], other[6], other[7])
        if n == 2:
            tickets["x"] = pt.pt_server_submit(mix, dim, L, NT, S, b, J, seed, sweeps, burn, hou,
                                               layout)
    res = _wait(pt, mix, tickets)
    pt.pt_server_stop(mix)
    assert np.array_equal(res["x"]["disorder"], r_alone["disorder"])
    assert res["x"]["n_meas"] == r_alone["n_meas"] == sweeps - burn


def test_server_rejects_oversized_and_bad_requests(pt):
    srv = pt.pt_server_start(1 << 20, steps_per_round=3)
    spec = (3, 32, 16, 1, 5, 0, False, 0)
    J, b, seed = _inputs(1, spec)
    t = pt.pt_server_submit(srv, 3, 32, 16, 1, b, J, seed, 5, 0)
    r = _wait(pt, srv, {0: t})[0]
    assert r["status"] == pt.PT_ENOMEM
    with pytest.raises(pt.PTError):
        pt.pt_server_submit(srv, 3, 32, 16, 1, b, J, seed, 5, 6)      # burn_in > sweeps
    with pytest.raises(pt.PTError):
        pt.pt_server_submit(srv, 3, 31, 16, 1, b, J, seed, 5, 0)      # odd L
    pt.pt_server_stop(srv)


def test_server_reports_round_trips_and_stops_at_equilibrium(pt):
    """A request keeping the replica walk returns its round-trip time and the
    logarithmic-binning check (Sec. 2.3), equal to the same job run alone; one
    asking to stop at equilibrium ends early, between rounds, with the check
    passed, and equals the job run alone for the steps it took."""
    dim, L, NT, S = 3, 4, 4, 2
    J = W.couplings_pm_j(S, L, dim, 61)
    b = W.geometric_betas(1.8, 2.6, NT)
    srv = pt.pt_server_start(1 << 30, steps_per_round=37)
    t_walk = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 71, 300, 20, walk=True)
    t_plain = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 71, 300, 20)
    t_eq = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 72, 20000, 10, walk=True,
                               until_equilibrated=True)
    res = _wait(pt, srv, {"walk": t_walk, "plain": t_plain, "eq": t_eq})
    pt.pt_server_stop(srv)
    assert res["plain"]["equilibrated"] == -1 and np.isnan(res["plain"]["tau_tunnel"])
    for key, seed, steps in (("walk", 71, 300), ("eq", 72, res["eq"]["n_meas"] + 10)):
        r = res[key]
        assert r["status"] == 0
        job = pt.pt_init(S, NT, L, dim, J, b, seed, walk=True)
        pt.pt_mcs(job, 10 if key == "eq" else 20)
        pt.pt_mcs(job, steps - (10 if key == "eq" else 20), measure=True)
        _, dis, nm = pt.pt_observables(job)
        _, _, tau, eq = pt.pt_tunnel_summary(pt.pt_get_walk(job)[2], steps)
        assert nm == r["n_meas"] and np.array_equal(r["disorder"], dis)
        assert r["tau_tunnel"] == tau and r["equilibrated"] == eq
        pt.pt_destroy(job)
    assert res["eq"]["equilibrated"] == 1 and res["eq"]["n_meas"] < 20000 - 10


def test_server_rejects_unguarded_stop(pt):
    srv = pt.pt_server_start(1 << 24, steps_per_round=3)
    J = W.couplings_pm_j(1, 4, 3, 1)
    b = W.geometric_betas(1.0, 2.0, 3)
    with pytest.raises(pt.PTError):
        pt.pt_server_submit(srv, 3, 4, 3, 1, b, J, 1, 10, 0, until_equilibrated=True)
    with pytest.raises(pt.PTError):
        pt.pt_server_submit(srv, 3, 4, 3, 1, b, J, 1, 10, 0, layout=0x40)
    pt.pt_server_stop(srv)


def test_server_reports_correlation_length(pt):
    """A request keeping the two-replica modes returns chi_SG(0), chi_SG(k_min)
    and xi per temperature, equal to the same job run alone; others NaN."""
    dim, L, NT, S = 3, 8, 4, 2
    J = W.couplings_pm_j(S, L, dim, 81)
    b = W.geometric_betas(0.8, 2.0, NT)
    srv = pt.pt_server_start(1 << 30, steps_per_round=9)
    t_m = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 5, 40, 10, modes=True)
    t_p = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 5, 40, 10)
    res = _wait(pt, srv, {"m": t_m, "p": t_p})
    pt.pt_server_stop(srv)
    assert np.isnan(res["p"]["correlation"]).all()
    job = pt.pt_init(S, NT, L, dim, J, b, 5, modes=True)
    pt.pt_mcs(job, 10)
    pt.pt_mcs(job, 30, measure=True)
    c0, ck, xi = pt.pt_correlation_length(job)
    got = res["m"]["correlation"]
    assert np.array_equal(got[:, 0], c0) and np.array_equal(got[:, 1], ck)
    assert np.array_equal(got[:, 2], xi, equal_nan=True)
    assert np.array_equal(res["m"]["disorder"], res["p"]["disorder"])


def test_server_measurement_interval(pt):
    """A request's measurement interval: the served result equals the job run
    alone with the same interval (Sec. 3 measures at intervals)."""
    dim, L, NT, S, sweeps, burn = 3, 8, 4, 2, 47, 9
    J = W.couplings_pm_j(S, L, dim, 82)
    b = W.geometric_betas(0.8, 2.0, NT)
    srv = pt.pt_server_start(1 << 30, steps_per_round=8)
    t = pt.pt_server_submit(srv, dim, L, NT, S, b, J, 6, sweeps, burn, measure_every=5, modes=True)
    r = _wait(pt, srv, {0: t})[0]
    pt.pt_server_stop(srv)
    job = pt.pt_init(S, NT, L, dim, J, b, 6, modes=True)
    pt.pt_set_measure_interval(job, 5)
    pt.pt_mcs(job, burn)
    pt.pt_mcs(job, sweeps - burn, measure=True)
    _, dis, nm = pt.pt_observables(job)
    assert r["n_meas"] == nm == len([t1 for t1 in range(burn + 1, sweeps + 1) if t1 % 5 == 0])
    assert np.array_equal(r["disorder"], dis)
    c0, ck, xi = pt.pt_correlation_length(job)
    assert np.array_equal(r["correlation"][:, 0], c0)


def test_server_cancel_leaves_other_results_unchanged(pt):
    """A queued and a running request are cancelled; every other request's
    result equals the same job run alone, bit for bit, and the cancelled ones
    report PT_ECANCELED (the failure-handling side of the served form)."""
    keep = {0: (3, 8, 4, 2, 40, 10, False, 0), 2: (3, 12, 5, 1, 30, 6, False, 1),
            4: (2, 16, 4, 2, 26, 8, True, 0)}
    long_run = (3, 16, 6, 1, 20000, 100, False, 0)   # cancelled while running
    queued = (3, 16, 4, 1, 50, 10, False, 0)         # cancelled while queued
    def nbytes(spec):
        dim, L, NT, S = spec[:4]
        return pt.pt_job_bytes(S, NT, L, dim, W.geometric_betas(0.6, 2.0, NT), layout=spec[7])
    # room for requests 0, 1 (the long one) and 2 together; 3 and 4 wait
    budget = nbytes(keep[0]) + nbytes(long_run) + nbytes(keep[2]) + 4096
    srv = pt.pt_server_start(budget, steps_per_round=2)
    specs = {0: keep[0], 1: long_run, 2: keep[2], 3: queued, 4: keep[4]}
    tickets = {}
    for n in range(5):
        dim, L, NT, S, sweeps, burn, hou, layout = specs[n]
        J, b, seed = _inputs(60 + n, specs[n])
        say(f"submit {specs[n]}")
        tickets[n] = pt.pt_server_submit(srv, dim, L, NT, S, b, J, seed, sweeps, burn, hou, layout)
    assert pt.pt_server_cancel(srv, tickets[3]) is True     # still queued
    t0 = time.time()
    while pt.pt_server_stats(srv)["rounds"] < 3:
        assert time.time() - t0 < 60, "no rounds"
        time.sleep(0.005)
    assert pt.pt_server_cancel(srv, tickets[1]) is True     # running
    res = _wait(pt, srv, tickets, timeout=180.0)
    stats = pt.pt_server_stats(srv)
    # a request that finished but was not polled yet cannot be cancelled
    J, b, seed = _inputs(70, keep[0])
    t_done = pt.pt_server_submit(srv, 3, 8, 4, 2, b, J, seed, 0, 0)
    t0 = time.time()
    while pt.pt_server_stats(srv)["completed"] < stats["completed"] + 1:
        assert time.time() - t0 < 60, "empty request did not finish"
        time.sleep(0.005)
    assert pt.pt_server_cancel(srv, t_done) is False
    assert pt.pt_server_poll(srv, t_done)["status"] == 0
    with pytest.raises(pt.PTError):
        pt.pt_server_cancel(srv, tickets[1])       # result already collected
    with pytest.raises(pt.PTError):
        pt.pt_server_cancel(srv, 10 ** 9)          # never issued
    pt.pt_server_stop(srv)
    assert res[1]["status"] == pt.PT_ECANCELED and res[3]["status"] == pt.PT_ECANCELED
    assert stats["cancelled"] == 2 and stats["queued"] == 0
    for n, spec in keep.items():
        dis, nm = _alone(pt, 60 + n, spec)
        assert res[n]["status"] == 0, (spec, res[n]["status"])
        assert res[n]["n_meas"] == nm == spec[4] - spec[5]
        assert np.array_equal(res[n]["disorder"], dis), spec
