"""Throughput benchmark: parallel-tempering Monte Carlo of the 3D +-J
Edwards-Anderson spin glass on one MI355X.

Workload (default "3d_l16"): L = 16 periodic, 1000 disorder samples x 2
replica sets x 32 temperatures (geometric T in [0.9, 2.0]), int8 spins and
couplings.  One step = one Monte Carlo step of the whole path: a checkerboard
Metropolis sweep of all 64,000 lattices, one replica-exchange pass and one
measurement (E, overlap moments).  All inputs are resident on the GPU before
the timed region.  Steps run fused (the persistent kernel, one sample per
workgroup resident in LDS, `--chunk` steps per launch); the same steps with
one launch per kernel are timed afterwards for comparison.

Also measured (each its own JSON object): the 2D L = 64 workload with a
Houdayer move every step (its own roofline); the time split into Metropolis,
Houdayer, exchange and measurement in t_update units of Eq. (11), per kernel
of the plain form and as differences of fused runs; the replica walk and the
two-replica modes; the batched form (2000 jobs of uneven L in one
graph-replayed persistent launch, int8 and packed layouts, against one job
per launch) and the served form (Poisson arrivals of mixed-L requests at 70%
of the measured capacity, HBM-budget admission; p50/p99 latency and
delivered flips/ns).

Prints one JSON line: spin flips/ns over the timed steps, the fused kernel's
roofline position (VALU-bound: integer issue slots), and the CPU oracle's
rate on a bounded sample of the same workload, one sample per process on the
host's cores (the single-core rate beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X VALU peak: 256 CUs x 128 32-bit lanes per clock x 2.4 GHz = 78.6 T
# lane-operations/s, the rate behind the published 157.3 TFLOP/s fp32 vector
# figure (an FMA counts two flops).  An instruction-rate probe measured on the
# GPU 0.72-0.79 of this for plain integer ops (v_add_u32, v_bitop3_b32) and half
# of it for the 32x32->64-bit multiply (v_mad_u64_u32), which therefore costs
# two issue slots (profiles/valu_issue_rates_gfx950.md).
PEAK_VALU_OPS = 256 * 128 * 2.4e9
# Algorithmic work per attempted flip, in issue slots: the site's share of one
# Philox4x32-10 call (10 rounds x 2 multiplies x 2 slots + 10 x 2 three-input
# xors, over 4 words = 15) plus the threshold compare (1).  The bit-sliced
# local field and classification (amortised over 16-32 sites of a word) are
# not counted.
OPS_PER_FLIP = 16
# The same for a Gaussian-coupling site in 2D: the Philox share (15), the four
# bond terms of its integer local field (4) and the threshold compare (1).
GAUSS_OPS_PER_FLIP = 20
# HBM bytes per launch of the fused kernel, keyed by (workload, layout,
# variant: 1 Houdayer | 2 measure), from rocprofv3 FETCH_SIZE / WRITE_SIZE
# scaled by a plain copy's readings (profiles/*_hbm_traffic.md).  Every
# sample is loaded once and stored once per launch, so the bytes do not depend
# on the number of steps a launch runs.  Entries are removed when the kernel
# changes until the counters are taken again.
TRAFFIC_PER_LAUNCH = {("3d_l16", "int8", 2): 572715904}
# The fused Gaussian kernel on the 2d_l64_gauss workload, keyed by steps per
# launch: it also re-reads the samples' coupling groups every step (those
# that miss the L2), so its bytes grow with the step count
# (profiles/k_gfused_2d_l64_gauss_hbm_traffic.md).
GAUSS_TRAFFIC_PER_LAUNCH = {100: 1582418816}


def _oracle_steps(args):
    """Worker: `n` oracle Monte Carlo steps of one sample (all replicas) of
    workload `name`; returns the seconds they took."""
    name, key, n = args
    import oracle
    from paper_2003_04621_amd import workloads as W
    wl = W.workload(name)
    J = wl.couplings()[[key]]
    ref = oracle.OracleJob(1, wl.replicas, wl.L, wl.dim, J, wl.betas, wl.seed, sample_keys=[key])
    t = time.perf_counter()
    ref.mcs(n, houdayer=wl.houdayer, measure=True)
    return time.perf_counter() - t


def cpu_baseline(wl, budget_s: float, cores: int):
    """The oracle on the host: one sample per process on `cores` processes at
    once (the paper's multi-threaded CPU comparison runs one disorder sample
    per thread), each for the same number of steps, about `budget_s` seconds;
    the single-process rate of the same sample is reported beside it.  Runs
    before anything touches the GPU (the worker processes are forked)."""
    import multiprocessing as mp
    per_sample_step = 2 * wl.replicas * wl.N
    dt2 = _oracle_steps((wl.name, 0, 2))
    n = max(1, int(budget_s / max(dt2 / 2, 1e-6)))
    one = _oracle_steps((wl.name, 0, n))
    single = per_sample_step * n / one / 1e9
    cores = max(1, min(cores, wl.samples))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        times = pool.map(_oracle_steps, [(wl.name, k, n) for k in range(cores)])
    wall = max(times)  # the processes run at the same time; the slowest sets the rate
    return {"value": round(per_sample_step * n * cores / wall / 1e9, 6), "unit": "flips/ns",
            "cores": cores, "kind": "oracle",
            "sample": f"samples 0..{cores - 1} of {wl.samples} (all {2 * wl.replicas} replicas), "
                      f"one per process on {cores} host cores at once, {n} Monte Carlo steps each, "
                      f"slowest process {wall:.1f} s",
            "single_core": {"value": round(single, 6), "unit": "flips/ns", "cores": 1,
                            "sample": f"sample 0, {n} steps, {one:.1f} s"},
            "host_cpus": os.cpu_count()}


def batched_mix(pt, torch, W, args):
    """Jobs of uneven size in one persistent launch: 2000 jobs of one sample,
    400 each at L = 8, 12, 16, 24, 32, 24 temperatures (geometric T in
    [0.9, 2.0]), sweep + exchange steps replayed from a captured hipGraph,
    launch shape chosen by the autotuner; int8 and packed spin layouts."""
    Ls = [8, 12, 16, 24, 32]
    per_L = args.batch_jobs // len(Ls)
    NT = 24
    betas = W.geometric_betas(0.9, 2.0, NT)
    out = {"workload": f"{per_L * len(Ls)} jobs x 1 sample x 2 x {NT} temperatures, 3D +-J, "
                       f"L in {Ls} (1:1:1:1:1)", "steps": args.batch_steps}
    for layout_name, layout in (("int8", pt.PT_LAYOUT_INT8), ("packed", pt.PT_LAYOUT_PACKED)):
        jobs = []
        n = 0
        for L in Ls:
            for _ in range(per_L):
                J = W.couplings_pm_j(1, L, 3, 1000 + n)
                jobs.append(pt.pt_init(1, NT, L, 3, J, betas, 2000 + n, layout=layout))
                n += 1
        flips = sum(2 * NT * j.N for j in jobs)
        batch = pt.pt_batch_create(jobs)
        cfg = pt.pt_batch_tune(batch, 3, cache_path=args.tune_cache)
        pt.pt_batch_run(batch, args.batch_chunk, graph=True)        # capture + warm-up
        torch.cuda.synchronize()
        reps = max(1, args.batch_steps // args.batch_chunk)
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            pt.pt_batch_run(batch, args.batch_chunk, graph=True)
            b.record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        value = flips * args.batch_chunk * reps / dt / 1e9
        achieved = OPS_PER_FLIP * flips * args.batch_chunk / (launch_ms * 1e-3) / 1e12
        # the same steps, one job per launch (no batch, no graph)
        plain_steps = 2
        for j in jobs:
            pt.pt_mcs(j, 1)              # each job's own launch list, built once
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(plain_steps):
            for j in jobs:
                pt.pt_mcs(j, 1)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        plain = flips * plain_steps / dtp / 1e9
        out[layout_name] = {
            "value": round(value, 2), "unit": "flips/ns", "tuned_config": list(cfg),
            "graph_replays": reps, "steps_per_replay": args.batch_chunk,
            "launch_ms": round(launch_ms, 3),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                         "peak": round(PEAK_VALU_OPS / 1e12, 3), "unit": "TOP/s",
                         "frac": round(achieved / (PEAK_VALU_OPS / 1e12), 4)},
            "plain_one_job_per_launch": round(plain, 3),
            "speedup_vs_plain": round(value / plain, 1)}
        pt.pt_batch_destroy(batch)
        for j in jobs:
            pt.pt_destroy(j)
        del jobs
    return out


def _requests(W, rng, n, seed0, Ls=(16, 24, 32, 48), nt=(16, 48), sweeps=(1e3, 1e4)):
    """n requests of the served mix: 3D +-J, one sample, L uniform in
    {16, 24, 32, 48}, 16..48 temperatures, 10^3..10^4 steps (log-uniform),
    half of them burn-in (other ranges as given)."""
    Ls = rng.choice(list(Ls), size=n)
    NTs = rng.integers(nt[0], nt[1] + 1, size=n)
    sweeps = np.exp(rng.uniform(np.log(sweeps[0]), np.log(sweeps[1]), size=n)).astype(int)
    reqs = []
    for i in range(n):
        L, NT = int(Ls[i]), int(NTs[i])
        reqs.append(dict(L=L, NT=NT, J=W.couplings_pm_j(1, L, 3, seed0 + i),
                         betas=W.geometric_betas(0.9, 2.0, NT), seed=seed0 + 2000 + i,
                         sweeps=int(sweeps[i]), flips=2 * NT * L ** 3 * int(sweeps[i])))
    return reqs


def _serve(pt, args, reqs, arrivals, until_eq=False):
    """Submits reqs[i] at arrivals[i] seconds and waits for every result.
    Also returns (seconds, flips) on the server's clock at the moment the
    last request was admitted: until then the queue was never empty.  With
    until_eq the requests keep the replica walk and end as soon as their
    round trips pass the logarithmic-binning check (their sweeps an upper
    bound)."""
    srv = pt.pt_server_start(args.serve_budget << 20, steps_per_round=args.serve_round)
    n = len(reqs)
    tickets, results = {}, {}
    saturated = None
    t0 = time.perf_counter()
    t_note = t0
    i = 0
    while len(results) < n:
        now = time.perf_counter() - t0
        if now + t0 - t_note > 15.0:
            t_note = now + t0
            print(f"# served: {len(results)}/{n} done, {i} submitted, {now:.0f} s",
                  file=sys.stderr, flush=True)
        while i < n and arrivals[i] <= now:
            r = reqs[i]
            tickets[i] = pt.pt_server_submit(srv, 3, r["L"], r["NT"], 1, r["betas"], r["J"],
                                             r["seed"], r["sweeps"], r["sweeps"] // 2,
                                             walk=until_eq, until_equilibrated=until_eq)
            i += 1
        if saturated is None and i == n:
            st = pt.pt_server_stats(srv)
            if st["admitted"] >= n:
                saturated = (st["uptime_s"], st["flips"])
        for k in list(tickets):
            res = pt.pt_server_poll(srv, tickets[k])
            if res is not None:
                results[k] = res
                del tickets[k]
        time.sleep(0.002)
    stats = pt.pt_server_stats(srv)
    pt.pt_server_stop(srv)
    span = max(r["t_done"] for r in results.values()) - min(r["t_submit"] for r in results.values())
    lat = np.array([results[k]["t_done"] - results[k]["t_submit"] for k in range(n)])
    bad = sum(1 for r in results.values() if r["status"] != 0)
    if until_eq:
        return stats, span, lat, bad, saturated, results
    return stats, span, lat, bad, saturated


def served(pt, torch, W, args):
    """Served form.  Capacity is measured first: a burst of requests of the
    mix submitted at once, more than the HBM budget admits together; flips
    per second while the queue is non-empty (until the last request is
    admitted).  Then Poisson arrivals at `serve_load` of that capacity;
    p50/p99 of completion minus submission and the flips/ns delivered."""
    rng = np.random.default_rng(args.serve_seed)
    burst = _requests(W, rng, args.serve_burst, 9000)
    stats_b, span_b, _, bad_b, sat = _serve(pt, args, burst, np.zeros(len(burst)))
    t_sat, flips_sat = sat if sat and sat[0] > 0 else (span_b, stats_b["flips"])
    capacity = flips_sat / t_sat / 1e9
    reqs = _requests(W, rng, args.serve_requests, 5000)
    mean_flips = float(np.mean([r["flips"] for r in reqs]))
    lam = args.serve_load * capacity * 1e9 / mean_flips       # jobs per second
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
    stats, span, lat, bad, _ = _serve(pt, args, reqs, arrivals)
    # time to an equilibrated result: the same kind of requests keeping the
    # replica walk, each ending once its round trips pass the binning check
    # (Sec. 2.3), at the same arrival rate
    eq = None
    if args.serve_eq_requests > 0:
        # smaller lattices than the mix above: at T_min = 0.9 the L >= 16
        # requests of that mix do not pass the check within 1e4 sweeps
        lo, hi = (float(x) for x in args.serve_eq_sweeps.split(","))
        reqs_e = _requests(W, rng, args.serve_eq_requests, 7000, Ls=(8, 12, 16), nt=(12, 24),
                           sweeps=(lo, hi))
        mean_e = float(np.mean([r["flips"] for r in reqs_e]))
        lam_e = args.serve_load * capacity * 1e9 / mean_e
        arr_e = np.cumsum(rng.exponential(1.0 / lam_e, size=len(reqs_e)))
        st_e, span_e, lat_e, bad_e, _, res_e = _serve(pt, args, reqs_e, arr_e, until_eq=True)
        done_eq = [k for k, r in res_e.items() if r["equilibrated"] == 1]
        used = [(reqs_e[k]["sweeps"] // 2 + res_e[k]["n_meas"]) / reqs_e[k]["sweeps"] for k in res_e]
        eq = {"workload": f"{len(reqs_e)} requests, Poisson arrivals at {lam_e:.2f}/s, 3D +-J, "
                          "one sample, L in {8,12,16}, 12-24 temperatures in [0.9, 2.0], replica "
                          "walk kept, each ending once its round trips pass the logarithmic-"
                          f"binning check (Sec. 2.3), at most {lo:.0e}-{hi:.0e} steps (half burn-in)",
              "requests": len(reqs_e), "equilibrated": len(done_eq),
              "p50_latency_s": round(float(np.percentile(lat_e, 50)), 4),
              "p99_latency_s": round(float(np.percentile(lat_e, 99)), 4),
              "p50_latency_equilibrated_s": (round(float(np.percentile(
                  [res_e[k]["t_done"] - res_e[k]["t_submit"] for k in done_eq], 50)), 4)
                  if done_eq else None),
              "mean_fraction_of_sweeps_run": round(float(np.mean(used)), 4),
              "value": round(st_e["flips"] / span_e / 1e9, 2), "unit": "flips/ns",
              "failed": bad_e}
    return {"workload": f"{len(reqs)} requests, Poisson arrivals at {lam:.2f}/s "
                        f"({args.serve_load:.0%} of the measured capacity), 3D +-J, one sample, "
                        "L in {16,24,32,48}, 16-48 temperatures, 1e3-1e4 steps (half burn-in)",
            "capacity": {"value": round(capacity, 2), "unit": "flips/ns",
                         "burst_requests": len(burst), "saturated_seconds": round(t_sat, 3),
                         "burst_seconds": round(span_b, 3),
                         "burst_flips_per_ns": round(stats_b["flips"] / span_b / 1e9, 2)},
            "hbm_budget_mib": args.serve_budget, "steps_per_round": args.serve_round,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "value": round(stats["flips"] / span / 1e9, 2), "unit": "flips/ns",
            "seconds": round(span, 3),
            "busy_fraction": round(stats["busy_s"] / span, 3),
            "peak_concurrent_jobs": int(stats["peak_jobs"]),
            "peak_admitted_mib": round(stats["peak_bytes"] / 2 ** 20, 1),
            "failed": bad + bad_b,
            "until_equilibrated": eq}


def fused_run(pt, torch, job, wl, K, chunk, houdayer, measure, layout_name, multi=False):
    """K fused steps of `job` in launches of `chunk` steps; the rate over the
    host clock and the kernel's roofline position from the HIP-event duration
    of its full-length launches (events on the job's stream)."""
    stream = torch.cuda.current_stream()
    chunk = max(1, min(chunk, K))
    starts = list(range(0, K, chunk))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in starts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (a, b), st in zip(ev, starts):
        a.record(stream)
        pt.pt_mcs(job, min(chunk, K - st), houdayer=houdayer, measure=measure, multi=multi)
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launch_ms = float(np.mean([a.elapsed_time(b) for (a, b), st in zip(ev, starts)
                               if K - st >= chunk]))
    achieved = OPS_PER_FLIP * wl.flips_per_sweep * chunk / (launch_ms * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12
    feat = (1 if houdayer else 0) | (2 if measure else 0)
    if pt.pt_get_plan(job, houdayer=houdayer, measure=measure, multi=multi)["mode"] == 3:
        feat |= 4  # split samples: the launch runs the split variant
    return elapsed, {
        "bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": TRAFFIC_PER_LAUNCH.get((wl.name, layout_name, feat)),
        "kernel": f"k_batch<{wl.dim}, {feat}> ({chunk} steps per launch)",
        "launch_ms": round(launch_ms, 4)}


def settle_gpu(pt, torch, scratch, wl, seconds):
    """An untimed busy period right before the timed region.  The GPU raises
    its clock over the first tens of milliseconds of sustained load and lowers
    it again within a tenth of a second of idling (on one box, 20-step
    launches of the 3D L=16 workload took 2.86 ms after an idle period,
    falling to 2.55 ms after about 20 ms of back-to-back work, and 2.83 ms
    again after 0.1 s of host-side set-up), so a scratch job of the same
    workload runs fused steps for `seconds`, a few launches queued ahead so
    that the GPU never idles between them.  The timed job is not touched: it
    gets exactly the requested warm-up steps.  The caller frees the scratch
    job after the timed region (freeing it here would idle the GPU)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            pt.pt_mcs(scratch, 20, houdayer=wl.houdayer, measure=True)
        torch.cuda.synchronize()
    return time.perf_counter() - t0


def phase_split(pt, torch, wl, layout, steps, warmup):
    """Time per phase of a Monte Carlo step in the paper's four-part
    breakdown (Metropolis, Houdayer, replica exchange, measurement), as
    t_update of Eq. (11): kernel time per replica and spin.  Plain form: each
    phase is its own launch (pt_sweep, pt_houdayer, pt_exchange, pt_measure),
    timed with HIP events on the job's stream.  Fused form: the differences
    between fused runs with and without the Houdayer move and the
    measurement (the sweep and the exchange share one kernel)."""
    stream = torch.cuda.current_stream()
    init = pt.pt_init_gauss if getattr(wl, "gauss", False) else pt.pt_init
    job = init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas, wl.seed, layout=layout)
    norm = wl.flips_per_sweep  # N_T N_C N_R N_B L^d
    pt.pt_mcs(job, warmup, houdayer=wl.houdayer, measure=True)
    phases = [("metropolis", lambda: pt.pt_sweep(job, 1))]
    if wl.houdayer:
        phases.append(("houdayer", lambda: pt.pt_houdayer(job)))
    phases += [("exchange", lambda: pt.pt_exchange(job)), ("measure", lambda: pt.pt_measure(job))]
    ev = {name: [] for name, _ in phases}
    torch.cuda.synchronize()
    for _ in range(steps):
        for name, fn in phases:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            ev[name].append((a, b))
    torch.cuda.synchronize()
    plain = {}
    total = 0.0
    for name, _ in phases:
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev[name]]))
        total += ms
        plain[name] = {"ms_per_step": round(ms, 5), "t_update_ns": round(ms * 1e6 / norm, 7)}
    for name in plain:
        plain[name]["share"] = round(plain[name]["ms_per_step"] / total, 4)

    def fused_ms(hou, meas, n):
        pt.pt_mcs(job, 2, houdayer=hou, measure=meas)       # work list built, warm
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        pt.pt_mcs(job, n, houdayer=hou, measure=meas)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    n = max(steps, 50)
    base = fused_ms(False, False, n)
    fused = {"metropolis+exchange": {"ms_per_step": round(base, 5),
                                     "t_update_ns": round(base * 1e6 / norm, 7)}}
    with_meas = fused_ms(wl.houdayer, True, n)
    if wl.houdayer:
        with_hou = fused_ms(True, False, n)
        d = with_hou - base
        fused["houdayer"] = {"ms_per_step": round(d, 5), "t_update_ns": round(d * 1e6 / norm, 7),
                             "us_per_cluster_pass": round(d * 1e3, 3),
                             "ns_per_pair": round(d * 1e6 / (wl.samples * wl.replicas), 3)}
        d = with_meas - with_hou
    else:
        d = with_meas - base
    fused["measure"] = {"ms_per_step": round(d, 5), "t_update_ns": round(d * 1e6 / norm, 7)}
    pt.pt_destroy(job)
    return {"workload": wl.name, "steps": steps, "plain": plain, "fused": fused,
            "unit_note": "t_update_ns = kernel ns per step / (samples x 2 sets x N_T x L^d), Eq. (11)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="3d_l16")
    ap.add_argument("--layout", choices=["int8", "packed"], default="int8")
    ap.add_argument("--chunk", type=int, default=500, help="steps per fused launch")
    ap.add_argument("--plain-steps", type=int, default=300,
                    help="steps re-timed with one launch per kernel (0: skip)")
    ap.add_argument("--houdayer-steps", type=int, default=1000,
                    help="steps of the 2D L=64 Houdayer workload (0: skip)")
    ap.add_argument("--multi-steps", type=int, default=1000,
                    help="steps of the 2D L=64 workload with multi-cluster moves (0: skip)")
    ap.add_argument("--gauss-steps", type=int, default=100,
                    help="steps of the 2D L=64 Gaussian-coupling workload (0: skip)")
    ap.add_argument("--phase-steps", type=int, default=100,
                    help="steps of the per-phase time split (0: skip)")
    ap.add_argument("--walk-steps", type=int, default=1000,
                    help="steps of the same workload with the replica walk kept (0: skip)")
    ap.add_argument("--modes-steps", type=int, default=1000,
                    help="steps of the same workload measuring the two-replica modes (0: skip)")
    ap.add_argument("--settle", type=float, default=1.0,
                    help="seconds of untimed work on a scratch job before timing (GPU clock)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="host processes of the CPU baseline (at most the host's CPUs)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-jobs", type=int, default=2000)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-chunk", type=int, default=100)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-burst", type=int, default=900, help="requests of the capacity burst")
    ap.add_argument("--serve-budget", type=int, default=2048, help="MiB")
    ap.add_argument("--serve-round", type=int, default=100)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-seed", type=int, default=31)
    ap.add_argument("--serve-eq-sweeps", default="1e4,5e4",
                    help="bounds of the equilibrium-stopped requests' steps (log-uniform)")
    ap.add_argument("--serve-eq-requests", type=int, default=500,
                    help="requests of the run that stops each job at equilibrium (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path shards by disorder sample and "
              "has no multi-GPU run; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2003_04621_amd import workloads as W
    wl = W.workload(args.workload)
    # the CPU baseline first: its worker processes are forked before the GPU is touched
    cpu = None
    if not args.no_cpu:
        print(f"# CPU oracle baseline ({args.cpu_cores} processes)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_seconds, min(args.cpu_cores, os.cpu_count() or 1))

    import torch
    from paper_2003_04621_amd import pt

    layout = pt.PT_LAYOUT_PACKED if args.layout == "packed" else pt.PT_LAYOUT_INT8
    torch.cuda.set_device(0)
    job = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas, wl.seed,
                     layout=layout)
    scratch = None
    if args.settle > 0:
        scratch = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas,
                             wl.seed + 1, layout=layout)
    flips_per_step = wl.flips_per_sweep
    print(f"# workload {wl.name}: S={wl.samples} NT={wl.replicas} L={wl.L} d={wl.dim} "
          f"layout={args.layout}; warmup {args.warmup}", file=sys.stderr, flush=True)
    pt.pt_mcs(job, args.warmup, houdayer=wl.houdayer, measure=True)
    torch.cuda.synchronize()
    # the clock-settling work runs right before the timed region: an idle
    # tenth of a second is enough for the clock to drop again
    settled = settle_gpu(pt, torch, scratch, wl, args.settle) if scratch is not None else 0.0

    K = args.steps
    elapsed, roofline = fused_run(pt, torch, job, wl, K, args.chunk, wl.houdayer, True, args.layout)
    value = flips_per_step * K / elapsed / 1e9
    if scratch is not None:
        pt.pt_destroy(scratch)

    # the same steps as separate per-step launches, for the fused/plain ratio
    plain = None
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        tp = time.perf_counter()
        pt.pt_mcs(job, args.plain_steps, houdayer=wl.houdayer, measure=True, plain=True)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        plain = {"value": round(flips_per_step * args.plain_steps / dtp / 1e9, 2),
                 "unit": "flips/ns", "steps": args.plain_steps,
                 "form": "one launch per kernel per step"}
    counters = pt.pt_get_counters(job)
    total = args.warmup + K + max(args.plain_steps, 0)
    assert counters["t"] == total and counters["n_meas"] == total, counters
    _, dis, n_meas = pt.pt_observables(job)
    pt.pt_destroy(job)

    # the 2D L = 64 workload with a Houdayer move every step
    hou = None
    if args.houdayer_steps > 0 and wl.name != "2d_l64":
        wh = W.workload("2d_l64")
        print(f"# workload {wh.name} with Houdayer moves", file=sys.stderr, flush=True)
        hj = pt.pt_init(wh.samples, wh.replicas, wh.L, wh.dim, wh.couplings(), wh.betas, wh.seed,
                        layout=layout)
        pt.pt_mcs(hj, args.warmup, houdayer=True, measure=True)
        el_h, roof_h = fused_run(pt, torch, hj, wh, args.houdayer_steps, args.chunk, True, True,
                                 args.layout)
        _, dis_h, _ = pt.pt_observables(hj)
        pt.pt_destroy(hj)
        hou = {"workload": f"{wh.name}: 2D +-J, L={wh.L}, {wh.samples} samples x 2 x {wh.replicas} "
                           "temperatures (power-law ladder, T in [0.2, 1.6]), sweep + Houdayer + "
                           "exchange + measure",
               "value": round(wh.flips_per_sweep * args.houdayer_steps / el_h / 1e9, 2),
               "unit": "flips/ns", "steps": args.houdayer_steps, "roofline": roof_h,
               "roofline_note": "achieved counts the Metropolis work only (16 slots per flip); "
                                "the Houdayer move is extra work in the same launches",
               "e_coldest": round(float(dis_h[0, 0]), 6)}

    # the same 2D workload with the multi-cluster variant of the Houdayer move
    multi = None
    if args.multi_steps > 0:
        wh = W.workload("2d_l64")
        print(f"# workload {wh.name} with multi-cluster Houdayer moves", file=sys.stderr, flush=True)
        mj = pt.pt_init(wh.samples, wh.replicas, wh.L, wh.dim, wh.couplings(), wh.betas, wh.seed,
                        layout=layout)
        pt.pt_mcs(mj, args.warmup, houdayer=True, measure=True, multi=True)
        el_m, roof_m = fused_run(pt, torch, mj, wh, args.multi_steps, args.chunk, True, True,
                                 args.layout, multi=True)
        _, dis_m, _ = pt.pt_observables(mj)
        pt.pt_destroy(mj)
        multi = {"workload": f"{wh.name} with every q = -1 cluster of a pair exchanged "
                             "independently (multi-cluster variant)",
                 "value": round(wh.flips_per_sweep * args.multi_steps / el_m / 1e9, 2),
                 "unit": "flips/ns", "steps": args.multi_steps, "roofline": roof_m,
                 "e_coldest": round(float(dis_m[0, 0]), 6)}

    # the 2D Gaussian-coupling workload (Sec. 4.2's second model; per-step kernels)
    gauss = None
    if args.gauss_steps > 0:
        wg = W.workload("2d_l64_gauss")
        print(f"# workload {wg.name}", file=sys.stderr, flush=True)
        gj = pt.pt_init_gauss(wg.samples, wg.replicas, wg.L, wg.dim, wg.couplings(), wg.betas,
                              wg.seed)
        pt.pt_mcs(gj, min(args.warmup, 20), houdayer=True, measure=True)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tg = time.perf_counter()
        ga.record(stream)
        pt.pt_mcs(gj, args.gauss_steps, houdayer=True, measure=True)
        gb.record(stream)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - tg
        g_ms = ga.elapsed_time(gb)
        # the same steps as one launch per kernel per step
        gplain = 20
        tp = time.perf_counter()
        pt.pt_mcs(gj, gplain, houdayer=True, measure=True, plain=True)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        _, dis_g, _ = pt.pt_observables(gj)
        pt.pt_destroy(gj)
        g_achieved = GAUSS_OPS_PER_FLIP * wg.flips_per_sweep * args.gauss_steps / (g_ms * 1e-3) / 1e12
        gauss = {"workload": f"{wg.name}: 2D Gaussian couplings (standard normal on the 2^-16 "
                             f"grid), L={wg.L}, {wg.samples} samples x 2 x {wg.replicas} "
                             "temperatures, sweep + Houdayer + exchange + measure",
                 "value": round(wg.flips_per_sweep * args.gauss_steps / dtg / 1e9, 2),
                 "unit": "flips/ns", "steps": args.gauss_steps,
                 "form": f"fused, {args.gauss_steps} steps in one launch of k_gfused<2, true, true>",
                 "roofline": {"bound": "alu", "achieved": round(g_achieved, 3),
                              "peak": round(PEAK_VALU_OPS / 1e12, 3), "unit": "TOP/s",
                              "frac": round(g_achieved / (PEAK_VALU_OPS / 1e12), 4),
                              "traffic": GAUSS_TRAFFIC_PER_LAUNCH.get(args.gauss_steps),
                              "kernel": "k_gfused<2, true, true>", "launch_ms": round(g_ms, 4),
                              "ops_per_flip": GAUSS_OPS_PER_FLIP},
                 "plain_form": {"value": round(wg.flips_per_sweep * gplain / dtp / 1e9, 2),
                                "unit": "flips/ns", "steps": gplain,
                                "form": "one launch per kernel per step"},
                 "e_coldest": round(float(dis_g[0, 0]), 6)}

    # the four-part time split (Sec. 4.5) of the workloads
    split = None
    if args.phase_steps > 0:
        print("# per-phase split", file=sys.stderr, flush=True)
        split = [phase_split(pt, torch, wl, layout, args.phase_steps, 20)]
        for other in ("2d_l64", "2d_l64_gauss"):
            if wl.name != other:
                split.append(phase_split(pt, torch, W.workload(other), layout, args.phase_steps, 20))

    # the same workload with the replica walk and its round trips kept
    walk = None
    if args.walk_steps > 0:
        print("# replica walk kept", file=sys.stderr, flush=True)
        wj = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas, wl.seed,
                        layout=layout, walk=True)
        pt.pt_mcs(wj, args.warmup, houdayer=wl.houdayer, measure=True)
        torch.cuda.synchronize()
        tw = time.perf_counter()
        for st in range(0, args.walk_steps, args.chunk):
            pt.pt_mcs(wj, min(args.chunk, args.walk_steps - st), houdayer=wl.houdayer, measure=True)
        torch.cuda.synchronize()
        dtw = time.perf_counter() - tw
        passes = pt.pt_get_counters(wj)["u"]
        trips = pt.pt_get_walk(wj)[2]
        _, _, tau, eq = pt.pt_tunnel_summary(trips, passes)
        walk = {"value": round(flips_per_step * args.walk_steps / dtw / 1e9, 2), "unit": "flips/ns",
                "steps": args.walk_steps, "passes": passes,
                "round_trips": int(trips[..., 0].sum()),
                "tau_tunnel": None if np.isnan(tau) else round(tau, 3),
                "equilibrated": eq}
        pt.pt_destroy(wj)

    # the same workload measuring the two-replica modes at every step
    modes = None
    if args.modes_steps > 0:
        print("# two-replica modes measured", file=sys.stderr, flush=True)
        mj = pt.pt_init(wl.samples, wl.replicas, wl.L, wl.dim, wl.couplings(), wl.betas, wl.seed,
                        layout=layout, modes=True)
        pt.pt_mcs(mj, args.warmup, houdayer=wl.houdayer)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        for st in range(0, args.modes_steps, args.chunk):
            pt.pt_mcs(mj, min(args.chunk, args.modes_steps - st), houdayer=wl.houdayer, measure=True)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - tm
        c0, ck, xi = pt.pt_correlation_length(mj)
        # the same job measuring every 10th step, as measurements usually are
        pt.pt_set_measure_interval(mj, 10)
        torch.cuda.synchronize()
        tm10 = time.perf_counter()
        for st in range(0, args.modes_steps, args.chunk):
            pt.pt_mcs(mj, min(args.chunk, args.modes_steps - st), houdayer=wl.houdayer, measure=True)
        torch.cuda.synchronize()
        dtm10 = time.perf_counter() - tm10
        modes = {"value": round(flips_per_step * args.modes_steps / dtm / 1e9, 2), "unit": "flips/ns",
                 "value_every_10": round(flips_per_step * args.modes_steps / dtm10 / 1e9, 2),
                 "steps": args.modes_steps,
                 "chi_sg_coldest": round(float(c0[0]), 4), "chi_sg_kmin_coldest": round(float(ck[0]), 4),
                 "xi_coldest": None if np.isnan(xi[0]) else round(float(xi[0]), 4),
                 "xi_hottest": None if np.isnan(xi[-1]) else round(float(xi[-1]), 4)}
        pt.pt_destroy(mj)

    batched = None
    if not args.no_batched:
        print("# batched form", file=sys.stderr, flush=True)
        batched = batched_mix(pt, torch, W, args)
    serve = None
    if not args.no_served:
        print("# served form", file=sys.stderr, flush=True)
        serve = served(pt, torch, W, args)
    out = {
        "metric": "spin flips/ns (1 GPU)", "value": round(value, 2), "unit": "flips/ns",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": wl.name, "dim": wl.dim, "L": wl.L, "samples": wl.samples,
                   "replica_sets": 2, "temperatures": wl.replicas,
                   "T_range": [round(1 / wl.betas[0], 6), round(1 / wl.betas[-1], 6)],
                   "spin_layout": args.layout,
                   "step": "sweep+houdayer+exchange+measure" if wl.houdayer
                   else "sweep+exchange+measure"},
        "roofline": roofline,
        "gpu_settle_s": round(settled, 3),
        "cpu_baseline": cpu,
        "plain_form": plain,
        "houdayer_2d": hou,
        "multicluster_2d": multi,
        "gauss_2d": gauss,
        "phase_split": split,
        "replica_walk": walk,
        "modes": modes,
        "batched": batched,
        "served": serve,
        "e_coldest": round(float(dis[0, 0]), 6), "binder_coldest": round(float(dis[0, 5]), 6),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
