"""Host-side planning of the fused kernels (no GPU needed): which workgroup
plan a job shape gets, that every plan fits the 160 KiB of LDS, that split
plans cover every configuration exactly once, and the device-byte bound the
request server admits by."""
import numpy as np
import pytest

from paper_2003_04621_amd import pt

LDS_BYTES = 160 * 1024
SHAPES = [(d, L, NT) for d in (2, 3) for L in range(4, 65, 4) for NT in (2, 3, 8, 16, 24, 33, 48, 96)]


@pytest.fixture(scope="module")
def lib():
    return pt.lib()


@pytest.mark.parametrize("houdayer,measure", [(False, False), (False, True), (True, True)])
def test_plans_fit_and_cover(lib, houdayer, measure):
    for d, L, NT in SHAPES:
        p = pt.pt_plan_query(d, L, NT, houdayer=houdayer, measure=measure)
        mode, parts, per, lds = p["mode"], p["parts"], p["per_part"], p["lds_bytes"]
        assert lds <= LDS_BYTES - 512, (d, L, NT, p)
        if mode in (0, 1):
            assert parts == 1 and per == 2 * NT
        elif mode == 2:
            assert parts == 2 and per == NT and not measure and not houdayer
        elif mode == 3:
            assert not houdayer and 1 <= parts <= 64
            assert parts * per >= 2 * NT and (parts - 1) * per < 2 * NT
        else:
            assert mode == -1 and lds == 0
        if houdayer:
            assert mode in (1, -1)
        else:
            assert mode != -1, (d, L, NT, p)    # every non-Houdayer shape has a fused plan


def test_resident_plans_are_monotone_in_replicas(lib):
    for d in (2, 3):
        for L in range(4, 65, 4):
            fits = [pt.pt_plan_query(d, L, NT, measure=True)["mode"] == 0 for NT in range(2, 65)]
            # once both sets stop fitting, they never fit again for more temperatures
            assert fits == sorted(fits, reverse=True), (d, L)


def test_plain_flag_and_known_shapes(lib):
    assert pt.pt_plan_query(3, 16, 32, measure=True, plain=True)["mode"] == -1
    # 3D L=16, 32 temperatures: spins 32768 B, couplings 3072 B, energies, maps,
    # thresholds, moments, exchange randoms and the exchange decisions as bits;
    # four such workgroups fit one CU's 160 KiB of LDS
    p = pt.pt_plan_query(3, 16, 32, measure=True)
    assert p == {"mode": 0, "parts": 1, "per_part": 64, "lds_bytes": 40056}
    assert 4 * p["lds_bytes"] <= 160 * 1024
    # keeping the replica walk adds its words (2 per slot) and the launch's
    # round-trip sums (32 x 3 64-bit)
    w = pt.pt_plan_query(3, 16, 32, measure=True, walk=True)
    assert w == {"mode": 0, "parts": 1, "per_part": 64,
                 "lds_bytes": 40056 + 4 * 2 * 64 + 8 * 32 * 3}
    # keeping the two-replica modes adds 16 wavefronts' plane counters (3 L
    # words each) and the item's mode sums (N_T x (L/2 + 1) 64-bit)
    m = pt.pt_plan_query(3, 16, 32, measure=True, modes=True)
    assert m == {"mode": 0, "parts": 1, "per_part": 64,
                 "lds_bytes": 40056 + 4 * 16 * 3 * 16 + 8 * 32 * 9}
    # a split sample keeping the modes needs more parts for the counters and sums
    sm = pt.pt_plan_query(3, 48, 48, measure=True, modes=True)
    assert sm["mode"] == 3 and sm["parts"] >= 12 and sm["lds_bytes"] <= 160 * 1024
    p = pt.pt_plan_query(3, 48, 48, measure=True)
    assert p["mode"] == 3 and p["parts"] == 12 and p["per_part"] == 8
    assert pt.pt_plan_query(2, 64, 24, houdayer=True, measure=True)["mode"] == 1
    assert pt.pt_plan_query(3, 64, 48, houdayer=True)["mode"] == -1


def test_plan_query_rejects_bad_shapes(lib):
    for args in [(4, 16, 8), (3, 15, 8), (3, 2, 8), (3, 66, 8), (3, 16, 1)]:
        with pytest.raises(pt.PTError):
            pt.pt_plan_query(*args)


def test_job_bytes(lib):
    b = 1.0 / np.linspace(0.9, 2.0, 32)
    one = pt.pt_job_bytes(1, 32, 16, 3, b)
    many = pt.pt_job_bytes(1000, 32, 16, 3, b)
    # the spins alone: 1000 x 64 lattices x 4096 int8 sites
    assert many >= 1000 * 64 * 4096 and many <= 1000 * one
    packed = pt.pt_job_bytes(1000, 32, 16, 3, b, layout=pt.PT_LAYOUT_PACKED)
    assert packed < many
    # the replica walk: two words per slot and 32 x 3 64-bit sums per sample
    assert pt.pt_job_bytes(1000, 32, 16, 3, b, walk=True) == many + 1000 * (64 * 8 + 768)
    assert pt.pt_job_bytes(1000, 32, 16, 3, b, modes=True) == many + 1000 * 32 * 9 * 8
    # a split plan brings its scratch: published energies and configurations
    b48 = 1.0 / np.linspace(0.9, 2.0, 48)
    assert pt.pt_job_bytes(1, 48, 48, 3, b48) > 96 * 48 ** 3 + 2 * 96 * 2 * 2304 * 4
    with pytest.raises(pt.PTError):
        pt.pt_job_bytes(1, 32, 16, 3, b[::-1])      # betas must decrease
    with pytest.raises(pt.PTError):
        pt.pt_job_bytes(0, 32, 16, 3, b)
