"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/pt.h declares, and rejects invalid arguments with
PT_EINVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(pt_\w+)\(", src, re.M)))


def test_header_and_binding_agree():
    from paper_2003_04621_amd import pt
    assert _declared() == sorted(pt.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2003_04621_amd import pt
    L = pt.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert pt.pt_version().startswith("ptsg")


def _init(**kw):
    from paper_2003_04621_amd import pt
    a = dict(S=2, NT=3, L=4, d=2, seed=1, flags=0)
    a.update(kw)
    N = a["L"] ** a["d"]
    J = kw.get("J", np.ones(a["S"] * a["d"] * N, np.int8))
    b = kw.get("betas", np.array([1.0, 0.5, 0.25])[: a["NT"]] if a["NT"] <= 3
               else np.linspace(2.0, 0.1, a["NT"]))
    J = np.ascontiguousarray(J, np.int8)
    b = np.ascontiguousarray(b, np.float64)
    h = C.c_void_p()
    rc = pt.lib().pt_init_ex(C.byref(h), a["S"], a["NT"], a["L"], a["d"],
                             J.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                             C.c_uint64(a["seed"]), a["flags"])
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(d=1), dict(d=4), dict(L=5), dict(L=2), dict(L=66), dict(S=0), dict(NT=1),
    dict(flags=7), dict(betas=np.array([1.0, 1.0, 0.5])), dict(betas=np.array([0.5, 1.0, 0.25])),
    dict(betas=np.array([1.0, 0.5, 0.0])), dict(betas=np.array([1.0, 0.5, np.nan])),
    dict(J=np.full(2 * 2 * 16, 2, np.int8)), dict(J=np.zeros(2 * 2 * 16, np.int8)),
])
def test_invalid_init_arguments_are_rejected(kw):
    from paper_2003_04621_amd import pt
    rc, h = _init(**kw)
    assert rc == pt.PT_EINVAL
    assert not h.value
    assert pt.pt_last_error() != ""


def test_null_handles_are_rejected():
    from paper_2003_04621_amd import pt
    L = pt.lib()
    assert L.pt_sweep(None, 1) == pt.PT_EINVAL
    assert L.pt_exchange(None) == pt.PT_EINVAL
    assert L.pt_observables(None, None, None, None) == pt.PT_EINVAL
    assert L.pt_destroy(None) == pt.PT_EINVAL
    h = C.c_void_p()
    assert L.pt_init(C.byref(h), 1, 2, 4, 2, None, None, 0) == pt.PT_EINVAL
    assert L.pt_set_measure_interval(None, 3) == pt.PT_EINVAL
    assert L.pt_get_walk(None, None, None, None) == pt.PT_EINVAL
    assert L.pt_get_modes(None, None) == pt.PT_EINVAL
    assert L.pt_correlation_length(None, None, None, None) == pt.PT_EINVAL
    assert L.pt_tunnel_summary(None, 1, 10, None, None, None, None) == pt.PT_EINVAL


def test_init_flags_and_queries_validated_on_host():
    """Unknown pt_init_ex flags are refused before any device call; the walk
    and mode flags are accepted by the host-only plan and byte queries."""
    from paper_2003_04621_amd import pt
    L = pt.lib()
    J = np.ones(2 * 16, np.int8)
    b = np.array([1.0, 0.5])
    h = C.c_void_p()
    for bad in (2, 0x40, 0x100):
        assert L.pt_init_ex(C.byref(h), 1, 2, 4, 2, pt._p(J), pt._p(b), 0, bad) == pt.PT_EINVAL
    out = np.zeros(4, np.int32)
    for flags in (pt.PT_TRACK_WALK, pt.PT_TRACK_MODES, pt.PT_TRACK_WALK | pt.PT_TRACK_MODES):
        assert L.pt_plan_query(3, 16, 8, flags | pt.PT_MCS_MEASURE, pt._p(out)) == pt.PT_OK
    assert L.pt_plan_query(3, 16, 8, 0x80, pt._p(out)) == pt.PT_EINVAL
    # the multi-cluster modifier only with Houdayer moves
    assert L.pt_plan_query(3, 16, 8, pt.PT_MCS_MULTICLUSTER, pt._p(out)) == pt.PT_EINVAL
    assert L.pt_plan_query(3, 16, 8, pt.PT_MCS_MULTICLUSTER | pt.PT_MCS_HOUDAYER,
                           pt._p(out)) == pt.PT_OK
    assert out[0] == 1
    # multi-cluster labels name at most 32768 sites: no fused plan beyond
    assert L.pt_plan_query(3, 34, 2, pt.PT_MCS_MULTICLUSTER | pt.PT_MCS_HOUDAYER,
                           pt._p(out)) == pt.PT_OK
    assert out[0] == -1


def test_allocator_hooks_must_be_paired():
    from paper_2003_04621_amd import pt
    L = pt.lib()
    assert L.pt_set_allocator(pt._ALLOC(lambda n, c: None), pt._FREE(), None) == pt.PT_EINVAL
    assert L.pt_set_allocator(pt._ALLOC(), pt._FREE(), None) == pt.PT_OK
