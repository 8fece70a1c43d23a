"""Python binding of the C ABI in include/pt.h (argument marshalling only).

Every function has the name of its C entry point and forwards to it through
ctypes; all simulation work runs in the gfx950 kernels of ``libptsg.so``.
PyTorch supplies device memory (its caching allocator, through
``pt_set_allocator``) and the stream (its current stream, through
``pt_set_stream``).  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptsg.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_ESTATE, PT_ECANCELED = 0, -1, -2, -3, -4, -5
PT_LAYOUT_INT8, PT_LAYOUT_PACKED = 0, 1
PT_TRACK_WALK = 0x10
PT_TRACK_MODES = 0x20
PT_TRACK_STATS = 0x80
PT_MCS_HOUDAYER, PT_MCS_MEASURE, PT_MCS_PLAIN, PT_BATCH_GRAPH = 1, 2, 4, 8
PT_MCS_MULTICLUSTER = 0x40
PT_SERVE_UNTIL_EQUILIBRATED = 0x100
PT_TUNE_LAYOUT = 0x200
PT_NOALLOC_MAX_ITEMS = 65536
_CODES = {PT_EINVAL: "PT_EINVAL", PT_ENOMEM: "PT_ENOMEM", PT_EDEVICE: "PT_EDEVICE",
          PT_ESTATE: "PT_ESTATE", PT_ECANCELED: "PT_ECANCELED"}

EXPORTS = [
    "pt_init", "pt_init_ex", "pt_sweep", "pt_exchange", "pt_houdayer", "pt_houdayer_multi",
    "pt_measure", "pt_mcs", "pt_mcs_noalloc",
    "pt_get_plan", "pt_plan_query", "pt_job_bytes", "pt_observables", "pt_destroy", "pt_get_spins", "pt_set_spins",
    "pt_set_layout", "pt_get_layout", "pt_get_energies",
    "pt_get_maps", "pt_get_counters", "pt_get_moments", "pt_get_walk", "pt_tunnel_summary",
    "pt_get_modes", "pt_correlation_length", "pt_get_stats",
    "pt_get_state", "pt_set_state",
    "pt_set_measure_interval", "pt_set_stream", "pt_set_allocator", "pt_last_error", "pt_version",
    "pt_batch_create", "pt_batch_set_stream", "pt_batch_run", "pt_batch_tune",
    "pt_batch_get_config", "pt_batch_set_config", "pt_batch_launch_shape", "pt_batch_destroy",
    "pt_server_start", "pt_server_submit", "pt_server_poll", "pt_server_poll_ex", "pt_server_stats",
    "pt_server_stop", "pt_server_cancel",
    "pt_init_gauss", "pt_get_energies64", "pt_get_moments8", "pt_gauss_accept_test",
    "pt_gauss_accept_host",
]


class PTRequest(C.Structure):
    _fields_ = [("dim", C.c_int32), ("L", C.c_int32), ("replicas", C.c_int32),
                ("samples", C.c_int32), ("betas", C.c_void_p), ("couplings", C.c_void_p),
                ("seed", C.c_uint64), ("sweeps", C.c_int32), ("burn_in", C.c_int32),
                ("flags", C.c_uint32), ("layout", C.c_uint32), ("measure_every", C.c_int32),
                ("reserved", C.c_int32)]


class PTResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("equilibrated", C.c_int32), ("n_meas", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("tau_tunnel", C.c_double)]


class PTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_hooks = None


def lib():
    """Loads libptsg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_2003_04621_amd.build.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P, I32, U32, U64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
        sig = {
            "pt_init": [C.POINTER(P), I32, I32, I32, I32, P, P, U64],
            "pt_init_ex": [C.POINTER(P), I32, I32, I32, I32, P, P, U64, U32],
            "pt_sweep": [P, I32], "pt_exchange": [P], "pt_houdayer": [P], "pt_houdayer_multi": [P],
            "pt_measure": [P],
            "pt_mcs": [P, I32, U32], "pt_mcs_noalloc": [P, I32, U32], "pt_get_plan": [P, U32, P], "pt_plan_query": [I32, I32, I32, U32, P],
            "pt_job_bytes": [I32, I32, I32, I32, U32, P, P], "pt_observables": [P, P, P, P], "pt_destroy": [P],
            "pt_get_spins": [P, P], "pt_set_spins": [P, P], "pt_get_energies": [P, P],
            "pt_set_layout": [P, U32], "pt_get_layout": [P, P],
            "pt_get_maps": [P, P, P], "pt_get_counters": [P, P], "pt_get_moments": [P, P],
            "pt_get_walk": [P, P, P, P], "pt_tunnel_summary": [P, I32, U64, P, P, P, P],
            "pt_get_modes": [P, P], "pt_correlation_length": [P, P, P, P], "pt_get_stats": [P, P],
            "pt_get_state": [P, P, C.POINTER(C.c_size_t)], "pt_set_state": [P, P, C.c_size_t],
            "pt_set_stream": [P, P], "pt_set_allocator": [_ALLOC, _FREE, P],
            "pt_set_measure_interval": [P, I32],
            "pt_batch_create": [P, I32, C.POINTER(P)], "pt_batch_set_stream": [P, P],
            "pt_batch_run": [P, I32, U32], "pt_batch_tune": [P, I32, U32, C.c_char_p],
            "pt_batch_get_config": [P, P], "pt_batch_set_config": [P, I32, I32, I32],
            "pt_batch_launch_shape": [P, P],
            "pt_batch_destroy": [P],
            "pt_server_start": [C.c_size_t, I32, C.POINTER(P)],
            "pt_server_submit": [P, C.POINTER(PTRequest), C.POINTER(C.c_uint64)],
            "pt_server_poll": [P, C.c_uint64, C.POINTER(PTResult), P],
            "pt_server_poll_ex": [P, C.c_uint64, C.POINTER(PTResult), P, P],
            "pt_server_stats": [P, P], "pt_server_stop": [P], "pt_server_cancel": [P, C.c_uint64],
            "pt_init_gauss": [C.POINTER(P), I32, I32, I32, I32, P, P, U64, U32],
            "pt_get_energies64": [P, P], "pt_get_moments8": [P, P],
            "pt_gauss_accept_test": [P, P, P, P, I32, I32],
            "pt_gauss_accept_host": [U32, C.c_double, C.c_int64],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.pt_last_error.argtypes = []
        L.pt_last_error.restype = C.c_char_p
        L.pt_version.argtypes = []
        L.pt_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PT_OK:
        raise PTError(rc, lib().pt_last_error().decode())


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def pt_last_error() -> str:
    return lib().pt_last_error().decode()


def pt_version() -> str:
    return lib().pt_version().decode()


def use_torch_memory() -> None:
    """Routes the library's device allocations through torch's caching
    allocator (on torch's current stream)."""
    global _hooks
    import torch

    def _alloc(size, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(size))
        except Exception:
            return None

    def _free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    hooks = (_ALLOC(_alloc), _FREE(_free))
    _check(lib().pt_set_allocator(hooks[0], hooks[1], None))
    _hooks = hooks


def pt_set_allocator(alloc=None, free=None):
    """pt_set_allocator(None, None) restores hipMalloc/hipFree."""
    global _hooks
    if alloc is None and free is None:
        _check(lib().pt_set_allocator(_ALLOC(), _FREE(), None))
        _hooks = None
        return
    hooks = (_ALLOC(alloc), _FREE(free))
    _check(lib().pt_set_allocator(hooks[0], hooks[1], None))
    _hooks = hooks


_live_jobs = weakref.WeakSet()


@atexit.register
def _destroy_live_jobs():
    # runs before torch's own exit handlers (registered earlier), so the
    # device memory goes back to the caching allocator while it still exists
    for job in list(_live_jobs):
        try:
            pt_destroy(job)
        except Exception:
            pass


class Job:
    """Owning handle of a pt_job plus its shape."""

    def __init__(self, handle, samples, replicas, L, dim, layout, walk=False, modes=False):
        self.h = handle
        self.S, self.NT, self.L, self.d, self.layout = samples, replicas, L, dim, layout
        self.walk, self.modes = bool(walk), bool(modes)
        self.gauss = False
        self.N = L ** dim
        _live_jobs.add(self)

    def __del__(self):
        try:
            if self.h:
                lib().pt_destroy(self.h)
                self.h = None
        except Exception:
            pass


def pt_init(samples, replicas, L, dim, couplings, betas, seed, layout=PT_LAYOUT_INT8,
            stream=None, walk=False, modes=False, stats=False) -> Job:
    """Creates a job; `stream` is a torch.cuda.Stream, a raw hipStream_t int,
    or None for torch's current stream (torch memory hooks are installed);
    `walk` keeps the replica walk and its round trips (PT_TRACK_WALK), `modes`
    the two-replica modes (PT_TRACK_MODES), `stats` the run diagnostics
    (PT_TRACK_STATS)."""
    import torch
    if _hooks is None:
        use_torch_memory()
    J = np.ascontiguousarray(couplings, dtype=np.int8)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.shape != (int(replicas),):
        raise PTError(PT_EINVAL, "betas must have shape (replicas,)")
    if J.size != int(samples) * int(dim) * int(L) ** int(dim):
        raise PTError(PT_EINVAL, "couplings must have samples*dim*L^dim entries")
    h = C.c_void_p()
    _check(lib().pt_init_ex(C.byref(h), int(samples), int(replicas), int(L), int(dim), _p(J),
                            _p(b), C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF),
                            int(layout) | (PT_TRACK_WALK if walk else 0)
                            | (PT_TRACK_MODES if modes else 0) | (PT_TRACK_STATS if stats else 0)))
    job = Job(h, int(samples), int(replicas), int(L), int(dim), int(layout), walk, modes)
    if stream is None:
        stream = torch.cuda.current_stream()
    pt_set_stream(job, stream)
    return job


def pt_init_gauss(samples, replicas, L, dim, couplings, betas, seed, layout=PT_LAYOUT_INT8,
                  stream=None) -> Job:
    """Creates a job with Gaussian couplings: float32 [samples][dim][L^dim] on
    the 2^-16 grid, |J| <= 8 (workloads.couplings_gauss); `stream` as
    pt_init's."""
    import torch
    if _hooks is None:
        use_torch_memory()
    J = np.ascontiguousarray(couplings, dtype=np.float32)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.shape != (int(replicas),):
        raise PTError(PT_EINVAL, "betas must have shape (replicas,)")
    if J.size != int(samples) * int(dim) * int(L) ** int(dim):
        raise PTError(PT_EINVAL, "couplings must have samples*dim*L^dim entries")
    h = C.c_void_p()
    _check(lib().pt_init_gauss(C.byref(h), int(samples), int(replicas), int(L), int(dim), _p(J),
                               _p(b), C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(layout)))
    job = Job(h, int(samples), int(replicas), int(L), int(dim), int(layout))
    job.gauss = True
    if stream is None:
        stream = torch.cuda.current_stream()
    pt_set_stream(job, stream)
    return job


def pt_get_energies64(job: Job) -> np.ndarray:
    """int64 [S][2NT]: 2^-16 units for Gaussian jobs."""
    out = np.zeros((job.S, 2 * job.NT), np.int64)
    _check(lib().pt_get_energies64(job.h, _p(out)))
    return out


def pt_get_moments8(job: Job) -> np.ndarray:
    """int64 [S][NT][8]: E, E^2 lo, Q, |Q|, Q^2, Q^4 lo, Q^4 hi, E^2 hi."""
    out = np.zeros((job.S, job.NT, 8), np.int64)
    _check(lib().pt_get_moments8(job.h, _p(out)))
    return out


def pt_gauss_accept_test(r, b, u, mode: int) -> np.ndarray:
    """Device acceptance decisions r < 2^32 exp(-b u 2^-16) (mode 0 Metropolis
    tiers, 1 exchange tiers, 2 double-double alone)."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.int64)
    if not (r.shape == b.shape == u.shape) or r.ndim != 1:
        raise PTError(PT_EINVAL, "r, b, u must be 1-D arrays of one length")
    out = np.zeros(r.shape, np.int32)
    _check(lib().pt_gauss_accept_test(_p(r), _p(b), _p(u), _p(out), int(r.size), int(mode)))
    return out


def pt_gauss_accept_host(r: int, b: float, u: int) -> int:
    """The double-double decision on the host (1 accept, 0 reject)."""
    rc = lib().pt_gauss_accept_host(int(r) & 0xFFFFFFFF, float(b), int(u))
    if rc < 0:
        _check(rc)
    return rc


def pt_set_measure_interval(job: Job, every: int) -> None:
    """Measured steps of pt_mcs / batches: 1-based sweep number a multiple of `every`."""
    _check(lib().pt_set_measure_interval(job.h, int(every)))


def pt_set_stream(job: Job, stream) -> None:
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
    _check(lib().pt_set_stream(job.h, C.c_void_p(raw)))


def pt_sweep(job: Job, n: int = 1) -> None:
    _check(lib().pt_sweep(job.h, int(n)))


def pt_exchange(job: Job) -> None:
    _check(lib().pt_exchange(job.h))


def pt_houdayer(job: Job) -> None:
    _check(lib().pt_houdayer(job.h))


def pt_houdayer_multi(job: Job) -> None:
    _check(lib().pt_houdayer_multi(job.h))


def pt_measure(job: Job) -> None:
    _check(lib().pt_measure(job.h))


def _step_flags(houdayer=False, measure=False, plain=False, multi=False):
    """pt_mcs flags; multi=True makes the Houdayer moves the multi-cluster
    variant (needs houdayer=True)."""
    return ((PT_MCS_HOUDAYER if houdayer else 0) | (PT_MCS_MEASURE if measure else 0)
            | (PT_MCS_PLAIN if plain else 0) | (PT_MCS_MULTICLUSTER if multi else 0))


def pt_mcs(job: Job, n: int, houdayer: bool = False, measure: bool = False,
           plain: bool = False, multi: bool = False) -> None:
    _check(lib().pt_mcs(job.h, int(n), _step_flags(houdayer, measure, plain, multi)))


def pt_mcs_noalloc(job: Job, n: int, houdayer: bool = False, measure: bool = False,
                   plain: bool = False, multi: bool = False) -> None:
    _check(lib().pt_mcs_noalloc(job.h, int(n), _step_flags(houdayer, measure, plain, multi)))


def pt_get_plan(job: Job, houdayer=False, measure=False, plain=False, multi=False) -> dict:
    """The fused plan pt_mcs takes for these flags: mode (0 both sets per
    workgroup, 1 with Houdayer room, 2 one set per workgroup, 3 split sample,
    -1 per-step kernels), workgroups per sample, configurations per
    workgroup, LDS bytes per workgroup."""
    flags = _step_flags(houdayer, measure, plain, multi)
    out = np.zeros(4, np.int32)
    _check(lib().pt_get_plan(job.h, flags, _p(out)))
    return dict(mode=int(out[0]), parts=int(out[1]), per_part=int(out[2]), lds_bytes=int(out[3]))


def pt_plan_query(dim: int, L: int, replicas: int, houdayer=False, measure=False,
                  plain=False, walk=False, modes=False, multi=False) -> dict:
    """pt_get_plan's report for a job of this shape, without creating it
    (host only)."""
    flags = (_step_flags(houdayer, measure, plain, multi) | (PT_TRACK_WALK if walk else 0)
             | (PT_TRACK_MODES if modes else 0))
    out = np.zeros(4, np.int32)
    _check(lib().pt_plan_query(int(dim), int(L), int(replicas), flags, _p(out)))
    return dict(mode=int(out[0]), parts=int(out[1]), per_part=int(out[2]), lds_bytes=int(out[3]))


def pt_job_bytes(samples: int, replicas: int, L: int, dim: int, betas, layout: int = PT_LAYOUT_INT8,
                 walk: bool = False, modes: bool = False) -> int:
    """Upper bound of the device bytes of a job of this shape (host only)."""
    layout = int(layout) | (PT_TRACK_WALK if walk else 0) | (PT_TRACK_MODES if modes else 0)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.size != replicas:
        raise PTError(PT_EINVAL, "betas must have `replicas` entries")
    out = np.zeros(1, np.uint64)
    _check(lib().pt_job_bytes(int(samples), int(replicas), int(L), int(dim), int(layout), _p(b), _p(out)))
    return int(out[0])


def pt_observables(job: Job):
    ps = np.zeros((job.S, job.NT, 5), np.float64)
    dis = np.zeros((job.NT, 6), np.float64)
    n = np.zeros(1, np.int64)
    _check(lib().pt_observables(job.h, _p(ps), _p(dis), _p(n)))
    return ps, dis, int(n[0])


def pt_destroy(job: Job) -> None:
    if job.h:
        _check(lib().pt_destroy(job.h))
        job.h = None


def pt_get_spins(job: Job) -> np.ndarray:
    out = np.zeros((job.S, 2 * job.NT, job.N), np.int8)
    _check(lib().pt_get_spins(job.h, _p(out)))
    return out


def pt_set_spins(job: Job, spins) -> None:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    if s.size != job.S * 2 * job.NT * job.N:
        raise PTError(PT_EINVAL, "spins must have samples*2*replicas*L^dim entries")
    _check(lib().pt_set_spins(job.h, _p(s)))


def pt_set_layout(job: Job, layout: int) -> None:
    _check(lib().pt_set_layout(job.h, int(layout)))
    job.layout = int(layout)


def pt_get_layout(job: Job) -> int:
    out = np.zeros(1, np.uint32)
    _check(lib().pt_get_layout(job.h, _p(out)))
    job.layout = int(out[0])
    return job.layout


def pt_get_energies(job: Job) -> np.ndarray:
    out = np.zeros((job.S, 2 * job.NT), np.int32)
    _check(lib().pt_get_energies(job.h, _p(out)))
    return out


def pt_get_maps(job: Job):
    sot = np.zeros((job.S, 2, job.NT), np.int32)
    tos = np.zeros((job.S, 2, job.NT), np.int32)
    _check(lib().pt_get_maps(job.h, _p(sot), _p(tos)))
    return sot, tos


def pt_get_counters(job: Job) -> dict:
    out = np.zeros(4, np.uint64)
    _check(lib().pt_get_counters(job.h, _p(out)))
    return dict(t=int(out[0]), u=int(out[1]), v=int(out[2]), n_meas=int(out[3]))


def pt_get_moments(job: Job) -> dict:
    out = np.zeros((job.S, job.NT, 7), np.int64)
    _check(lib().pt_get_moments(job.h, _p(out)))
    names = ["E", "E2", "Q", "AQ", "Q2"]
    d = {n: out[:, :, i].copy() for i, n in enumerate(names)}
    d["Q4"] = out[:, :, 5:7].view(np.uint64).copy()
    return d


def pt_get_walk(job: Job):
    """(label [S][2NT] int32, begin [S][2NT] uint32, trips [S][32][3] uint64)."""
    lab = np.zeros((job.S, 2 * job.NT), np.int32)
    beg = np.zeros((job.S, 2 * job.NT), np.uint32)
    trips = np.zeros((job.S, 32, 3), np.uint64)
    _check(lib().pt_get_walk(job.h, _p(lab), _p(beg), _p(trips)))
    return lab, beg, trips


def pt_get_stats(job: Job) -> np.ndarray:
    """Run diagnostics [S][NT][24] (int64) of a job created with stats=True:
    accepted Metropolis flips at temperature k, accepted exchanges of
    (k, k+1), Houdayer passes that exchanged sites, the sites exchanged, and
    their histogram by floor(log2) (20 bins)."""
    out = np.zeros((job.S, job.NT, 24), np.int64)
    _check(lib().pt_get_stats(job.h, _p(out)))
    return out


def pt_get_modes(job: Job) -> np.ndarray:
    """Accumulated two-replica modes A(delta), [S][NT][L/2+1] int64."""
    out = np.zeros((job.S, job.NT, job.L // 2 + 1), np.int64)
    _check(lib().pt_get_modes(job.h, _p(out)))
    return out


def pt_correlation_length(job: Job):
    """(chi_SG(0), chi_SG(k_min), xi) per temperature, disorder-averaged."""
    c0 = np.zeros(job.NT, np.float64)
    ck = np.zeros(job.NT, np.float64)
    xi = np.zeros(job.NT, np.float64)
    _check(lib().pt_correlation_length(job.h, _p(c0), _p(ck), _p(xi)))
    return c0, ck, xi


def pt_tunnel_summary(trips, passes: int):
    """(tau_b [32], err_b [32], tau, equilibrated) from round-trip bins
    [..., 32, 3], every leading index pooled."""
    t = np.ascontiguousarray(trips, dtype=np.uint64).reshape(-1, 32, 3)
    tau_b = np.zeros(32, np.float64)
    err_b = np.zeros(32, np.float64)
    tau = np.zeros(1, np.float64)
    eq = np.zeros(1, np.int32)
    _check(lib().pt_tunnel_summary(_p(t), t.shape[0], int(passes), _p(tau_b), _p(err_b),
                                   _p(tau), _p(eq)))
    return tau_b, err_b, float(tau[0]), int(eq[0])


def pt_get_state(job: Job) -> bytes:
    n = C.c_size_t(0)
    _check(lib().pt_get_state(job.h, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().pt_get_state(job.h, C.cast(buf, C.c_void_p), C.byref(n)))
    return buf.raw[: n.value]


def pt_set_state(job: Job, state: bytes) -> None:
    buf = C.create_string_buffer(state, len(state))
    _check(lib().pt_set_state(job.h, C.cast(buf, C.c_void_p), len(state)))


# --------------------------------------------------------------------------
# batched form
# --------------------------------------------------------------------------
class Batch:
    """Owning handle of a pt_batch; keeps its jobs alive."""

    def __init__(self, handle, jobs):
        self.h = handle
        self.jobs = list(jobs)

    def __del__(self):
        try:
            if self.h:
                lib().pt_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass


def pt_batch_create(jobs, stream=None) -> Batch:
    arr = (C.c_void_p * len(jobs))(*[j.h for j in jobs])
    h = C.c_void_p()
    _check(lib().pt_batch_create(arr, len(jobs), C.byref(h)))
    b = Batch(h, jobs)
    if stream is not None:
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        _check(lib().pt_batch_set_stream(b.h, C.c_void_p(raw)))
    return b


def _flags(houdayer, measure, graph=False, multi=False):
    return ((PT_MCS_HOUDAYER if houdayer else 0) | (PT_MCS_MEASURE if measure else 0)
            | (PT_BATCH_GRAPH if graph else 0) | (PT_MCS_MULTICLUSTER if multi else 0))


def pt_batch_run(batch: Batch, mcs: int, houdayer=False, measure=False, graph=False,
                 multi=False) -> None:
    _check(lib().pt_batch_run(batch.h, int(mcs), _flags(houdayer, measure, graph, multi)))


def pt_batch_tune(batch: Batch, trial_mcs: int = 3, houdayer=False, measure=False,
                  cache_path: str | None = None, layouts=False) -> tuple:
    path = cache_path.encode() if cache_path else None
    flags = _flags(houdayer, measure) | (PT_TUNE_LAYOUT if layouts else 0)
    rc = lib().pt_batch_tune(batch.h, int(trial_mcs), flags, path)
    msg = lib().pt_last_error().decode() if rc != PT_OK else ""
    for j in batch.jobs:  # the layout axis may have moved the jobs
        out = np.zeros(1, np.uint32)
        if lib().pt_get_layout(j.h, _p(out)) == PT_OK:
            j.layout = int(out[0])
    if rc != PT_OK:
        raise PTError(rc, msg)
    return pt_batch_get_config(batch)


def pt_batch_get_config(batch: Batch) -> tuple:
    out = np.zeros(3, np.int32)
    _check(lib().pt_batch_get_config(batch.h, _p(out)))
    return tuple(int(v) for v in out)


def pt_batch_launch_shape(batch: Batch) -> dict:
    """The grid of the batch's last launch: workgroups, threads per workgroup
    and workgroups resident per CU."""
    out = np.zeros(3, np.int32)
    _check(lib().pt_batch_launch_shape(batch.h, _p(out)))
    return {"blocks": int(out[0]), "threads": int(out[1]), "per_cu": int(out[2])}


def pt_batch_set_config(batch: Batch, threads: int, sets: int, order: int) -> None:
    _check(lib().pt_batch_set_config(batch.h, int(threads), int(sets), int(order)))


def pt_batch_destroy(batch: Batch) -> None:
    if batch.h:
        _check(lib().pt_batch_destroy(batch.h))
        batch.h = None


# --------------------------------------------------------------------------
# served form
# --------------------------------------------------------------------------
class Server:
    def __init__(self, handle):
        self.h = handle
        self.replicas = {}

    def __del__(self):
        try:
            if self.h:
                lib().pt_server_stop(self.h)
                self.h = None
        except Exception:
            pass


def pt_server_start(hbm_budget: int, steps_per_round: int = 100) -> Server:
    h = C.c_void_p()
    _check(lib().pt_server_start(C.c_size_t(int(hbm_budget)), int(steps_per_round), C.byref(h)))
    return Server(h)


def pt_server_submit(server: Server, dim, L, replicas, samples, betas, couplings, seed, sweeps,
                     burn_in, houdayer=False, layout=PT_LAYOUT_INT8, walk=False,
                     until_equilibrated=False, modes=False, measure_every=1,
                     multi=False) -> int:
    b = np.ascontiguousarray(betas, dtype=np.float64)
    J = np.ascontiguousarray(couplings, dtype=np.int8)
    flags = ((PT_MCS_HOUDAYER if houdayer else 0) | (PT_MCS_MULTICLUSTER if multi else 0)
             | (PT_SERVE_UNTIL_EQUILIBRATED if until_equilibrated else 0))
    req = PTRequest(int(dim), int(L), int(replicas), int(samples), b.ctypes.data, J.ctypes.data,
                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(sweeps), int(burn_in), flags,
                    int(layout) | (PT_TRACK_WALK if walk else 0) | (PT_TRACK_MODES if modes else 0),
                    int(measure_every), 0)
    t = C.c_uint64(0)
    _check(lib().pt_server_submit(server.h, C.byref(req), C.byref(t)))
    server.replicas[t.value] = int(replicas)
    return t.value


def pt_server_poll(server: Server, ticket: int):
    """None while pending; else a dict of status, n_meas, times, the
    disorder averages and, for requests keeping the walk, tau_tunnel and
    equilibrated (-1 otherwise)."""
    res = PTResult()
    nt = server.replicas[ticket]
    dis = np.zeros((nt, 6), np.float64)
    corr = np.zeros((nt, 3), np.float64)
    rc = lib().pt_server_poll_ex(server.h, C.c_uint64(ticket), C.byref(res), _p(dis), _p(corr))
    if rc == 1:
        return None
    _check(rc)
    del server.replicas[ticket]
    return dict(status=res.status, n_meas=res.n_meas, t_submit=res.t_submit,
                t_admit=res.t_admit, t_done=res.t_done, disorder=dis,
                tau_tunnel=res.tau_tunnel, equilibrated=res.equilibrated, correlation=corr)


def pt_server_stats(server: Server) -> dict:
    out = np.zeros(11, np.float64)
    _check(lib().pt_server_stats(server.h, _p(out)))
    keys = ["flips", "busy_s", "rounds", "admitted", "completed", "peak_bytes", "peak_jobs",
            "uptime_s", "queued", "running", "cancelled"]
    return dict(zip(keys, out.tolist()))


def pt_server_cancel(server: Server, ticket: int) -> bool:
    """Cancels a queued or running request (its poll result then has status
    PT_ECANCELED); False if it had already finished (its result stands)."""
    rc = lib().pt_server_cancel(server.h, C.c_uint64(ticket))
    if rc == 1:
        return False
    _check(rc)
    return True


def pt_server_stop(server: Server) -> None:
    if server.h:
        _check(lib().pt_server_stop(server.h))
        server.h = None
